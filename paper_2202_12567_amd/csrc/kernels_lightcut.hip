// Global light cut (Sec. 3, step 1; Sec. 6): the cut of the full light tree
// that the lightcut method picks for the whole image, with the visibility
// bounded by 1, the split test run for all nodes of one tree level at once.
//
// Node table (k_lc_leaves, then k_lc_nodes once per height): a leaf is one
// VPL; split node f keeps the light of one child drawn by quantised
// intensity (TAG_LTREE), I_f = I_l + I_r, box = union of the boxes.
//
// Per sample pixel x (k_lc_samples): M_c = kd_c / pi + ks (e + 2) / (2 pi)
// (the material bound) and est(x), the unoccluded sum of the current cut's
// entries, kept in FP64 and updated by every split f -> (a kept, b):
// est += I_b (S(rep_b) - S(rep_a)) (k_lc_update over chunks of splits, then
// k_lc_est in chunk order, so the sums do not depend on scheduling).
//
// Per level (k_lc_test, k_lc_select, k_lc_update, k_lc_est):
//   bound(x, f) = c_ub / max(d_min^2, r_min^2) * sum_c M_c I_f,c
//   d_min = distance from x to f's box, h = max over the box of n . (y - x),
//   c_ub = 0 if h <= 0 else min(1, h / d_min) (1 if d_min = 0);
//   rho(f) = max over the samples of bound / est (b / 0 = inf, 0 / 0 = 0),
//   folded across workgroups by an integer atomicMax on the float bits
//   (rho >= 0, so the bits order as the values).
// Every frontier node that is not a single VPL fails when rho > eps; the
// failing nodes all split unless that would take the cut past its cap, in
// which case the cap - |cut| largest rho split (ties to the lower id, found
// by an MSB-first radix select on (~bits(rho), id)) and the cut is final.
//
// Output (k_lc_mark, k_lc_count, k_lc_scan_blocks, k_lc_emit, k_lc_above): the cut by smallest leaf and
// the tree above it with the cut's nodes as leaves 0 .. n_g - 1 and the
// split nodes after them by increasing tree id.

#include <algorithm>

#include "vplmc_internal.h"
#include "lightcut.h"
#include "shading.h"
#include "tree_nodes.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
constexpr int LT = 256;          // threads of the grid kernels
constexpr int CHUNK = 4 * LT;    // samples per tile of the split test
constexpr int ST = 1024;         // threads of the single-workgroup kernels
constexpr int UPD = LC_UPDATE_CHUNK;
constexpr int OT = 256;               // threads of the ordering kernels
constexpr int OE = LC_ORDER_BLOCK;    // leaves per ordering block

__global__ void k_lc_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_lc_leaves(LightcutView v, vplmc_lights L) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= v.n) return;
    const size_t N = 2 * (size_t)v.n - 1;
    const int j = clamp_index(v.perm[x], L.n);
    v.rep[x] = j;
    const float p[9] = {L.x[j], L.y[j], L.z[j], L.nx[j], L.ny[j], L.nz[j], L.ir[j], L.ig[j], L.ib[j]};
#pragma unroll
    for (int k = 0; k < 9; ++k) v.lights[k * N + x] = p[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v.bbox[k * N + x] = p[k];
        v.bbox[(3 + k) * N + x] = p[k];
    }
}

__global__ void k_lc_nodes(LightcutView v, int32_t lo, int32_t hi, uint64_t seed) {
    const int idx = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= hi) return;
    const size_t N = 2 * (size_t)v.n - 1;
    const int f = v.order[idx], k = f - v.n;
    combine_node(v.rep, v.lights, v.bbox, N, f, v.left[k], v.right[k], seed, TAG_LTREE);
}

__device__ __forceinline__ double entry_sum(const PointData &q, const Light &L, float r_min2) {
    float o0, o1, o2;
    entry_unoccluded(q, L, r_min2, o0, o1, o2);
    return ((double)o0 + (double)o1) + (double)o2;
}

__device__ __forceinline__ float inverse(double e) { return e > 0.0 ? (float)(1.0 / e) : INFINITY; }

// material bounds of the sample pixels and the estimate of the cut {root};
// the level state starts with the root in the cut and in the frontier
__global__ void k_lc_samples(LightcutView v, vplmc_points pts, float r_min2) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = 2 * (size_t)v.n - 1;
    const int root = (int)N - 1;
    if (s == 0) {
        v.ctl[0] = 1;
        v.ctl[1] = 0;
        v.ctl[2] = 1;
        v.ctl[3] = 0;
        v.ctl[4] = 0;
        v.front[0] = root;
        v.rho_f[0] = 0;
        v.state[root] = 1;
    }
    if (s >= v.S) return;
    const PointData q = load_point(pts, v.sample_ids[s]);
    const float spec = q.ks > 0.0f ? q.ks * (q.e + 2.0f) * (0.5f * INV_PI) : 0.0f;
    const size_t S = v.S;
    const float p[9] = {q.x.x, q.x.y, q.x.z, q.n.x, q.n.y, q.n.z,
                        fmaf(q.kd0, INV_PI, spec), fmaf(q.kd1, INV_PI, spec), fmaf(q.kd2, INV_PI, spec)};
#pragma unroll
    for (int k = 0; k < 9; ++k) v.samp[k * S + s] = p[k];
    const double e = entry_sum(q, node_light(v.lights, N, root, false), r_min2);
    v.est[s] = e;
    v.inv_est[s] = inverse(e);
}

// rho of the frontier nodes of the level (parity p): tiles of (node, CHUNK
// samples), one workgroup per tile, grid-stride over the tiles
__global__ __launch_bounds__(LT) void k_lc_test(LightcutView v, int p, float r_min2) {
    __shared__ float red[LT / WAVE];
    const int nf = v.ctl[p];
    const int nchunk = (v.S + CHUNK - 1) / CHUNK;
    const int64_t tiles = (int64_t)nf * nchunk;
    const int32_t *cur = v.front + (size_t)p * v.F;
    uint32_t *rho = v.rho_f + (size_t)p * v.F;
    const size_t N = 2 * (size_t)v.n - 1, S = v.S;
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int i = (int)(tile / nchunk), c = (int)(tile % nchunk);
        const int f = cur[i];
        if (f < v.n) continue;                   // a single VPL: exact, never split
        const float lx = v.bbox[f], ly = v.bbox[N + f], lz = v.bbox[2 * N + f];
        const float hx = v.bbox[3 * N + f], hy = v.bbox[4 * N + f], hz = v.bbox[5 * N + f];
        const float I0 = v.lights[6 * N + f], I1 = v.lights[7 * N + f], I2 = v.lights[8 * N + f];
        float best = 0.0f;
#pragma unroll
        for (int k = 0; k < CHUNK / LT; ++k) {
            const int s = c * CHUNK + k * LT + t;
            if (s < v.S) {
                const float x = v.samp[s], y = v.samp[S + s], z = v.samp[2 * S + s];
                const float nx = v.samp[3 * S + s], ny = v.samp[4 * S + s], nz = v.samp[5 * S + s];
                const float gx = fmaxf(fmaxf(lx - x, x - hx), 0.0f);
                const float gy = fmaxf(fmaxf(ly - y, y - hy), 0.0f);
                const float gz = fmaxf(fmaxf(lz - z, z - hz), 0.0f);
                const float d2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
                const float h = fmaxf(nx * (lx - x), nx * (hx - x)) + fmaxf(ny * (ly - y), ny * (hy - y)) +
                                fmaxf(nz * (lz - z), nz * (hz - z));
                float cub = 0.0f;
                if (h > 0.0f) cub = d2 > 0.0f ? fminf(1.0f, h / sqrtf(d2)) : 1.0f;
                const float m = fmaf(v.samp[6 * S + s], I0, fmaf(v.samp[7 * S + s], I1, v.samp[8 * S + s] * I2));
                const float b = cub / fmaxf(d2, r_min2) * m;
                const float r = b > 0.0f ? b * v.inv_est[s] : 0.0f;
                best = fmaxf(best, r);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) best = fmaxf(best, __shfl_xor(best, o, WAVE));
        if (lane == 0) red[w] = best;
        __syncthreads();
        if (t == 0) {
            float m = red[0];
            for (int k = 1; k < LT / WAVE; ++k) m = fmaxf(m, red[k]);
            atomicMax(&rho[i], __float_as_uint(m));
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(x, o, WAVE);
        if (lane >= o) x += u;
    }
    return x;
}

template <int T>
__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t *sm) {
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, WAVE);
    if (lane == 0) sm[w] = x;
    __syncthreads();
    uint32_t tot = 0;
    for (int k = 0; k < T / WAVE; ++k) tot += sm[k];
    __syncthreads();
    return tot;
}

// exclusive scan over the T threads of the block; the block total in *total
template <int T>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *total, uint32_t *sm) {
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const uint32_t incl = wave_incl_scan(x, lane);
    if (lane == WAVE - 1) sm[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < T / WAVE; ++k) {
        if (k < w) base += sm[k];
        tot += sm[k];
    }
    __syncthreads();
    *total = tot;
    return base + incl - x;
}

// ascending key = descending rho, then ascending id
__device__ __forceinline__ uint64_t cap_key(uint32_t rho_bits, int f) {
    return ((uint64_t)(~rho_bits) << 32) | (uint64_t)(uint32_t)f;
}

// the split decisions of the level (parity p), one workgroup
__global__ __launch_bounds__(ST) void k_lc_select(LightcutView v, int p, double eps, float *rho_out) {
    __shared__ uint32_t sm[ST / WAVE];
    __shared__ uint32_t hist[256];
    __shared__ uint64_t prefix_s;
    __shared__ uint32_t want_s, carry_s;
    const int t = threadIdx.x;
    const int q = p ^ 1;
    const int nf = v.ctl[p];
    if (v.ctl[4] != 0 || nf == 0) {
        if (t == 0) {
            v.ctl[q] = 0;
            v.ctl[3] = 0;
        }
        return;
    }
    const int32_t *cur = v.front + (size_t)p * v.F;
    const uint32_t *rho = v.rho_f + (size_t)p * v.F;
    int32_t *nxt = v.front + (size_t)q * v.F;
    uint32_t *nrho = v.rho_f + (size_t)q * v.F;
    const int n = v.n;
    uint32_t fails = 0;
    for (int i = t; i < nf; i += ST) {
        const int f = cur[i];
        if (f >= n) {
            const float r = __uint_as_float(rho[i]);
            fails += (double)r > eps ? 1u : 0u;
            if (rho_out) rho_out[f] = r;
        }
    }
    const uint32_t F = block_sum<ST>(fails, sm);
    const int n_cut = v.ctl[2];
    int64_t room = (int64_t)v.cap - n_cut;
    if (room < 0) room = 0;
    const bool capped = (int64_t)F > room;
    // the room-th smallest key of the failing nodes (rank room - 1)
    if (t == 0) {
        prefix_s = 0;
        want_s = (uint32_t)(room > 0 ? room - 1 : 0);
    }
    __syncthreads();
    if (capped && room > 0) {
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            if (t < 256) hist[t] = 0;
            __syncthreads();
            const uint64_t pre = prefix_s;
            for (int i = t; i < nf; i += ST) {
                const int f = cur[i];
                if (f < n || !((double)__uint_as_float(rho[i]) > eps)) continue;
                const uint64_t key = cap_key(rho[i], f);
                if (pass == 0 || (key >> (shift + 8)) == (pre >> (shift + 8)))
                    atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (t == 0) {
                uint32_t want = want_s, acc = 0;
                int b = 0;
                for (; b < 255; ++b) {
                    if (acc + hist[b] > want) break;
                    acc += hist[b];
                }
                want_s = want - acc;
                prefix_s = pre | ((uint64_t)b << shift);
            }
            __syncthreads();
        }
    }
    const uint64_t T = prefix_s;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int i0 = 0; i0 < nf; i0 += ST) {
        const int i = i0 + t;
        uint32_t ch = 0;
        int f = 0;
        if (i < nf) {
            f = cur[i];
            if (f >= n && (double)__uint_as_float(rho[i]) > eps)
                ch = !capped ? 1u : (room > 0 && cap_key(rho[i], f) <= T ? 1u : 0u);
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<ST>(ch, &tot, sm);
        const uint32_t j = carry_s + ex;
        if (ch) {
            const int l = v.left[f - n], r = v.right[f - n];
            v.split[j] = f;
            nxt[2 * j] = l;
            nxt[2 * j + 1] = r;
            nrho[2 * j] = 0;
            nrho[2 * j + 1] = 0;
            v.state[f] = 2;
            v.state[l] = 1;
            v.state[r] = 1;
        }
        __syncthreads();
        if (t == 0) carry_s += tot;
        __syncthreads();
    }
    if (t == 0) {
        const int ns = (int)carry_s;
        v.ctl[3] = ns;
        v.ctl[q] = 2 * ns;
        v.ctl[2] = n_cut + ns;
        if (capped) v.ctl[4] = 1;
    }
}

// est(x) changes of the level's splits, one chunk of UPD splits per blockIdx.y.
// Split node f holds the light of its kept child a, so replacing f by a and
// b changes est by A(a) + A(b) - A(f) = I_b (S(rep_b) - S(rep_a)) channel by
// channel, S the lighting at unit intensity: two entries per split.
__global__ __launch_bounds__(LT) void k_lc_update(LightcutView v, vplmc_points pts, float r_min2) {
    __shared__ float lt[15][UPD];    // rep_a position, normal; rep_b position, normal; I_b
    const int ns = v.ctl[3];
    const int c = blockIdx.y;
    const int b0 = c * UPD;
    if (b0 >= ns) return;
    const int cnt = ns - b0 < UPD ? ns - b0 : UPD;
    const size_t N = 2 * (size_t)v.n - 1;
    for (int k = threadIdx.x; k < cnt; k += LT) {
        const int f = v.split[b0 + k];
        const int l = v.left[f - v.n], r = v.right[f - v.n];
        const int a = v.rep[f] == v.rep[l] ? l : r, b = a == l ? r : l;
#pragma unroll
        for (int pl = 0; pl < 6; ++pl) {
            lt[pl][k] = v.lights[pl * N + a];
            lt[6 + pl][k] = v.lights[pl * N + b];
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) lt[12 + ch][k] = v.lights[(6 + ch) * N + b];
    }
    __syncthreads();
    const int s = blockIdx.x * LT + threadIdx.x;
    if (s >= v.S) return;
    const PointData q = load_point(pts, v.sample_ids[s]);
    double acc = 0.0;
    for (int k = 0; k < cnt; ++k) {
        const float i0 = lt[12][k], i1 = lt[13][k], i2 = lt[14][k];
        const Light La{{lt[0][k], lt[1][k], lt[2][k]}, {lt[3][k], lt[4][k], lt[5][k]}, i0, i1, i2};
        const Light Lb{{lt[6][k], lt[7][k], lt[8][k]}, {lt[9][k], lt[10][k], lt[11][k]}, i0, i1, i2};
        acc += entry_sum(q, Lb, r_min2) - entry_sum(q, La, r_min2);
    }
    v.part[(size_t)c * v.S + s] = acc;
}

// est(x) += the chunks' changes in chunk order
__global__ void k_lc_est(LightcutView v) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int ns = v.ctl[3];
    if (s >= v.S || ns == 0) return;
    double e = v.est[s];
    for (int c = 0; c * UPD < ns; ++c) e += v.part[(size_t)c * v.S + s];
    v.est[s] = e;
    v.inv_est[s] = inverse(e);
}

__global__ void k_lc_mark(LightcutView v) {
    const size_t N = 2 * (size_t)v.n - 1;
    const size_t f = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (f < N && v.state[f] == 1) v.leafmark[v.min_leaf[f]] = (int32_t)f;
}

// Output order in three passes over blocks of OE leaves (and split nodes
// n + x for the same x): counts per block, their exclusive scan, then each
// block's own scan.  Cut nodes are numbered by smallest leaf, split nodes
// n_cut + their rank by tree id.
__global__ __launch_bounds__(OT) void k_lc_count(LightcutView v) {
    __shared__ uint32_t sm[OT / WAVE];
    const int b = blockIdx.x, t = threadIdx.x, n = v.n;
    uint32_t cl = 0, cs = 0;
    for (int k = 0; k < OE / OT; ++k) {
        const int x = b * OE + k * OT + t;
        if (x < n && v.leafmark[x] >= 0) ++cl;
        if (x < n - 1 && v.state[n + x] == 2) ++cs;
    }
    const uint32_t tl = block_sum<OT>(cl, sm);
    const uint32_t ts = block_sum<OT>(cs, sm);
    if (t == 0) {
        v.blk[b] = tl;
        v.blk[gridDim.x + b] = ts;
    }
}

__global__ __launch_bounds__(ST) void k_lc_scan_blocks(LightcutView v, int nb, int32_t *n_cut, int32_t *cut_offsets) {
    __shared__ uint32_t sm[ST / WAVE];
    __shared__ uint32_t carry_s;
    const int t = threadIdx.x;
    uint32_t totals[2];
    for (int a = 0; a < 2; ++a) {
        uint32_t *c = v.blk + (size_t)a * nb;
        if (t == 0) carry_s = 0;
        __syncthreads();
        for (int b0 = 0; b0 < nb; b0 += ST) {
            const int b = b0 + t;
            const uint32_t x = b < nb ? c[b] : 0;
            uint32_t tot;
            const uint32_t ex = block_excl_scan<ST>(x, &tot, sm);
            if (b < nb) c[b] = carry_s + ex;
            __syncthreads();
            if (t == 0) carry_s += tot;
            __syncthreads();
        }
        totals[a] = carry_s;
        __syncthreads();
    }
    if (t == 0) {
        *n_cut = (int32_t)totals[0];
        cut_offsets[totals[0]] = v.n;
        v.ctl[5] = (int32_t)totals[0];
    }
}

__global__ __launch_bounds__(OT) void k_lc_emit(LightcutView v, int nb, int32_t *cut_nodes, int32_t *cut_offsets) {
    __shared__ uint32_t sm[OT / WAVE];
    const int b = blockIdx.x, t = threadIdx.x, n = v.n;
    const uint32_t ng = (uint32_t)v.ctl[5];
    uint32_t cl = v.blk[b], cs = v.blk[nb + b];
    for (int k = 0; k < OE / OT; ++k) {
        const int x = b * OE + k * OT + t;
        const int f = x < n ? v.leafmark[x] : -1;
        const bool sp = x < n - 1 && v.state[n + x] == 2;
        uint32_t tl, ts;
        const uint32_t el = block_excl_scan<OT>(f >= 0 ? 1u : 0u, &tl, sm);
        const uint32_t es = block_excl_scan<OT>(sp ? 1u : 0u, &ts, sm);
        if (f >= 0) {
            const uint32_t j = cl + el;
            cut_nodes[j] = f;
            cut_offsets[j] = x;
            v.ren[f] = (int32_t)j;
        }
        if (sp) v.ren[n + x] = (int32_t)(ng + cs + es);
        cl += tl;
        cs += ts;
    }
}

__global__ void k_lc_above(LightcutView v, int32_t *above_left, int32_t *above_right, int32_t *n_cut) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = v.n;
    if (k >= n - 1 || v.state[n + k] != 2) return;
    const int j = v.ren[n + k] - *n_cut;
    if (above_left) above_left[j] = v.ren[v.left[k]];
    if (above_right) above_right[j] = v.ren[v.right[k]];
}

unsigned grid_for(size_t n, int threads) {
    return (unsigned)std::min<size_t>((n + threads - 1) / threads, 1u << 20);
}

}  // namespace

int launch_lightcut(hipStream_t st, const LightcutView &v, const int32_t *level_off, int32_t height_max,
                    int32_t depth, const vplmc_points &pts, const vplmc_lights &vpls, double eps, float r_min,
                    uint64_t seed, int32_t *n_cut, int32_t *cut_nodes, int32_t *cut_offsets, int32_t *above_left,
                    int32_t *above_right, float *rho) {
    const size_t N = 2 * (size_t)v.n - 1;
    const float r_min2 = r_min * r_min;
    hipLaunchKernelGGL(k_lc_fill_u32, dim3(grid_for(N, LT)), dim3(LT), 0, st, v.state, N, 0u);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lc_fill_u32, dim3(grid_for(v.n, LT)), dim3(LT), 0, st, (uint32_t *)v.leafmark, (size_t)v.n,
                       0xffffffffu);
    VPLMC_HIP(hipGetLastError());
    if (rho) {
        hipLaunchKernelGGL(k_lc_fill_u32, dim3(grid_for(N, LT)), dim3(LT), 0, st, (uint32_t *)rho, N,
                           0xbf800000u);   // -1.0f: not tested
        VPLMC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_lc_leaves, dim3(grid_for(v.n, LT)), dim3(LT), 0, st, v, vpls);
    VPLMC_HIP(hipGetLastError());
    for (int h = 1; h <= height_max; ++h) {
        const int lo = level_off[h - 1], hi = level_off[h];
        if (hi > lo) {
            hipLaunchKernelGGL(k_lc_nodes, dim3(grid_for(hi - lo, LT)), dim3(LT), 0, st, v, lo, hi, seed);
            VPLMC_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_lc_samples, dim3(grid_for(std::max(v.S, 1), LT)), dim3(LT), 0, st, v, pts, r_min2);
    VPLMC_HIP(hipGetLastError());
    const unsigned test_grid = 2048;
    const int max_splits = v.cap < v.n ? v.cap : v.n;   // splits per level stay below both
    const unsigned upd_chunks = (unsigned)((max_splits + UPD - 1) / UPD);
    for (int lvl = 0; lvl < depth; ++lvl) {
        const int p = lvl & 1;
        if (v.S > 0) {
            hipLaunchKernelGGL(k_lc_test, dim3(test_grid), dim3(LT), 0, st, v, p, r_min2);
            VPLMC_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_lc_select, dim3(1), dim3(ST), 0, st, v, p, eps, rho);
        VPLMC_HIP(hipGetLastError());
        if (v.S > 0 && lvl + 1 < depth) {
            hipLaunchKernelGGL(k_lc_update, dim3(grid_for(v.S, LT), upd_chunks), dim3(LT), 0, st, v, pts, r_min2);
            VPLMC_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_lc_est, dim3(grid_for(v.S, LT)), dim3(LT), 0, st, v);
            VPLMC_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_lc_mark, dim3(grid_for(N, LT)), dim3(LT), 0, st, v);
    VPLMC_HIP(hipGetLastError());
    const int nb = (v.n + OE - 1) / OE;
    hipLaunchKernelGGL(k_lc_count, dim3(nb), dim3(OT), 0, st, v);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lc_scan_blocks, dim3(1), dim3(ST), 0, st, v, nb, n_cut, cut_offsets);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lc_emit, dim3(nb), dim3(OT), 0, st, v, nb, cut_nodes, cut_offsets);
    VPLMC_HIP(hipGetLastError());
    if (v.n > 1 && (above_left || above_right)) {
        hipLaunchKernelGGL(k_lc_above, dim3(grid_for(v.n - 1, LT)), dim3(LT), 0, st, v, above_left, above_right,
                           n_cut);
        VPLMC_HIP(hipGetLastError());
    }
    return VPLMC_OK;
}

}  // namespace vplmc
