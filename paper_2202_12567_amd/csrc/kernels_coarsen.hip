// Per-slice light coarsening (Sec. 4): the global cut's clusters are the
// leaves of a binary tree (the light tree above the cut); every slice merges
// sibling pairs, least cost first, into a coarser cut of its own, and the
// pixel draws that priced the merges become the first pass of the coarsened
// slice matrix (Sec. 5).
//
// Node table (once per frame, k_node_table): a split node f with children l,
// r keeps the light (position, normal) of one child a, drawn with probability
// Q_a / (Q_l + Q_r), Q = max(1, floor(2^24 t / max(t_l, t_r))), t = R + G + B
// in FP64 of the FP32 intensities; I_f = fp32(fp64(I_l) + fp64(I_r)).
//
// Draw counts (once per frame, k_leaf_draws): leaf x gets
// k_x = floor(K Q_x / sum Q) of the K row draws of each slice (Q quantised
// over all leaves), capped at m' per slice.
//
// Merge errors (per slice, k_coarsen_eps in kernels_eval.hip) fill
// eps(f) = max over the rows drawn below f and the channels of
// I_b |S(., rep_b) - S(., rep_a)|, S the lighting at unit intensity.
//
// Merge decisions (per slice, k_coarsen_merge): cost(f) = eps(f) +
// cost(dropped child), eff(f) = max(cost(f), eff(children)).  Taking pairs by
// least (eff, height, id) until the slice has n_max columns, then while eff
// stays below the bound, never below q columns, merges exactly the first L
// nodes of that order, L = min(n_g - q, max(n_g - n_max, #{eff < bound})):
// eff and height grow from child to parent, so every node's key exceeds its
// descendants' keys and the pair at the head of the order is always
// available.  The L-th key is found by an MSB-first radix select.

#include "vplmc_internal.h"
#include "tree_nodes.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
constexpr int CT = 1024;   // threads of the per-frame and per-slice workgroups

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, WAVE);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan over a CT-thread block; the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *sm) {
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const uint32_t incl = wave_incl_scan(v, lane);
    if (lane == WAVE - 1) sm[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < CT / WAVE; ++k) {
        if (k < w) base += sm[k];
        tot += sm[k];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// Split nodes level by level (children first): kept / dropped child,
// representative, light, intensity, bbox, member count.  Leaves were written
// by the cluster table (planes of stride NC); member counts of leaves come
// from the cut.
__global__ __launch_bounds__(CT) void k_node_table(CoarsenTree tr, const int32_t *__restrict__ cut_offsets,
                                                   uint64_t seed, int32_t *rep, float *lights, float *bbox,
                                                   int32_t *members, int32_t *kept, int32_t *dropped) {
    const int ng = tr.n_leaves, t = threadIdx.x;
    const size_t N = (size_t)(2 * ng - 1);
    for (int x = t; x < ng; x += CT) members[x] = cut_offsets[x + 1] - cut_offsets[x];
    __syncthreads();
    for (int h = 1; h <= tr.height_max; ++h) {
        for (int idx = tr.level_off[h - 1] + t; idx < tr.level_off[h]; idx += CT) {
            const int f = tr.order[idx], k = f - ng;
            const int l = tr.left[k], r = tr.right[k];
            const int a = combine_node(rep, lights, bbox, N, f, l, r, seed, TAG_TREE);
            kept[k] = a;
            dropped[k] = a == l ? r : l;
            members[f] = members[l] + members[r];
        }
        __syncthreads();
    }
}

// k_x = floor(K Q_x / sum Q) over the leaves, and its exclusive prefix
// (kpre[n_g] = the draws per slice before the cap at m').
__global__ __launch_bounds__(CT) void k_leaf_draws(int32_t ng, const float *__restrict__ lights, int64_t K,
                                                   int32_t *quota, int64_t *kpre) {
    __shared__ double dmax[CT / WAVE];
    __shared__ unsigned long long qsum[CT / WAVE];
    __shared__ uint32_t sm[CT / WAVE];
    __shared__ unsigned long long carry_s;
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const size_t N = (size_t)(2 * ng - 1);
    double m = 0.0;
    for (int x = t; x < ng; x += CT) {
        const double tx = total_t(lights[6 * N + x], lights[7 * N + x], lights[8 * N + x]);
        m = tx > m ? tx : m;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double u = __shfl_xor(m, o, WAVE);
        m = u > m ? u : m;
    }
    if (lane == 0) dmax[w] = m;
    __syncthreads();
    double tmax = 0.0;
    for (int k = 0; k < CT / WAVE; ++k) tmax = dmax[k] > tmax ? dmax[k] : tmax;
    unsigned long long qs = 0;
    for (int x = t; x < ng; x += CT)
        qs += quantise(total_t(lights[6 * N + x], lights[7 * N + x], lights[8 * N + x]), tmax);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) qs += __shfl_xor(qs, o, WAVE);
    if (lane == 0) qsum[w] = qs;
    if (t == 0) carry_s = 0;
    __syncthreads();
    unsigned long long Q = 0;
    for (int k = 0; k < CT / WAVE; ++k) Q += qsum[k];
    for (int x0 = 0; x0 < ng; x0 += CT) {
        const int x = x0 + t;
        uint32_t kx = 0;
        if (x < ng) {
            const uint64_t qx = quantise(total_t(lights[6 * N + x], lights[7 * N + x], lights[8 * N + x]), tmax);
            kx = (uint32_t)(((uint64_t)K * qx) / (uint64_t)Q);
            quota[x] = (int32_t)kx;
        }
        // a chunk of CT quotas sums to at most K < 2^31
        uint32_t tot;
        const uint32_t ex = block_excl_scan(kx, &tot, sm);
        const unsigned long long c = carry_s;
        if (x < ng) kpre[x] = (int64_t)(c + ex);
        __syncthreads();
        if (t == 0) carry_s = c + tot;
        __syncthreads();
    }
    if (t == 0) kpre[ng] = (int64_t)carry_s;
}

// merge key of split node f: eff bits, height, id (eff >= 0, so its bits order as the value)
__device__ __forceinline__ uint64_t merge_key(float eff, int height, int f) {
    return ((uint64_t)__float_as_uint(eff) << 32) | ((uint64_t)(uint32_t)height << 16) | (uint64_t)(uint32_t)f;
}

// One workgroup per slice: costs, the merged prefix of the key order, the
// columns (nodes whose parent is not merged, ordered by their smallest leaf)
// and the column of every leaf.  Writes the slice's column count to desc.
__global__ __launch_bounds__(CT) void k_coarsen_merge(SliceDesc *desc, CoarsenTree tr, CoarsenSlices cs,
                                                      double bound, int32_t *columns) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sm[CT / WAVE];
    __shared__ uint32_t cnt_s[CT / WAVE];
    __shared__ uint64_t prefix_s;
    __shared__ uint32_t want_s;
    __shared__ uint32_t carry_s;
    const int s = blockIdx.x, t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const SliceDesc d = desc[s];
    const int ng = tr.n_leaves, ns = ng - 1, NC = 2 * ng - 1;
    const float *eps = cs.eps + (size_t)s * ns;
    float *cost = cs.cost + (size_t)s * ns;
    float *eff = cs.eff + (size_t)s * ns;
    uint8_t *merged = cs.merged + (size_t)s * ns;
    int32_t *top = cs.top + (size_t)s * NC;
    int32_t *lcol = cs.leaf_col + (size_t)s * ng;
    // costs bottom-up, one height at a time (FP32, as the decisions are taken)
    for (int h = 1; h <= tr.height_max; ++h) {
        for (int idx = tr.level_off[h - 1] + t; idx < tr.level_off[h]; idx += CT) {
            const int f = tr.order[idx], k = f - ng;
            const int db = cs.dropped[k], l = tr.left[k], r = tr.right[k];
            const float c = eps[k] + (db >= ng ? cost[db - ng] : 0.0f);
            cost[k] = c;
            const float el = l >= ng ? eff[l - ng] : 0.0f, er = r >= ng ? eff[r - ng] : 0.0f;
            eff[k] = fmaxf(c, fmaxf(el, er));
        }
        __syncthreads();
    }
    // L = min(n_g - q, max(n_g - n_max, #{eff < bound}))
    uint32_t below = 0;
    for (int k = t; k < ns; k += CT) below += (double)eff[k] < bound ? 1u : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) below += __shfl_xor(below, o, WAVE);
    if (lane == 0) cnt_s[w] = below;
    __syncthreads();
    int64_t B = 0;
    for (int k = 0; k < CT / WAVE; ++k) B += cnt_s[k];
    int64_t L = (int64_t)ng - d.nmax;
    if (L < B) L = B;
    if (L > (int64_t)ng - d.qr) L = (int64_t)ng - d.qr;
    if (L < 0) L = 0;
    // the L-th smallest key (rank L - 1), 8 bits at a time from the top
    if (t == 0) {
        prefix_s = 0;
        want_s = (uint32_t)(L > 0 ? L - 1 : 0);
    }
    __syncthreads();
    if (L > 0 && L < ns) {
        for (int p = 0; p < 8; ++p) {
            const int shift = 56 - 8 * p;
            if (t < 256) hist[t] = 0;
            __syncthreads();
            const uint64_t pre = prefix_s;
            for (int k = t; k < ns; k += CT) {
                const uint64_t key = merge_key(eff[k], tr.height[ng + k], ng + k);
                if (p == 0 || (key >> (shift + 8)) == (pre >> (shift + 8)))
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
    for (int k = t; k < ns; k += CT)
        merged[k] = L >= ns ? 1 : (L == 0 ? 0 : (merge_key(eff[k], tr.height[ng + k], ng + k) <= T ? 1 : 0));
    if (t == 0) top[NC - 1] = NC - 1;
    __syncthreads();
    // top-down: a child of a merged node belongs to its parent's column
    for (int h = tr.height_max; h >= 1; --h) {
        for (int idx = tr.level_off[h - 1] + t; idx < tr.level_off[h]; idx += CT) {
            const int f = tr.order[idx], k = f - ng;
            const int tf = top[f];
            const bool mg = merged[k] != 0;
            top[tr.left[k]] = mg ? tf : tr.left[k];
            top[tr.right[k]] = mg ? tf : tr.right[k];
        }
        __syncthreads();
    }
    // columns in order of their smallest leaf: a leaf starts a column iff it
    // is the smallest leaf below its column's node
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int x0 = 0; x0 < ng; x0 += CT) {
        const int x = x0 + t;
        uint32_t st = 0;
        int tx = 0;
        if (x < ng) {
            tx = top[x];
            st = tr.min_leaf[tx] == x ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan(st, &tot, sm);
        const uint32_t c = carry_s;
        if (st) {
            columns[d.cl_off + c + ex] = tx;
            lcol[x] = (int32_t)(c + ex);
        }
        __syncthreads();
        if (t == 0) carry_s = c + tot;
        __syncthreads();
    }
    // every other leaf takes its column's index from the column's first leaf
    for (int x = t; x < ng; x += CT) {
        const int x0 = tr.min_leaf[top[x]];
        if (x0 != x) lcol[x] = lcol[x0];
    }
    if (t == 0) desc[s].n = (int32_t)carry_s;
}

// index of the leaf holding draw r: kpre[x] <= r < kpre[x + 1]
__device__ __forceinline__ int leaf_of_draw(const int64_t *__restrict__ kpre, int ng, int64_t r) {
    int lo = 0, hi = ng;   // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (kpre[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// First pass of the coarsened slices: draw (s, r) of leaf x observes the
// entry (its row, the column of x) in both occupancy bitmaps.
__global__ void k_coarsen_pass1(const SliceDesc *__restrict__ desc, int64_t total, int64_t K, CoarsenSlices cs,
                                int32_t ng, uint32_t *bm, uint32_t *bmt) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int s = (int)(g / K);
    const int64_t r = g - (int64_t)s * K;
    if (r >= cs.kpre[ng]) return;
    const SliceDesc d = desc[s];
    const int x = leaf_of_draw(cs.kpre, ng, r);
    if (r - cs.kpre[x] >= d.m) return;
    const uint32_t i = cs.zeta[g];
    const uint32_t j = (uint32_t)cs.leaf_col[(size_t)s * ng + x];
    atomicOr(bm + d.off_bm + (int64_t)i * d.words_row + (j >> 5), 1u << (j & 31));
    atomicOr(bmt + d.off_bmt + (int64_t)j * d.words_col + (i >> 5), 1u << (i & 31));
}

// per row: number of first-pass entries (into ptr[row + 1])
__global__ void k_rowcount(const SliceDesc *__restrict__ desc, int S, int64_t total_rows,
                           const uint32_t *__restrict__ bm, int32_t *ptr) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total_rows) return;
    int lo = 0, hi = S;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (desc[mid].off_row - mid <= g) lo = mid; else hi = mid;
    }
    const SliceDesc d = desc[lo];
    const int64_t i = g - (d.off_row - lo);
    const uint32_t *row = bm + d.off_bm + i * d.words_row;
    int c = 0;
    for (int w = 0; w < d.words_row; ++w) c += __popc(row[w]);
    ptr[d.off_row + i + 1] = c;
}

// ptr[0] = 0, ptr[k + 1] = ptr[k] + count[k] over the slice's m rows; then the
// slice's first-pass count and second-pass target go to desc
__global__ __launch_bounds__(CT) void k_rowptr(SliceDesc *desc, int32_t *ptr, int32_t pass2_ppm) {
    __shared__ uint32_t sm[CT / WAVE];
    __shared__ uint32_t carry_s;
    const int s = blockIdx.x, t = threadIdx.x;
    const SliceDesc d = desc[s];
    int32_t *p = ptr + d.off_row;
    if (t == 0) {
        p[0] = 0;
        carry_s = 0;
    }
    __syncthreads();
    for (int k0 = 0; k0 < d.m; k0 += CT) {
        const int k = k0 + t;
        const uint32_t v = k < d.m ? (uint32_t)p[k + 1] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot, sm);
        const uint32_t c = carry_s;
        if (k < d.m) p[k + 1] = (int32_t)(c + ex + v);
        __syncthreads();
        if (t == 0) carry_s = c + tot;
        __syncthreads();
    }
    if (t == 0) {
        const int64_t D = (int64_t)d.m * d.n;
        const int64_t N1 = carry_s;
        int64_t N2 = ((int64_t)pass2_ppm * D + 500000) / 1000000;
        if (N2 > D - N1) N2 = D - N1;
        desc[s].N1 = (int32_t)N1;
        desc[s].N2 = (int32_t)N2;
    }
}

// Omega1 of every slice in row-major order (one thread per row)
__global__ void k_rowkeys(const SliceDesc *__restrict__ desc, int S, int64_t total_rows,
                          const uint32_t *__restrict__ bm, const int32_t *__restrict__ ptr, uint32_t *omega1) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total_rows) return;
    int lo = 0, hi = S;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (desc[mid].off_row - mid <= g) lo = mid; else hi = mid;
    }
    const SliceDesc d = desc[lo];
    const int64_t i = g - (d.off_row - lo);
    const uint32_t *row = bm + d.off_bm + i * d.words_row;
    int64_t pos = d.off1 + ptr[d.off_row + i];
    for (int w = 0; w < d.words_row; ++w) {
        uint32_t word = row[w];
        while (word) {
            const int b = __ffs(word) - 1;
            word &= word - 1;
            omega1[pos++] = ((uint32_t)i << 16) | (uint32_t)(32 * w + b);
        }
    }
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

int launch_node_table(hipStream_t st, const CoarsenTree &tr, const int32_t *cut_offsets, uint64_t seed, int32_t *rep,
                      float *lights, float *bbox, int32_t *members, int32_t *kept, int32_t *dropped) {
    hipLaunchKernelGGL(k_node_table, dim3(1), dim3(CT), 0, st, tr, cut_offsets, seed, rep, lights, bbox, members,
                       kept, dropped);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_leaf_draws(hipStream_t st, int32_t ng, const float *lights, int64_t K, int32_t *quota, int64_t *kpre) {
    hipLaunchKernelGGL(k_leaf_draws, dim3(1), dim3(CT), 0, st, ng, lights, K, quota, kpre);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_coarsen_merge(hipStream_t st, const vplmc_plan &plan, SliceDesc *desc, const CoarsenTree &tr,
                         const CoarsenSlices &cs, int32_t *columns) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_coarsen_merge, dim3(plan.n_slices), dim3(CT), 0, st, desc, tr, cs, plan.bound, columns);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_coarsen_pass1(hipStream_t st, const vplmc_plan &plan, SliceDesc *desc, const CoarsenSlices &cs,
                         uint32_t *bm, uint32_t *bmt, int32_t *row_ptr, uint32_t *omega1) {
    const int S = plan.n_slices;
    if (S <= 0) return VPLMC_OK;
    const int64_t draws = (int64_t)S * plan.pixels;
    if (draws > 0) {
        hipLaunchKernelGGL(k_coarsen_pass1, dim3(blocks_for(draws, 256)), dim3(256), 0, st, desc, draws,
                           (int64_t)plan.pixels, cs, plan.n_leaves, bm, bmt);
        VPLMC_HIP(hipGetLastError());
    }
    const int64_t rows = plan.tot_row - S;
    hipLaunchKernelGGL(k_rowcount, dim3(blocks_for(rows, 256)), dim3(256), 0, st, desc, S, rows, bm, row_ptr);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rowptr, dim3(S), dim3(CT), 0, st, desc, row_ptr, plan.pass2_ppm);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rowkeys, dim3(blocks_for(rows, 256)), dim3(256), 0, st, desc, S, rows, bm, row_ptr, omega1);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
