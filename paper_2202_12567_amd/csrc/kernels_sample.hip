// Cluster table of the cut (Sec. 4), the two sampling passes (Sec. 5) and
// the CSR / CSC ordering of every slice's samples.
//
// Sampled entries of slice s are packed as (i << 16) | j (row i < m',
// column j < n').  Each slice keeps two occupancy bitmaps of its m' x n'
// matrix: row-major (words_row = ceil(n'/32) words per row) and
// column-major (words_col = ceil(m'/32) words per column).  They make the
// second pass's "not sampled yet" test a single bit probe and turn the CSR
// and CSC orderings into popcount prefix sums: the position of (i, j) in
// row-major order is the number of set bits before it.

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int slice_of(const SliceDesc *__restrict__ desc, int S, int64_t g, int which) {
    // last slice whose start offset is <= g (which: 0 off1, 1 off2, 2 row base, 3 col base)
    int lo = 0, hi = S;   // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        int64_t o;
        switch (which) {
            case 0: o = desc[mid].off1; break;
            case 1: o = desc[mid].off2; break;
            case 2: o = desc[mid].off_row - mid; break;      // rows before slice mid
            default: o = desc[mid].off_colptr - mid; break;  // columns before slice mid
        }
        if (o <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Keyed balanced Feistel permutation of [0, 2^(2h)): 4 rounds,
// F_r(R) = Philox(key = (seed, s), ctr = (R, r, TAG_PASS1, 0)).a & (2^h - 1).
__device__ __forceinline__ uint64_t feistel(uint64_t x, uint64_t seed, uint64_t s, int h) {
    const uint64_t mask = (1ull << h) - 1ull;
    uint64_t L = x >> h, R = x & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t F = philox(seed, s, R, (uint64_t)r, TAG_PASS1, 0).a & mask;
        const uint64_t nL = R;
        R = L ^ F;
        L = nL;
    }
    return (L << h) | R;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, WAVE);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan over a 256-thread block; returns the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *sm) {
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const uint32_t incl = wave_incl_scan(v, lane);
    if (lane == WAVE - 1) sm[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) {
        if (k < w) base += sm[k];
        tot += sm[k];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// number of ids outside [0, hi)
__global__ void k_count_out_of_range(const int32_t *__restrict__ ids, int64_t n, int32_t hi,
                                     unsigned long long *bad) {
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += (ids[i] < 0 || ids[i] >= hi) ? 1ull : 0ull;
    if (c) atomicAdd(bad, c);
}

// number of offsets that break 0 = offsets[0] <= offsets[1] <= ... <= offsets[n]
__global__ void k_count_unordered(const int32_t *__restrict__ offsets, int64_t n, unsigned long long *bad) {
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        c += (i == 0 ? offsets[0] != 0 : offsets[i] < offsets[i - 1]) ? 1ull : 0ull;
    if (c) atomicAdd(bad, c);
}

__global__ void k_philox(uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t n, uint64_t *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U64x4 r = philox(k0, k1, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    out[4 * i] = r.a;
    out[4 * i + 1] = r.b;
    out[4 * i + 2] = r.c;
    out[4 * i + 3] = r.d;
}

// One thread per cluster: representative drawn with probability ~ quantised
// member intensity, intensity = FP64 member sum, bbox of member positions.
// Planes of `stride` floats (the tree's node count when coarsening follows).
__global__ void k_cluster_table(vplmc_lights v, vplmc_cut cut, uint64_t seed, int32_t *rep_out,
                                float *lights, float *bbox, int32_t stride) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = cut.n_clusters;
    if (c >= nc) return;
    const int b = cut.offsets[c], e = cut.offsets[c + 1];
    double smax = 0.0;
    for (int k = b; k < e; ++k) {
        const int id = clamp_index(cut.members[k], v.n);
        const double sk = ((double)v.ir[id] + (double)v.ig[id]) + (double)v.ib[id];
        smax = sk > smax ? sk : smax;
    }
    uint64_t total = 0;
    for (int k = b; k < e; ++k) {
        const int id = clamp_index(cut.members[k], v.n);
        const double sk = ((double)v.ir[id] + (double)v.ig[id]) + (double)v.ib[id];
        uint64_t w = 1;
        if (smax > 0.0) {
            const double f = floor((16777216.0 * sk) / smax);
            w = f > 1.0 ? (uint64_t)f : 1ull;
        }
        total += w;
    }
    int rep = e > b ? clamp_index(cut.members[b], v.n) : -1;
    if (e > b) {
        const uint64_t u = mulhi64(philox(seed, 0, (uint64_t)c, 0, TAG_REP, 0).a, total);
        uint64_t acc = 0;
        for (int k = b; k < e; ++k) {
            const int id = clamp_index(cut.members[k], v.n);
            const double sk = ((double)v.ir[id] + (double)v.ig[id]) + (double)v.ib[id];
            uint64_t w = 1;
            if (smax > 0.0) {
                const double f = floor((16777216.0 * sk) / smax);
                w = f > 1.0 ? (uint64_t)f : 1ull;
            }
            acc += w;
            if (acc > u) {
                rep = id;
                break;
            }
        }
    }
    double sr = 0.0, sg = 0.0, sb = 0.0;
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    for (int k = b; k < e; ++k) {
        const int id = clamp_index(cut.members[k], v.n);
        sr += (double)v.ir[id];
        sg += (double)v.ig[id];
        sb += (double)v.ib[id];
        lo0 = fminf(lo0, v.x[id]); hi0 = fmaxf(hi0, v.x[id]);
        lo1 = fminf(lo1, v.y[id]); hi1 = fmaxf(hi1, v.y[id]);
        lo2 = fminf(lo2, v.z[id]); hi2 = fmaxf(hi2, v.z[id]);
    }
    rep_out[c] = rep;
    const int r = rep < 0 ? 0 : rep;
    const size_t N = (size_t)stride;
    lights[0 * N + c] = v.x[r];
    lights[1 * N + c] = v.y[r];
    lights[2 * N + c] = v.z[r];
    lights[3 * N + c] = v.nx[r];
    lights[4 * N + c] = v.ny[r];
    lights[5 * N + c] = v.nz[r];
    lights[6 * N + c] = (float)sr;
    lights[7 * N + c] = (float)sg;
    lights[8 * N + c] = (float)sb;
    bbox[0 * N + c] = lo0;
    bbox[1 * N + c] = lo1;
    bbox[2 * N + c] = lo2;
    bbox[3 * N + c] = hi0;
    bbox[4 * N + c] = hi1;
    bbox[5 * N + c] = hi2;
}

// First pass: sample k of slice s is walk(k) of the keyed permutation.
__global__ void k_pass1(const SliceDesc *__restrict__ desc, int S, int64_t total, uint64_t seed,
                        uint32_t *omega1, uint32_t *bm, uint32_t *bmt) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int s = slice_of(desc, S, g, 0);
    const SliceDesc d = desc[s];
    const uint64_t k = (uint64_t)(g - d.off1);
    const uint64_t D = (uint64_t)d.m * (uint64_t)d.n;
    int b = D > 1 ? 64 - __clzll((long long)(D - 1)) : 0;
    b = b < 2 ? 2 : b;
    const int h = (b + 1) / 2;
    uint64_t e = feistel(k, seed, (uint64_t)s, h);
    while (e >= D) e = feistel(e, seed, (uint64_t)s, h);   // cycle-walking; ends in k's cycle
    const uint32_t i = (uint32_t)(e / (uint64_t)d.n), j = (uint32_t)(e % (uint64_t)d.n);
    omega1[g] = (i << 16) | j;
    atomicOr(bm + d.off_bm + (int64_t)i * d.words_row + (j >> 5), 1u << (j & 31));
    atomicOr(bmt + d.off_bmt + (int64_t)j * d.words_col + (i >> 5), 1u << (i & 31));
}

// Per-(slice, column) statistics of t = R + G + B over the first pass, one
// thread per column walking the column's first-pass entries in row order
// (a CSC ordering of the first pass alone), so every sum has a fixed order.
__global__ void k_colstats(const SliceDesc *__restrict__ desc, int S, int64_t total_cols,
                           const int32_t *__restrict__ col_ptr, const float *__restrict__ csc_val,
                           int32_t *cnt, float *mn, float *mx, double *sum, double *sumsq, int32_t *zeros) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total_cols) return;
    const int s = slice_of(desc, S, g, 3);
    const SliceDesc d = desc[s];
    const int64_t j = g - (d.off_colptr - s);
    if (j >= d.n) return;   // past a coarsened slice's columns
    const int b = col_ptr[d.off_colptr + j], e = col_ptr[d.off_colptr + j + 1];
    float lo = INFINITY, hi = 0.f;
    double s1 = 0.0, s2 = 0.0;
    int z = 0;
    for (int p = b; p < e; ++p) {
        const float *v = csc_val + 3 * (d.off_omega + p);
        const float tv = (v[0] + v[1]) + v[2];
        lo = fminf(lo, tv);
        hi = fmaxf(hi, tv);
        s1 += (double)tv;
        s2 += (double)tv * (double)tv;
        z += tv == 0.f;
    }
    const int64_t o = d.off_col + j;
    cnt[o] = e - b;
    mn[o] = e > b ? lo : 0.f;
    mx[o] = e > b ? hi : 0.f;
    sum[o] = s1;
    sumsq[o] = s2;
    zeros[o] = z;
}

// g(j) = max - min (Sec. 5, f(i) = 1) quantised to q_j = max(1, floor(2^24 g / max g))
// (0 where g = 0; all 1 if every g is 0) and its inclusive uint64 prefix.
// With logits (the learned proposal), w_j = max(1, floor(2^24 exp(y_j - max y)))
// in FP64 from the FP32 logits instead; a slice with any non-finite logit
// keeps the g weights and is flagged.  A positive mix (the density
// g(j) + mix mean g, a baseline for the learned proposal) offsets the g
// weights by c = floor(mix sum q / n') and rescales them,
// w_j = max(1, floor(2^24 (q_j + c) / (2^24 + c))); mix = +inf gives w_j = 1.
__device__ __forceinline__ uint32_t g_weight(float gj, float gmax) {
    if (!(gj > 0.f)) return 0u;
    const double f = floor((16777216.0 * (double)gj) / (double)gmax);
    return f > 1.0 ? (uint32_t)f : 1u;
}

__global__ __launch_bounds__(256) void k_weights(const SliceDesc *__restrict__ desc, const int32_t *cnt,
                                                 const float *mn, const float *mx, const float *logits, float mix,
                                                 uint32_t *w, uint64_t *prefix, int32_t *stats) {
    __shared__ uint32_t sm[8];
    __shared__ float smax[4];
    __shared__ int bad_s;
    __shared__ uint64_t carry_s;
    const int s = blockIdx.x;
    const SliceDesc d = desc[s];
    const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
    if (t == 0) bad_s = 0;
    __syncthreads();
    float gmax = 0.f, ymax = -INFINITY;
    for (int j = t; j < d.n; j += 256) {
        const int64_t o = d.off_col + j;
        const float gj = cnt[o] > 0 ? mx[o] - mn[o] : 0.f;
        gmax = fmaxf(gmax, gj);
        if (logits) {
            const float y = logits[o];
            if (!isfinite(y)) bad_s = 1;
            ymax = fmaxf(ymax, y);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) gmax = fmaxf(gmax, __shfl_xor(gmax, o, WAVE));
    if (lane == 0) smax[wv] = gmax;
    __syncthreads();
    gmax = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    __syncthreads();
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ymax = fmaxf(ymax, __shfl_xor(ymax, o, WAVE));
    if (lane == 0) smax[wv] = ymax;
    __syncthreads();
    ymax = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    const bool learned = logits != nullptr && !bad_s;
    if (logits && bad_s && t == 0) stats[4 * s + 1] |= VPLMC_SLICE_FALLBACK;
    const bool uniform = !(gmax > 0.f) || (!learned && isinf(mix));
    // the offset of the mixed density: c = floor(mix sum q / n') over the g weights
    uint64_t c = 0;
    if (!learned && !uniform && mix > 0.f) {
        uint64_t sq = 0;
        for (int j = t; j < d.n; j += 256) {
            const int64_t o = d.off_col + j;
            sq += g_weight(cnt[o] > 0 ? mx[o] - mn[o] : 0.f, gmax);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, WAVE);
        __shared__ uint64_t ssum[4];
        if (lane == 0) ssum[wv] = sq;
        __syncthreads();
        const uint64_t tot = (ssum[0] + ssum[1]) + (ssum[2] + ssum[3]);
        c = (uint64_t)floor(((double)mix * (double)tot) / (double)d.n);
    }
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int j0 = 0; j0 < d.n; j0 += 256) {
        const int j = j0 + t;
        uint32_t wj = 0;
        if (j < d.n) {
            const int64_t o = d.off_col + j;
            if (learned) {
                const double f = floor(16777216.0 * exp((double)logits[o] - (double)ymax));
                wj = f > 1.0 ? (uint32_t)f : 1u;
            } else if (uniform) {
                wj = 1;
            } else {
                wj = g_weight(cnt[o] > 0 ? mx[o] - mn[o] : 0.f, gmax);
                if (c > 0) {
                    const double f = floor((16777216.0 * (double)(wj + c)) / (double)(16777216ull + c));
                    wj = f > 1.0 ? (uint32_t)f : 1u;
                }
            }
            w[d.off_col + j] = wj;
        }
        // inclusive uint64 prefix.  Weights are <= 2^24, so an exclusive sum of
        // at most 255 of them fits in 32 bits, but a whole chunk of 256 may
        // reach 2^32 exactly: the chunk total is carried in 64 bits as the last
        // lane's inclusive prefix, not as the 32-bit block total.
        uint32_t tot;
        const uint32_t ex = block_excl_scan(wj, &tot, sm);
        const uint64_t carry = carry_s;
        const uint64_t incl = carry + (uint64_t)ex + wj;
        if (j < d.n) prefix[d.off_col + j] = incl;
        __syncthreads();
        if (t == 255) carry_s = incl;
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t load_word(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Second pass (Sec. 5): attempt t draws column j by the integer CDF of w and
// row i uniformly, and is accepted iff (i, j) is not sampled yet.  A block
// tests P2_THREADS consecutive attempts at once; an attempt is accepted iff
// its entry is not in the bitmap and no earlier attempt of the same batch
// drew it (the smallest attempt per entry, found through an LDS hash table),
// which is exactly the sequential rule.  Stops after N2 acceptances or
// 64 N2 + 65536 attempts.
constexpr int P2_LDS = 6144;       // prefix entries staged in LDS (48 KiB)
constexpr int P2_THREADS = 1024;   // attempts per batch
constexpr int P2_HASH = 4096;      // hash slots (load <= 1/4)
constexpr uint32_t P2_EMPTY = 0xFFFFFFFFu;

__global__ __launch_bounds__(P2_THREADS) void k_pass2(const SliceDesc *__restrict__ desc, uint64_t seed,
                                                      const uint64_t *__restrict__ prefix_all, uint32_t *bm,
                                                      uint32_t *bmt, uint32_t *omega2, int32_t *stats) {
    __shared__ uint64_t P[P2_LDS];
    __shared__ uint32_t hkey[P2_HASH];
    __shared__ uint32_t hmin[P2_HASH];
    __shared__ uint32_t sm[P2_THREADS / WAVE];
    __shared__ int accepted_s;
    const int s = blockIdx.x;
    const SliceDesc d = desc[s];
    const int t = threadIdx.x;
    const int m = d.m, n = d.n;
    const int64_t D = (int64_t)m * n;
    const int N2 = d.N2;
    uint32_t *out = omega2 + d.off2;
    uint32_t *bmr = bm + d.off_bm;
    uint32_t *bmc = bmt + d.off_bmt;
    if (t == 0) accepted_s = 0;
    __syncthreads();
    if (N2 > 0 && (int64_t)d.N1 + N2 == D) {
        // every remaining entry, row-major: scan the row-major bitmap in word order
        const int64_t words = (int64_t)m * d.words_row;
        for (int64_t w0 = 0; w0 < words; w0 += P2_THREADS) {
            const int64_t w = w0 + t;
            uint32_t freeb = 0;
            int i = 0, jb = 0;
            if (w < words) {
                i = (int)(w / d.words_row);
                jb = (int)(w % d.words_row) * 32;
                // (words past a coarsened slice's columns hold no entry)
                const int valid = n - jb >= 32 ? 32 : (n - jb > 0 ? n - jb : 0);
                const uint32_t vmask = valid == 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
                freeb = ~load_word(bmr + w) & vmask;
            }
            uint32_t tot;
            const uint32_t base = block_excl_scan(__popc(freeb), &tot, sm);
            const int a0 = accepted_s;
            uint32_t pos = (uint32_t)a0 + base;
            while (freeb) {
                const int b = __ffs(freeb) - 1;
                freeb &= freeb - 1;
                const uint32_t j = (uint32_t)(jb + b);
                out[pos++] = ((uint32_t)i << 16) | j;
                atomicOr(bmr + w, 1u << b);
                atomicOr(bmc + (int64_t)j * d.words_col + (i >> 5), 1u << (i & 31));
            }
            __syncthreads();
            if (t == 0) accepted_s = a0 + (int)tot;
            __syncthreads();
        }
    } else if (N2 > 0) {
        const uint64_t *pre = prefix_all + d.off_col;
        const bool in_lds = n <= P2_LDS;
        if (in_lds)
            for (int j = t; j < n; j += P2_THREADS) P[j] = pre[j];
        for (int h = t; h < P2_HASH; h += P2_THREADS) {
            hkey[h] = P2_EMPTY;
            hmin[h] = P2_EMPTY;
        }
        __syncthreads();
        const uint64_t totalw = pre[n - 1];
        const int64_t cap = 64 * (int64_t)N2 + 65536;
        for (int64_t tb = 0; tb < cap; tb += P2_THREADS) {
            const int acc0 = accepted_s;
            if (acc0 >= N2) break;
            const int64_t at = tb + t;
            bool cand = false;
            uint32_t key = 0xFFFFFFFFu, i = 0, j = 0;
            if (at < cap) {
                const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)at, 0, TAG_PASS2, 0);
                const uint64_t u = mulhi64(r.a, totalw);
                int lo = 0, hi = n - 1;      // least j with P[j] > u
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const uint64_t pm = in_lds ? P[mid] : pre[mid];
                    if (pm > u) hi = mid; else lo = mid + 1;
                }
                j = (uint32_t)lo;
                i = (uint32_t)mulhi64(r.b, (uint64_t)m);
                const uint32_t word = load_word(bmr + (int64_t)i * d.words_row + (j >> 5));
                cand = ((word >> (j & 31)) & 1u) == 0u;
                key = (i << 16) | j;
            }
            // smallest attempt of the batch per entry: open addressing, linear probing
            int slot = 0;
            if (cand) {
                slot = (int)((key * 2654435761u) >> 20) & (P2_HASH - 1);
                for (;;) {
                    const uint32_t old = atomicCAS(&hkey[slot], P2_EMPTY, key);
                    if (old == P2_EMPTY || old == key) break;
                    slot = (slot + 1) & (P2_HASH - 1);
                }
                atomicMin(&hmin[slot], (uint32_t)t);
            }
            __syncthreads();
            const bool acc = cand && hmin[slot] == (uint32_t)t;
            uint32_t tot;
            const uint32_t rank = block_excl_scan(acc ? 1u : 0u, &tot, sm);
            if (cand) {                       // every used slot is cleared by its entries
                hkey[slot] = P2_EMPTY;
                hmin[slot] = P2_EMPTY;
            }
            if (acc && acc0 + (int)rank < N2) {
                out[acc0 + rank] = key;
                atomicOr(bmr + (int64_t)i * d.words_row + (j >> 5), 1u << (j & 31));
                atomicOr(bmc + (int64_t)j * d.words_col + (i >> 5), 1u << (i & 31));
            }
            __syncthreads();
            if (t == 0) accepted_s = min(N2, acc0 + (int)tot);
            __syncthreads();
        }
    }
    __syncthreads();
    if (t == 0) {
        stats[4 * s + 3] = accepted_s;
        if (accepted_s < N2) stats[4 * s + 1] |= VPLMC_SLICE_SHORTFALL;
    }
}

// Popcount prefix of each bitmap row (one wavefront per row): wpre[w] = set
// bits before word w within the row; the row total goes to ptr[row + 1].
__global__ void k_rowscan(const SliceDesc *__restrict__ desc, int S, int64_t total_rows, int cols,
                          const uint32_t *__restrict__ bm, uint16_t *wpre, int32_t *ptr) {
    const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (g >= total_rows) return;
    const int s = slice_of(desc, S, g, cols ? 3 : 2);
    const SliceDesc d = desc[s];
    int64_t r, words, base_word, ptr_base;
    if (!cols) {
        r = g - (d.off_row - s);
        words = d.words_row;
        base_word = d.off_bm;
        ptr_base = d.off_row;
    } else {
        r = g - (d.off_colptr - s);
        if (r >= d.n) return;   // past a coarsened slice's columns
        words = d.words_col;
        base_word = d.off_bmt;
        ptr_base = d.off_colptr;
    }
    const uint32_t *row = bm + base_word + r * words;
    uint16_t *pre = wpre + base_word + r * words;
    uint32_t run = 0;
    for (int64_t w0 = 0; w0 < words; w0 += WAVE) {
        const int64_t w = w0 + lane;
        const uint32_t c = w < words ? (uint32_t)__popc(row[w]) : 0u;
        const uint32_t incl = wave_incl_scan(c, lane);
        if (w < words) pre[w] = (uint16_t)(run + incl - c);
        run += __shfl(incl, WAVE - 1, WAVE);
    }
    if (lane == 0) ptr[ptr_base + r + 1] = (int32_t)run;
}

// ptr[0] = 0, ptr[k + 1] = ptr[k] + count[k]: in-place inclusive scan per slice.
__global__ __launch_bounds__(256) void k_ptrscan(const SliceDesc *__restrict__ desc, int cols, int32_t *ptr) {
    __shared__ uint32_t sm[8];
    __shared__ uint32_t carry_s;
    const int s = blockIdx.x;
    const SliceDesc d = desc[s];
    const int64_t base = cols ? d.off_colptr : d.off_row;
    const int len = cols ? d.n : d.m;
    const int t = threadIdx.x;
    if (t == 0) {
        ptr[base] = 0;
        carry_s = 0;
    }
    __syncthreads();
    for (int k0 = 0; k0 < len; k0 += 256) {
        const int k = k0 + t;
        const uint32_t v = k < len ? (uint32_t)ptr[base + k + 1] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot, sm);
        const uint32_t carry = carry_s;
        if (k < len) ptr[base + k + 1] = (int32_t)(carry + ex + v);
        __syncthreads();
        if (t == 0) carry_s = carry + tot;
        __syncthreads();
    }
}

// parts of a column with c samples: p = max(1, ceil(c / ELL_LMAX)) of
// l = ceil(c / p) samples, the last one c - (p - 1) l
__device__ __forceinline__ void part_shape(int c, int &p, int &l) {
    p = c > ELL_LMAX ? (c + ELL_LMAX - 1) / ELL_LMAX : 1;
    l = (c + p - 1) / p;
}

// Scatter one pass's samples: a slice completed in global memory gets its CSC
// copy (and its CSR copy when csr_col is given); a slice completed from the
// ELL copy (when ell.row is given) gets only its ELL slot, whose position
// follows from the CSC rank.
__global__ void k_scatter(const SliceDesc *__restrict__ desc, int S, int64_t total, int which,
                          const int32_t *__restrict__ stats, const uint32_t *__restrict__ keys,
                          const float *__restrict__ vals, const uint32_t *__restrict__ bm,
                          const uint32_t *__restrict__ bmt, const uint16_t *__restrict__ wpre,
                          const uint16_t *__restrict__ wpret, const int32_t *__restrict__ row_ptr,
                          const int32_t *__restrict__ col_ptr, int32_t *csr_col, float *csr_val,
                          int32_t *csc_row, float *csc_val, EllView ell) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int s = slice_of(desc, S, g, which);
    const SliceDesc d = desc[s];
    const int64_t k = g - (which ? d.off2 : d.off1);
    if (which ? k >= stats[4 * s + 3] : k >= d.N1) return;
    const uint32_t key = keys[g];
    const uint32_t i = key >> 16, j = key & 0xFFFFu;
    // a slice completed from its ELL copy gets only that copy
    const bool to_ell = ell.row && d.ell;
    const int64_t wc = d.off_bmt + (int64_t)j * d.words_col + (i >> 5);
    const int64_t pc = col_ptr[d.off_colptr + j] + wpret[wc] + __popc(bmt[wc] & ((1u << (i & 31)) - 1u));
    const float v0 = vals[3 * g], v1 = vals[3 * g + 1], v2 = vals[3 * g + 2];
    const int64_t o = d.off_omega;
    if (csr_col && !to_ell) {
        const int64_t wr = d.off_bm + (int64_t)i * d.words_row + (j >> 5);
        const int64_t pr = row_ptr[d.off_row + i] + wpre[wr] + __popc(bm[wr] & ((1u << (j & 31)) - 1u));
        csr_col[o + pr] = (int32_t)j;
        csr_val[3 * (o + pr)] = v0;
        csr_val[3 * (o + pr) + 1] = v1;
        csr_val[3 * (o + pr) + 2] = v2;
    }
    if (!to_ell) {
        csc_row[o + pc] = (int32_t)i;
        csc_val[3 * (o + pc)] = v0;
        csc_val[3 * (o + pc) + 1] = v1;
        csc_val[3 * (o + pc) + 2] = v2;
    }
    if (to_ell) {
        const int32_t *cp = col_ptr + d.off_colptr;
        const int k2 = (int)(pc - cp[j]);
        int p, l;
        part_shape(cp[j + 1] - cp[j], p, l);
        const int u = k2 / l, kl = k2 - u * l;
        const int32_t sp = ell.ppos[d.off_part + ell.pbase[d.off_colptr + j] + u];
        const int64_t e = d.off_ell + ell.grp[d.off_grp + (sp >> 6)] + 64 * (int64_t)kl + (sp & 63);
        ell.row[e] = (uint16_t)i;
        ell.val[3 * e] = v0;
        ell.val[3 * e + 1] = v1;
        ell.val[3 * e + 2] = v2;
    }
}

// ELL parts of a slice: per column the first part (pbase), the parts sorted by
// length, descending (counting sort over the lengths; the order among equal
// lengths is immaterial to every result), and the offsets of the 64-part
// groups, a group taking 64 x the length of its first part.
__global__ __launch_bounds__(1024) void k_partsort(const SliceDesc *__restrict__ desc,
                                                   const int32_t *__restrict__ col_ptr, EllView ell) {
    __shared__ uint32_t hist[ELL_LMAX + 1];
    __shared__ uint32_t sm[1024 / WAVE];
    __shared__ uint32_t nsplit;
    const SliceDesc d = desc[blockIdx.x];
    if (!d.ell) return;
    const int n = d.n, t = threadIdx.x;
    const int32_t *cp = col_ptr + d.off_colptr;
    int32_t *pb = ell.pbase + d.off_colptr;
    int2 *part = ell.part + d.off_part;
    int32_t *ppos = ell.ppos + d.off_part;
    int32_t *grp = ell.grp + d.off_grp;
    if (t <= ELL_LMAX) hist[t] = 0;
    if (t == 0) nsplit = 0;
    uint32_t carry = 0, tot;
    for (int j0 = 0; j0 < n; j0 += 1024) {
        const int j = j0 + t;
        int p = 0, l;
        if (j < n) part_shape(cp[j + 1] - cp[j], p, l);
        const uint32_t ex = block_excl_scan((uint32_t)p, &tot, sm);
        if (j < n) pb[j] = (int32_t)(carry + ex);
        carry += tot;
    }
    const int P = (int)carry;
    if (t == 0) pb[n] = P;
    __syncthreads();
    for (int j = t; j < n; j += 1024) {
        const int c = cp[j + 1] - cp[j];
        int p, l;
        part_shape(c, p, l);
        for (int u = 0; u < p; ++u) atomicAdd(&hist[min(l, c - u * l)], 1u);
        if (p > 1) ell.split[d.off_col + atomicAdd(&nsplit, 1u)] = j;
    }
    __syncthreads();
    if (t == 0) ell.nsplit[blockIdx.x] = (int32_t)nsplit;
    if (t == 0) {
        uint32_t run = 0;
        for (int b = ELL_LMAX; b >= 0; --b) {
            const uint32_t h = hist[b];
            hist[b] = run;
            run += h;
        }
    }
    __syncthreads();
    for (int j = t; j < n; j += 1024) {
        const int c = cp[j + 1] - cp[j];
        int p, l;
        part_shape(c, p, l);
        for (int u = 0; u < p; ++u) {
            const uint32_t pos = atomicAdd(&hist[min(l, c - u * l)], 1u);
            part[pos] = make_int2(j | (min(l, c - u * l) << 16) | ((p > 1 ? 1 : 0) << 23), pb[j] + u);
            ppos[pb[j] + u] = (int32_t)pos;
        }
    }
    __threadfence_block();
    __syncthreads();
    const int G = (P + 63) / 64;
    carry = 0;
    for (int g0 = 0; g0 < G; g0 += 1024) {
        const int g = g0 + t;
        uint32_t len = 0;
        if (g < G) {
            len = 64u * (uint32_t)((part[64 * g].x >> 16) & 0x7F);
        }
        const uint32_t ex = block_excl_scan(len, &tot, sm);
        if (g < G) grp[g] = (int32_t)(carry + ex);
        carry += tot;
    }
    if (t == 0) grp[G] = (int32_t)carry;
}

// First-pass entries given by a caller (stage calls): each key of slice s
// (k < N1) sets its bit in both occupancy bitmaps; a key outside the slice, or
// one already set, is counted in *bad and sets nothing.
__global__ void k_keys_bitmap(const SliceDesc *__restrict__ desc, int S, int64_t total,
                              const uint32_t *__restrict__ keys, uint32_t *bm, uint32_t *bmt,
                              unsigned long long *bad) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int s = slice_of(desc, S, g, 0);
    const SliceDesc d = desc[s];
    if (g - d.off1 >= d.N1) return;
    const uint32_t key = keys[g];
    const uint32_t i = key >> 16, j = key & 0xFFFFu;
    if ((int)i >= d.m || (int)j >= d.n) {
        atomicAdd(bad, 1ull);
        return;
    }
    const uint32_t old = atomicOr(bm + d.off_bm + (int64_t)i * d.words_row + (j >> 5), 1u << (j & 31));
    if (old & (1u << (j & 31))) {
        atomicAdd(bad, 1ull);
        return;
    }
    atomicOr(bmt + d.off_bmt + (int64_t)j * d.words_col + (i >> 5), 1u << (i & 31));
}

// inclusive uint64 prefix of given column weights, one block per slice
__global__ __launch_bounds__(256) void k_prefix_given(const SliceDesc *__restrict__ desc, const uint32_t *w,
                                                      uint64_t *prefix) {
    __shared__ uint64_t carry_s;
    __shared__ uint64_t wsum[4];
    const int s = blockIdx.x, t = threadIdx.x;
    const SliceDesc d = desc[s];
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int j0 = 0; j0 < d.n; j0 += 256) {
        const int j = j0 + t;
        // weights may be anything up to 2^32 - 1 here: the block sum is kept in 64 bits
        const uint64_t wj = j < d.n ? (uint64_t)w[d.off_col + j] : 0ull;
        uint64_t incl = wj;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint64_t u = __shfl_up(incl, o, WAVE);
            if ((t % WAVE) >= o) incl += u;
        }
        if (t % WAVE == WAVE - 1) wsum[t / WAVE] = incl;
        __syncthreads();
        uint64_t base = carry_s;
        for (int k = 0; k < t / WAVE; ++k) base += wsum[k];
        if (j < d.n) prefix[d.off_col + j] = base + incl;
        __syncthreads();
        if (t == 255) carry_s = base + incl;
        __syncthreads();
    }
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

int launch_keys_bitmap(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *keys,
                       uint32_t *bm, uint32_t *bmt, unsigned long long *bad) {
    if (plan.tot1 <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_keys_bitmap, dim3(blocks_for(plan.tot1, 256)), dim3(256), 0, st, desc, plan.n_slices,
                       plan.tot1, keys, bm, bmt, bad);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_prefix_given(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *w,
                        uint64_t *prefix) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_prefix_given, dim3(plan.n_slices), dim3(256), 0, st, desc, w, prefix);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v) {
    if (n == 0) return VPLMC_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_count_out_of_range(hipStream_t st, const int32_t *ids, int64_t n, int32_t hi, unsigned long long *bad) {
    if (n <= 0) return VPLMC_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_count_out_of_range, dim3(blocks), dim3(256), 0, st, ids, n, hi, bad);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_count_unordered(hipStream_t st, const int32_t *offsets, int64_t n, unsigned long long *bad) {
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 256) / 256);
    hipLaunchKernelGGL(k_count_unordered, dim3(blocks), dim3(256), 0, st, offsets, n, bad);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_philox(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t n, uint64_t *out) {
    if (n <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, st, k0, k1, ctr, n, out);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_cluster_table(hipStream_t st, const vplmc_lights &v, const vplmc_cut &cut, uint64_t seed,
                         int32_t *rep, float *lights, float *bbox, int32_t stride) {
    if (cut.n_clusters <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_cluster_table, dim3(blocks_for(cut.n_clusters, 64)), dim3(64), 0, st, v, cut, seed,
                       rep, lights, bbox, stride);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_pass1(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, uint64_t seed,
                 uint32_t *omega1, uint32_t *bm, uint32_t *bmt) {
    if (plan.tot1 <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_pass1, dim3(blocks_for(plan.tot1, 256)), dim3(256), 0, st, desc, plan.n_slices,
                       plan.tot1, seed, omega1, bm, bmt);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_colstats(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *omega1,
                    const float *val1, const uint32_t *bmt, uint16_t *wpret, int32_t *col_ptr, int32_t *csc_row,
                    float *csc_val, int32_t *cnt, float *mn, float *mx, double *sum, double *sumsq, int32_t *zeros) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    const int S = plan.n_slices;
    const int64_t cols = plan.tot_col;
    // CSC ordering of the first pass alone (the column-major bitmap holds only it now)
    hipLaunchKernelGGL(k_rowscan, dim3(blocks_for(cols * WAVE, 256)), dim3(256), 0, st, desc, S, cols, 1, bmt, wpret,
                       col_ptr);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ptrscan, dim3(S), dim3(256), 0, st, desc, 1, col_ptr);
    VPLMC_HIP(hipGetLastError());
    if (plan.tot1 > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(plan.tot1, 256)), dim3(256), 0, st, desc, S, plan.tot1, 0,
                           (const int32_t *)nullptr, omega1, val1, (const uint32_t *)nullptr, bmt,
                           (const uint16_t *)nullptr, wpret, (const int32_t *)nullptr, col_ptr, (int32_t *)nullptr,
                           (float *)nullptr, csc_row, csc_val, EllView{});
        VPLMC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_colstats, dim3(blocks_for(cols, 256)), dim3(256), 0, st, desc, S, cols, col_ptr, csc_val,
                       cnt, mn, mx, sum, sumsq, zeros);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_weights(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *cnt,
                   const float *mn, const float *mx, const float *logits, float mix, uint32_t *w, uint64_t *prefix,
                   int32_t *stats) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_weights, dim3(plan.n_slices), dim3(256), 0, st, desc, cnt, mn, mx, logits, mix, w, prefix,
                       stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_pass2(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, uint64_t seed,
                 const uint64_t *prefix, uint32_t *bm, uint32_t *bmt, uint32_t *omega2, int32_t *stats) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_pass2, dim3(plan.n_slices), dim3(P2_THREADS), 0, st, desc, seed, prefix, bm, bmt, omega2,
                       stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_sort(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *bm,
                const uint32_t *bmt, uint16_t *wpre, uint16_t *wpret, int32_t *row_ptr, int32_t *col_ptr,
                const uint32_t *omega1, const float *val1, const uint32_t *omega2, const float *val2,
                const int32_t *stats, int32_t *csr_col, float *csr_val, int32_t *csc_row, float *csc_val,
                const EllView &ell) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    const int S = plan.n_slices;
    const int64_t rows = plan.tot_row - S;     // sum of m
    const int64_t cols = plan.tot_col;         // sum of n
    // row order (CSR) only for slices completed in global memory
    const bool csr = plan.n_ell < S;
    if (csr) {
        hipLaunchKernelGGL(k_rowscan, dim3(blocks_for(rows * WAVE, 256)), dim3(256), 0, st, desc, S, rows, 0, bm,
                           wpre, row_ptr);
        VPLMC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rowscan, dim3(blocks_for(cols * WAVE, 256)), dim3(256), 0, st, desc, S, cols, 1, bmt,
                       wpret, col_ptr);
    VPLMC_HIP(hipGetLastError());
    if (csr) {
        hipLaunchKernelGGL(k_ptrscan, dim3(S), dim3(256), 0, st, desc, 0, row_ptr);
        VPLMC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ptrscan, dim3(S), dim3(256), 0, st, desc, 1, col_ptr);
    VPLMC_HIP(hipGetLastError());
    if (plan.n_ell > 0) {
        hipLaunchKernelGGL(k_partsort, dim3(S), dim3(1024), 0, st, desc, col_ptr, ell);
        VPLMC_HIP(hipGetLastError());
    }
    if (plan.tot1 > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(plan.tot1, 256)), dim3(256), 0, st, desc, S, plan.tot1, 0,
                           stats, omega1, val1, bm, bmt, wpre, wpret, row_ptr, col_ptr, csr_col, csr_val, csc_row,
                           csc_val, ell);
        VPLMC_HIP(hipGetLastError());
    }
    if (plan.tot2 > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(plan.tot2, 256)), dim3(256), 0, st, desc, S, plan.tot2, 1,
                           stats, omega2, val2, bm, bmt, wpre, wpret, row_ptr, col_ptr, csr_col, csr_val, csc_row,
                           csc_val, ell);
        VPLMC_HIP(hipGetLastError());
    }
    return VPLMC_OK;
}

}  // namespace vplmc
