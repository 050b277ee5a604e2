// Completion of the slices whose X does not fit in LDS (rank 32, or tall
// slices), with X and Y in global memory, as a sequence of launches per
// iteration over all such slices of a rank bucket, so that every phase has
// the whole GPU and the launch boundaries order the phases (no workgroup
// waits for another):
//   init    (workgroup per slice)  scale, initial factors, GY, X system
//   rows    (per 64-row block)     residuals of the row's samples, R_i Y^T,
//                                  X+_i = X_i F + T_i Inv, U, Lambda (q/4 lanes per row)
//   ysys    (workgroup per slice)  residual norm and the stop test, GX = X+^T X+,
//                                  C = X+^T X, Y system
//   cols    (per 256-column block) residuals again from X and Y, X+^T R_j,
//                                  Y+_j = F Y_j + Inv T_j, V, Pi (q/4 lanes per column)
//   xsys    (workgroup per slice)  GY = Y+^T Y+, X system for the next iteration
//   final   (workgroup per slice)  the final X into the X region, statistics
// The two X buffers alternate by iteration parity.  The q x q systems (the X
// system in FP64, the Y system's FP32 rounding) and the slice's stop state live in
// GADM_SYS_BYTES per slice.  The iteration is the one the LDS-resident kernel
// runs (Appendix A, in the sparse-residual form of kernels_adm.hip); the Grams
// are sums in a fixed order, so results are bitwise reproducible.

#include "adm_common.h"

namespace vplmc {
namespace {

// rows and columns with at most this many samples are taken side by side by
// lane groups of a wavefront, longer ones by the whole wavefront each
// (measured on the rank-32 coarsened 1080p frame: 633 ms of completion at
// 256, 646 at 128, 663 at 64)
constexpr int GADM_LIGHT = 256;
// samples of a row or column whose loads a lane group issues together
constexpr int GADM_BATCH = 4;
// LDS tile of the Gram launches (floats): small enough for two workgroups
// per CU beside the q x q system's state
constexpr int GADM_STAGE = 4096;

struct GadmArgs {
    const SliceDesc *desc;
    const int32_t *ids;                  // the group's slices
    const int32_t *rowp, *colp;          // count + 1: prefixes of the slices' row and column blocks
    int32_t count;
    uint64_t seed;
    int32_t max_iter, mode;
    float tol, alpha0, beta0, gamma;
    const int32_t *row_ptr_all, *csr_col_all;
    const float *csr_val_all;
    const int32_t *col_ptr_all, *csc_row_all;
    const float *csc_val_all;
    float *X_all, *Xn_all, *Xp_all, *Lam_all, *Y_all, *Yp_all, *Pi_all, *scale_all;
    int32_t *stats_all;
    char *gsys;
    double *ge2;                         // the group's first row block slot
};

struct GSys {
    double *F, *Inv;                     // Q x Q, the X system: F = G Inv, Inv = (G + a I)^-1
    float *Ff, *If;                      // the Y system in FP32: Ff[a][b] = (Inv C)[a][b], If = Inv
    int32_t *state;                      // done, iterations, FP32 bits of the residual, all-zero
    double *dstate;                      // ||P_Omega M|| / s0, s0
};

__device__ __forceinline__ GSys gsys_of(char *base, int s) {
    char *p = base + (size_t)s * GADM_SYS_BYTES;
    GSys g;
    g.F = reinterpret_cast<double *>(p);
    g.Inv = g.F + 32 * 32;
    g.Ff = reinterpret_cast<float *>(p + 2 * 32 * 32 * 8);
    g.If = g.Ff + 32 * 32;
    g.state = reinterpret_cast<int32_t *>(p + 2 * 32 * 32 * 8 + 2 * 32 * 32 * 4);
    g.dstate = reinterpret_cast<double *>(p + 2 * 32 * 32 * 8 + 2 * 32 * 32 * 4 + 16);
    return g;
}

// Workgroups of a launch are dispatched to the 8 XCDs in turn (workgroup w to
// XCD w mod 8), each XCD with its own L2.  A row or column launch deals its
// blocks to the XCDs in chunks of XCD_CHUNK consecutive blocks, so that a
// slice's blocks (which read the same X and Y) mostly share an L2, while the
// costly first blocks (slices in decreasing cost) still spread over every
// XCD; the tail beyond the last whole round keeps w.
constexpr int N_XCD = 8;
constexpr int XCD_CHUNK = 16;
__device__ __forceinline__ int xcd_item(int w, int n) {
    constexpr int R = N_XCD * XCD_CHUNK;
    if (w >= n / R * R) return w;
    const int x = w % N_XCD, t = w / N_XCD;
    return ((t / XCD_CHUNK) * N_XCD + x) * XCD_CHUNK + t % XCD_CHUNK;
}

// A block's n rows or columns (items first .. first + n - 1 of the CSR/CSC
// pointer ptr) in decreasing sample count, ties by index, as keys
// (2^23 - 1 - count) << 8 | item sorted ascending in LDS (bitonic, N a power
// of two, at least n, at most the workgroup's threads); returns how many have
// more than GADM_LIGHT samples (they come first).  All threads call.
__device__ __forceinline__ int count_of_key(int key) { return 0x7FFFFF - (key >> 8); }
template <int N>
__device__ int sort_by_count(int *order, const int32_t *__restrict__ ptr, int first, int n, int t) {
    static_assert(N <= 256 && (N & (N - 1)) == 0, "a power of two, 8-bit item index");
    if (t < N) {
        int key = 0x7FFFFFFF;
        if (t < n) {
            const int cnt = ptr[first + t + 1] - ptr[first + t];
            key = ((0x7FFFFF - min(cnt, 0x7FFFFF)) << 8) | t;
        }
        order[t] = key;
    }
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            const int o = t ^ stride;
            if (t < N && o > t) {
                const int u = order[t], v = order[o];
                if ((u > v) == ((t & size) == 0)) {
                    order[t] = v;
                    order[o] = u;
                }
            }
        }
    return __syncthreads_count(t < n && count_of_key(order[t]) > GADM_LIGHT);
}

// item b of a launch over the group's blocks: the slice position k with
// pre[k] <= b < pre[k + 1]
__device__ __forceinline__ int block_slice(const int32_t *__restrict__ pre, int count, int b) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Cross Gram C = A^T B of two (rows x Q) FP32 matrices into sh.C, streamed
// through LDS like gram_rows (half a stage each).
template <int Q, int PCAP, int THREADS>
__device__ void gram_cross(AdmShared<Q> &sh, const float *__restrict__ A, const float *__restrict__ B, int rows,
                           float *part, float *stage) {
    constexpr int P = Q * Q, QB = Q / 4, NB = QB * QB;
    constexpr int HALF = GADM_STAGE / 2;
    constexpr int TR = HALF / Q;
    constexpr int NL = HALF / 4 / THREADS;
    static_assert(NL >= 1 && NL * 4 * THREADS == HALF, "tile split");
    const int t = fresh_tid();
    const int groups = min(THREADS / NB, PCAP / P);
    const int g = t / NB, blk = t % NB;
    const int a0 = 4 * (blk / QB), b0 = 4 * (blk % QB);
    const float4 *A4 = reinterpret_cast<const float4 *>(A);
    const float4 *B4 = reinterpret_cast<const float4 *>(B);
    const int64_t tot4 = (int64_t)rows * (Q / 4);
    const int ntiles = (rows + TR - 1) / TR;
    float acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.f;
    float4 *sa = reinterpret_cast<float4 *>(stage);
    float4 *sb = reinterpret_cast<float4 *>(stage + HALF);
    for (int tile = 0; tile < ntiles; ++tile) {
        float4 ba[NL], bb[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int64_t idx = (int64_t)tile * (HALF / 4) + u * THREADS + t;
            ba[u] = idx < tot4 ? A4[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
            bb[u] = idx < tot4 ? B4[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            sa[u * THREADS + t] = ba[u];
            sb[u * THREADS + t] = bb[u];
        }
        __syncthreads();
        const int rt = min(TR, rows - tile * TR);
        if (g < groups) {
            for (int r = g; r < rt; r += groups) {
                const float4 u = sa[(r * Q + a0) / 4];
                const float4 v = sb[(r * Q + b0) / 4];
                const float ua[4] = {u.x, u.y, u.z, u.w}, vb[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(ua[x], vb[y], acc[x][y]);
            }
        }
    }
    if (g < groups) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) part[g * P + (a0 + x) * Q + b0 + y] = acc[x][y];
    }
    __syncthreads();
    for (int e = t; e < P; e += THREADS) {
        float v = 0.f;
        for (int gg = 0; gg < groups; ++gg) v += part[gg * P + e];
        sh.C[e] = v;
    }
    __syncthreads();
}

// sh.F, sh.Inv of the X system (F = G Inv, Inv = (G + a I)^-1) from sh.G, stored into the slice's state
template <int Q, int THREADS>
__device__ void gadm_x_system(AdmShared<Q> &sh, const GSys &g, double alpha) {
    const int t = fresh_tid();
    spd_inverse<Q>(sh, alpha);
    for (int e = t; e < Q * Q; e += THREADS) {
        const int a = e / Q, b = e % Q;
        double v = 0.0;
        for (int l = 0; l < Q; ++l) v += (double)sh.G[a * Q + l] * sh.Inv[l * Q + b];
        g.F[e] = v;
        g.Inv[e] = sh.Inv[e];
    }
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_init(GadmArgs a) {
    constexpr int NW = THREADS / WAVE;
    __shared__ AdmShared<Q> sh;
    constexpr int PCAP = (NW * Q * Q > 2 * 1024) ? NW * Q * Q : 2 * 1024;
    __shared__ float part[PCAP];
    __shared__ __align__(16) float stage[GADM_STAGE];
    const int s = __builtin_amdgcn_readfirstlane(a.ids[blockIdx.x]);
    const SliceDesc d = a.desc[s];
    const int m = d.m, n = d.n;
    const int qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    const GSys g = gsys_of(a.gsys, s);
    const uint64_t seed = a.seed;
    const int32_t fixed_iters = a.mode;
    const int32_t *row_ptr = a.row_ptr_all + d.off_row;
    const float *csr_val = a.csr_val_all + 3 * d.off_omega;
    float *Xa = a.X_all + d.off_x;
    float *Xp = a.Xp_all + d.off_x;
    float *Lam = a.Lam_all + d.off_x;
    float *Y = a.Y_all + d.off_y;
    float *Yp = a.Yp_all + d.off_y;
    float *Pi = a.Pi_all + d.off_y;
    float *scale_all = a.scale_all;
    int32_t *st = a.stats_all + 4 * s;
    const int nnz = row_ptr[m];
    if (t == 0) {
        g.state[0] = 0;
        g.state[1] = a.max_iter;
        g.state[2] = __float_as_int(0.f);
        g.state[3] = 0;
    }

    // ---- scale s0 = mean sampled value; ||P_Omega M|| ----
    double sum = 0.0, sumsq = 0.0;
    for (int p = t; p < 3 * nnz; p += THREADS) {
        const double v = (double)csr_val[p];
        sum += v;
        sumsq += v * v;
    }
    sum = wave_sum_d(sum);
    sumsq = wave_sum_d(sumsq);
    if (lane == 0) {
        sh.red[wave] = sum;
        sh.red[16 + wave] = sumsq;
    }
    __syncthreads();
    double tot = 0.0, totsq = 0.0;
    for (int w = 0; w < NW; ++w) {
        tot += sh.red[w];
        totsq += sh.red[16 + w];
    }
    __syncthreads();
    if (!(nnz > 0 && tot > 0.0)) {
        for (int e = t; e < m * Q; e += THREADS) Xa[e] = 0.f;
        for (int e = t; e < 3 * n * Q; e += THREADS) Y[e] = 0.f;
        if (t == 0) {
            scale_all[s] = 0.f;
            st[0] = 0;
            st[1] |= VPLMC_SLICE_ALL_ZERO;
            st[2] = __float_as_int(0.f);
            g.state[0] = 1;     // done
            g.state[1] = 0;     // iterations
            g.state[3] = 1;     // all zero: the stats stand
        }
        return;
    }
    const double s0 = tot / (3.0 * (double)nnz);
    const float inv_s0 = (float)(1.0 / s0);
    const double normM = sqrt(totsq) / s0;
    if (t == 0) {
        scale_all[s] = (float)s0;
        g.dstate[0] = normM;
        g.dstate[1] = s0;
    }

    // ---- initial factors: fp32(u24(Philox) * fp32(2 / sqrt q)), or (mode bit 1)
    // the contents of the X and Y regions ----
    const float cq = (float)(2.0 / sqrt((double)qr));
    const bool given = (fixed_iters & 2) != 0;
    const bool nonneg = (fixed_iters & 4) == 0;    // mode bit 2: projections off
    for (int e = t; e < m * Q; e += THREADS) {
        const int i = e / Q, k = e % Q;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)i, (uint64_t)k, TAG_INITX, 0);
        const float v = k < qr ? (given ? Xa[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
        Xa[e] = v;
        Xp[e] = v;
        Lam[e] = 0.f;
    }
    for (int e = t; e < 3 * n * Q; e += THREADS) {
        const int j = e / (3 * Q), c = (e / Q) % 3, k = e % Q;
        const uint64_t col = (uint64_t)c * (uint64_t)n + (uint64_t)j;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)k, col, TAG_INITY, 0);
        const float v = k < qr ? (given ? Y[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
        Y[e] = v;
        Yp[e] = v;
        Pi[e] = 0.f;
    }
    __threadfence_block();
    __syncthreads();


    gram_rows<Q, PCAP, THREADS, GADM_STAGE>(sh, Y, 3 * n, part, stage);
    gadm_x_system<Q, THREADS>(sh, g, (double)a.alpha0 * (3.0 * n) / qr);
    (void)wave;
    (void)lane;
    (void)inv_s0;
}

// Sum over an aligned group of L lanes (L = 1, 2, 4 or 8) by DPP exchanges:
// within quads, then between the two quads of a half row.  Every lane of the
// group ends with the same bits (each step adds the same two operands).
template <int L>
__device__ __forceinline__ float group_sum(float v) {
    static_assert(L == 1 || L == 2 || L == 4 || L == 8, "group of 1, 2, 4 or 8 lanes");
    if constexpr (L >= 2)   // quad_perm [1, 0, 3, 2]
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    if constexpr (L >= 4)   // quad_perm [2, 3, 0, 1]
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    if constexpr (L >= 8)   // row_half_mirror
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    return v;
}

// Phase A of the global-memory completion, per 64-row block.  A row is held
// by a group of Q/4 lanes, each with four of the q components of X_i and of
// R_i Y^T, so a sampled Y_j is three coalesced loads per group.  The block's
// rows are sorted by sample count: rows of more than GADM_LIGHT samples are
// taken one at a time by a whole wavefront (group g walking samples g, g + G,
// ..., the groups' partial sums added in a fixed tree), the others 64/(Q/4)
// to a pass of a wavefront, a pass taking rows of similar length.
// X+_i = X_i F + T_i Inv with T_i = R_i Y^T + a U_i - L_i in FP64.
template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_rows(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    constexpr int L = Q / 4;        // lanes per row
    constexpr int G = WAVE / L;     // rows per pass of a wavefront
    static_assert(Q % 4 == 0 && L <= 8, "four components per lane, at most eight lanes per row");
    __shared__ __align__(16) double shF[Q * Q];
    __shared__ __align__(16) double shInv[Q * Q];
    __shared__ __align__(16) float stage[NW * G * 2 * Q];   // per row slot: X_i (q), T_i (q)
    __shared__ int order[GADM_RB];                          // the block's rows by decreasing count
    static_assert(GADM_RB <= THREADS, "one row of a block per thread in the sort");
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int k = block_slice(a.rowp, a.count, b);
    const int s = __builtin_amdgcn_readfirstlane(a.ids[k]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const int m = d.m, n = d.n, qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    const int r_beg = (b - a.rowp[k]) * GADM_RB, r_end = min(m, r_beg + GADM_RB);
    for (int e = t; e < Q * Q; e += THREADS) {
        shF[e] = g.F[e];
        shInv[e] = g.Inv[e];
    }
    const bool nonneg = (a.mode & 4) == 0;
    const float inv_s0 = (float)(1.0 / g.dstate[1]);
    const double alpha = (double)a.alpha0 * (3.0 * n) / qr;
    const float alpha_f = (float)alpha;
    const float ga = (float)((double)a.gamma * alpha);
    const float inv_alpha = (float)(1.0 / alpha);
    const int32_t *row_ptr = a.row_ptr_all + d.off_row;
    const int32_t *csr_col = a.csr_col_all + d.off_omega;
    const float *csr_val = a.csr_val_all + 3 * d.off_omega;
    const float *X = ((it & 1) ? a.Xn_all : a.X_all) + d.off_x;
    float *Xn = ((it & 1) ? a.X_all : a.Xn_all) + d.off_x;
    float *Xp = a.Xp_all + d.off_x;
    float *Lam = a.Lam_all + d.off_x;
    const float *Y = a.Y_all + d.off_y;
    const int slot = lane / L, k0 = 4 * (lane % L);
    const bool lead = lane % L == 0;
    __syncthreads();
    double e2 = 0.0;

    // GADM_BATCH samples of row i at local positions p + u * step, active
    // while below lim (group-uniform): r = M - X_i . Y_j per channel,
    // acc += sum_c r_c Y_j(c), the squared residual on the group's first lane.
    // The loads of the batch are issued together; an inactive sample reads
    // the slice's first sample (every slice in this launch has one) and adds
    // nothing.
    auto samples = [&](int p, int step, int lim, int beg, const float (&x)[4], float (&acc)[4]) {
        bool act[GADM_BATCH];
        int pos[GADM_BATCH], jj[GADM_BATCH];
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
            act[u] = p + u * step < lim;
            pos[u] = act[u] ? beg + p + u * step : 0;
            jj[u] = csr_col[pos[u]];
        }
        float mv[GADM_BATCH][3];
        float4 yv[GADM_BATCH][3];
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mv[u][c] = csr_val[3 * pos[u] + c];
            const float *yj = Y + (size_t)jj[u] * 3 * Q + k0;
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[u][c] = *reinterpret_cast<const float4 *>(yj + c * Q);
        }
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
            const float y[3][4] = {{yv[u][0].x, yv[u][0].y, yv[u][0].z, yv[u][0].w},
                                   {yv[u][1].x, yv[u][1].y, yv[u][1].z, yv[u][1].w},
                                   {yv[u][2].x, yv[u][2].y, yv[u][2].z, yv[u][2].w}};
            float r[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float dd = 0.f;
#pragma unroll
                for (int e = 0; e < 4; ++e) dd = fmaf(x[e], y[c][e], dd);
                const float rc = mv[u][c] * inv_s0 - group_sum<L>(dd);
                r[c] = act[u] ? rc : 0.f;
            }
            if (act[u] && lead) e2 += (double)(r[0] * r[0]) + (double)(r[1] * r[1]) + (double)(r[2] * r[2]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[e] = fmaf(r[0], y[0][e], fmaf(r[1], y[1][e], fmaf(r[2], y[2][e], acc[e])));
        }
    };
    // T_i staged beside X_i in the row's LDS slot (the group's lanes)
    auto stage_row = [&](int i, const float (&x)[4], const float (&acc)[4], float *wst, float (&lam)[4]) {
        const float4 u = *reinterpret_cast<const float4 *>(Xp + (size_t)i * Q + k0);
        const float4 l = *reinterpret_cast<const float4 *>(Lam + (size_t)i * Q + k0);
        lam[0] = l.x; lam[1] = l.y; lam[2] = l.z; lam[3] = l.w;
        *reinterpret_cast<float4 *>(wst + k0) = make_float4(x[0], x[1], x[2], x[3]);
        *reinterpret_cast<float4 *>(wst + Q + k0) =
            make_float4(acc[0] + alpha_f * u.x - l.x, acc[1] + alpha_f * u.y - l.y, acc[2] + alpha_f * u.z - l.z,
                        acc[3] + alpha_f * u.w - l.w);
    };
    // components k0..k0+3 of X+_i, then U and Lambda
    auto finish_row = [&](int i, const float *wst, const float (&lam)[4]) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int l = 0; l < Q; ++l) {
            const double xl = (double)wst[l], tl = (double)wst[Q + l];
            const double2 f01 = *reinterpret_cast<const double2 *>(shF + l * Q + k0);
            const double2 f23 = *reinterpret_cast<const double2 *>(shF + l * Q + k0 + 2);
            const double2 h01 = *reinterpret_cast<const double2 *>(shInv + l * Q + k0);
            const double2 h23 = *reinterpret_cast<const double2 *>(shInv + l * Q + k0 + 2);
            v[0] += xl * f01.x + tl * h01.x;
            v[1] += xl * f01.y + tl * h01.y;
            v[2] += xl * f23.x + tl * h23.x;
            v[3] += xl * f23.y + tl * h23.y;
        }
        float xn[4], un[4], ln[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            xn[e] = (float)v[e];
            un[e] = nonneg ? fmaxf(0.f, xn[e] + lam[e] * inv_alpha) : xn[e] + lam[e] * inv_alpha;
            ln[e] = lam[e] + ga * (xn[e] - un[e]);
        }
        const size_t w = (size_t)i * Q + k0;
        *reinterpret_cast<float4 *>(Xn + w) = make_float4(xn[0], xn[1], xn[2], xn[3]);
        *reinterpret_cast<float4 *>(Xp + w) = make_float4(un[0], un[1], un[2], un[3]);
        *reinterpret_cast<float4 *>(Lam + w) = make_float4(ln[0], ln[1], ln[2], ln[3]);
    };
    auto load_x = [&](int i, float (&x)[4]) {
        const float4 u = *reinterpret_cast<const float4 *>(X + (size_t)i * Q + k0);
        x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w;
    };

    // the block's rows in decreasing sample count: a pass takes rows of
    // similar length; the longer ones come first and are dealt to the
    // wavefronts in turn
    const int nloc = r_end - r_beg;
    const int n_heavy = sort_by_count<GADM_RB>(order, row_ptr, r_beg, nloc, t);

    // the longer rows, one at a time by the whole wavefront
    for (int h = wave; h < n_heavy; h += NW) {
        const int ih = r_beg + (order[h] & 0xFF);
        const int hbeg = row_ptr[ih], hcnt = row_ptr[ih + 1] - hbeg;
        float x[4], acc[4] = {0.f, 0.f, 0.f, 0.f}, lam[4];
        load_x(ih, x);
        for (int p0 = 0; p0 < hcnt; p0 += G * GADM_BATCH) samples(p0 + slot, G, hcnt, hbeg, x, acc);
        // groups differ in lane bits log2(L) and up: add them pairwise
#pragma unroll
        for (int o = L; o < WAVE; o <<= 1)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += __shfl_xor(acc[e], o, WAVE);
        float *hst = stage + wave * G * 2 * Q;   // slot 0 of the wavefront
        if (slot == 0) stage_row(ih, x, acc, hst, lam);
        wave_lds_sync();
        if (slot == 0) finish_row(ih, hst, lam);
        wave_lds_sync();
    }
    // the others side by side, G to a pass; the pass's first is its longest
    for (int pb = n_heavy + wave * G; pb < nloc; pb += NW * G) {
        const int sp = pb + slot;
        const bool in = sp < nloc;
        int i = 0, beg = 0, lc = 0;
        if (in) {
            i = r_beg + (order[sp] & 0xFF);
            beg = row_ptr[i];
            lc = row_ptr[i + 1] - beg;
        }
        const int mc = __builtin_amdgcn_readfirstlane(count_of_key(order[pb]));
        float *wst = stage + (wave * G + slot) * 2 * Q;
        float x[4] = {0.f, 0.f, 0.f, 0.f}, acc[4] = {0.f, 0.f, 0.f, 0.f}, lam[4];
        if (in) load_x(i, x);
        for (int p = 0; p < mc; p += GADM_BATCH) samples(p, 1, lc, beg, x, acc);
        if (in) stage_row(i, x, acc, wst, lam);
        wave_lds_sync();
        if (in) finish_row(i, wst, lam);
        // the next row's stage overwrites this slot
        wave_lds_sync();
    }
    e2 = wave_sum_d(e2);
    __shared__ double red[NW];
    if (lane == 0) red[wave] = e2;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int w = 0; w < NW; ++w) tot += red[w];
        a.ge2[b] = tot;
    }
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_ysys(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    __shared__ AdmShared<Q> sh;
    constexpr int PCAP = (NW * Q * Q > 2 * 1024) ? NW * Q * Q : 2 * 1024;
    __shared__ float part[PCAP];
    __shared__ __align__(16) float stage[GADM_STAGE];
    __shared__ int stop_s;
    const int k = blockIdx.x;
    const int s = __builtin_amdgcn_readfirstlane(a.ids[k]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const int m = d.m, qr = d.qr;
    const int t = threadIdx.x;
    if (t == 0) {
        // the squared residuals of the slice's row blocks, in block order
        double e2 = 0.0;
        for (int rb = a.rowp[k]; rb < a.rowp[k + 1]; ++rb) e2 += a.ge2[rb];
        const double err = sqrt(e2) / g.dstate[0];
        g.state[2] = __float_as_int((float)err);
        const bool stop = !(a.mode & 1) && err < (double)a.tol;
        if (stop) {
            g.state[0] = 1;
            g.state[1] = it;
        }
        stop_s = stop ? 1 : 0;
    }
    __syncthreads();
    if (stop_s) return;
    const float *X = ((it & 1) ? a.Xn_all : a.X_all) + d.off_x;
    const float *Xn = ((it & 1) ? a.X_all : a.Xn_all) + d.off_x;
    gram_rows<Q, PCAP, THREADS, GADM_STAGE>(sh, Xn, m, part, stage);
    gram_cross<Q, PCAP, THREADS>(sh, Xn, X, m, part, stage);
    // the Y system; the column launch reads its FP32 rounding
    const double beta = (double)a.beta0 * (double)m / qr;
    spd_inverse<Q>(sh, beta);
    for (int e = t; e < Q * Q; e += THREADS) {
        const int aa = e / Q, bb = e % Q;   // Ff[a][b] = sum_l Inv[a][l] C[l][b]
        double v = 0.0;
        for (int l = 0; l < Q; ++l) v += sh.Inv[aa * Q + l] * (double)sh.C[l * Q + bb];
        g.Ff[e] = (float)v;
        g.If[e] = (float)sh.Inv[e];
    }
}

// Phase B of the global-memory completion, per 256-column block.  A column is
// held by a group of Q/4 lanes, each with four of the q components of Y_j and
// of X+^T R_j for the three channels, so a sampled row X_i / X+_i is one
// coalesced load per group.  The block's columns are sorted by sample count
// and taken as the rows are in k_gadm_rows: the longest one at a time by a
// whole wavefront, the others 64/(Q/4) to a pass.
// Y+_j = F Y_j + Inv T_j with T_j = X+^T R_j + b V_j - P_j uses the FP32
// copies of the two q x q matrices, transposed in LDS.
template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_cols(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    constexpr int L = Q / 4;        // lanes per column
    constexpr int G = WAVE / L;     // columns per pass of a wavefront
    static_assert(Q % 4 == 0 && L <= 8, "four components per lane, at most eight lanes per column");
    __shared__ __align__(16) float Ft[Q * Q];    // Ft[l][k] = (Inv C)[k][l]
    __shared__ __align__(16) float It[Q * Q];    // It[l][k] = Inv[k][l]
    __shared__ __align__(16) float stage[NW * G * 6 * Q];   // per column slot: Y_j (3q), T_j (3q)
    __shared__ int order[GADM_CB];                          // the block's columns by decreasing count
    static_assert(GADM_CB <= THREADS, "one column of a block per thread in the sort");
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int k = block_slice(a.colp, a.count, b);
    const int s = __builtin_amdgcn_readfirstlane(a.ids[k]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const int m = d.m, qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    const int c_beg = (b - a.colp[k]) * GADM_CB, c_end = min(d.n, c_beg + GADM_CB);
    for (int e = t; e < Q * Q; e += THREADS) {
        const int r = e / Q, c = e % Q;
        Ft[c * Q + r] = g.Ff[e];
        It[c * Q + r] = g.If[e];
    }
    const bool nonneg = (a.mode & 4) == 0;
    const float inv_s0 = (float)(1.0 / g.dstate[1]);
    const double beta = (double)a.beta0 * (double)m / qr;
    const float beta_f = (float)beta;
    const float gb = (float)((double)a.gamma * beta);
    const float inv_beta = (float)(1.0 / beta);
    const int32_t *col_ptr = a.col_ptr_all + d.off_colptr;
    const int32_t *csc_row = a.csc_row_all + d.off_omega;
    const float *csc_val = a.csc_val_all + 3 * d.off_omega;
    const float *X = ((it & 1) ? a.Xn_all : a.X_all) + d.off_x;
    const float *Xn = ((it & 1) ? a.X_all : a.Xn_all) + d.off_x;
    float *Y = a.Y_all + d.off_y;
    float *Yp = a.Yp_all + d.off_y;
    float *Pi = a.Pi_all + d.off_y;
    const int slot = lane / L, k0 = 4 * (lane % L);
    __syncthreads();

    // GADM_BATCH samples of column j at local positions p + u * step, active
    // while below lim (group-uniform): r = M - X_i . Y_j per channel,
    // acc += X+_i r.  The loads of the batch are issued together; an inactive
    // sample reads the slice's first sample and adds nothing.
    auto samples = [&](int p, int step, int lim, int beg, const float (&y)[3][4], float (&acc)[3][4]) {
        bool act[GADM_BATCH];
        int pos[GADM_BATCH], ii[GADM_BATCH];
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
            act[u] = p + u * step < lim;
            pos[u] = act[u] ? beg + p + u * step : 0;
            ii[u] = csc_row[pos[u]];
        }
        float mv[GADM_BATCH][3];
        float4 xa[GADM_BATCH], xb[GADM_BATCH];
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mv[u][c] = csc_val[3 * pos[u] + c];
            xa[u] = *reinterpret_cast<const float4 *>(X + (size_t)ii[u] * Q + k0);
            xb[u] = *reinterpret_cast<const float4 *>(Xn + (size_t)ii[u] * Q + k0);
        }
#pragma unroll
        for (int u = 0; u < GADM_BATCH; ++u) {
            const float xr[4] = {xa[u].x, xa[u].y, xa[u].z, xa[u].w};
            const float xn[4] = {xb[u].x, xb[u].y, xb[u].z, xb[u].w};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float dd = 0.f;
#pragma unroll
                for (int e = 0; e < 4; ++e) dd = fmaf(xr[e], y[c][e], dd);
                const float rc = mv[u][c] * inv_s0 - group_sum<L>(dd);
                const float r = act[u] ? rc : 0.f;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(xn[e], r, acc[c][e]);
            }
        }
    };
    auto load_y = [&](int j, float (&y)[3][4]) {
        const float4 *yj = reinterpret_cast<const float4 *>(Y + (size_t)j * 3 * Q + k0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 u = yj[c * Q / 4];
            y[c][0] = u.x; y[c][1] = u.y; y[c][2] = u.z; y[c][3] = u.w;
        }
    };
    // T_j staged beside Y_j in the column's LDS slot (the group's lanes)
    auto stage_column = [&](int j, const float (&y)[3][4], const float (&acc)[3][4], float *wst, float (&pv)[3][4]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 v = *reinterpret_cast<const float4 *>(Yp + (size_t)j * 3 * Q + c * Q + k0);
            const float4 pp = *reinterpret_cast<const float4 *>(Pi + (size_t)j * 3 * Q + c * Q + k0);
            pv[c][0] = pp.x; pv[c][1] = pp.y; pv[c][2] = pp.z; pv[c][3] = pp.w;
            *reinterpret_cast<float4 *>(wst + c * Q + k0) = make_float4(y[c][0], y[c][1], y[c][2], y[c][3]);
            *reinterpret_cast<float4 *>(wst + 3 * Q + c * Q + k0) =
                make_float4(acc[c][0] + beta_f * v.x - pp.x, acc[c][1] + beta_f * v.y - pp.y,
                            acc[c][2] + beta_f * v.z - pp.z, acc[c][3] + beta_f * v.w - pp.w);
        }
    };
    // components k0..k0+3 of Y+_j for the three channels, then U, P and Y
    auto finish_column = [&](int j, const float *wst, const float (&pv)[3][4]) {
        float o[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) o[c][e] = 0.f;
#pragma unroll 2
        for (int l = 0; l < Q; l += 4) {
            float yl[3][4], tl[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 u = *reinterpret_cast<const float4 *>(wst + c * Q + l);
                const float4 v = *reinterpret_cast<const float4 *>(wst + 3 * Q + c * Q + l);
                yl[c][0] = u.x; yl[c][1] = u.y; yl[c][2] = u.z; yl[c][3] = u.w;
                tl[c][0] = v.x; tl[c][1] = v.y; tl[c][2] = v.z; tl[c][3] = v.w;
            }
#pragma unroll
            for (int ll = 0; ll < 4; ++ll) {
                const float4 f = *reinterpret_cast<const float4 *>(Ft + (l + ll) * Q + k0);
                const float4 h = *reinterpret_cast<const float4 *>(It + (l + ll) * Q + k0);
                const float fa[4] = {f.x, f.y, f.z, f.w}, ha[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[c][e] = fmaf(fa[e], yl[c][ll], fmaf(ha[e], tl[c][ll], o[c][e]));
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float un[4], pn[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                un[e] = nonneg ? fmaxf(0.f, o[c][e] + pv[c][e] * inv_beta) : o[c][e] + pv[c][e] * inv_beta;
                pn[e] = pv[c][e] + gb * (o[c][e] - un[e]);
            }
            const size_t w = (size_t)j * 3 * Q + c * Q + k0;
            *reinterpret_cast<float4 *>(Yp + w) = make_float4(un[0], un[1], un[2], un[3]);
            *reinterpret_cast<float4 *>(Pi + w) = make_float4(pn[0], pn[1], pn[2], pn[3]);
            *reinterpret_cast<float4 *>(Y + w) = make_float4(o[c][0], o[c][1], o[c][2], o[c][3]);
        }
    };

    // the block's columns in decreasing sample count: a pass takes columns of
    // similar length; the longer ones come first and are dealt to the
    // wavefronts in turn
    const int nloc = c_end - c_beg;
    const int n_heavy = sort_by_count<GADM_CB>(order, col_ptr, c_beg, nloc, t);

    // the longer columns, one at a time by the whole wavefront
    for (int h = wave; h < n_heavy; h += NW) {
        const int jh = c_beg + (order[h] & 0xFF);
        const int hbeg = col_ptr[jh], hcnt = col_ptr[jh + 1] - hbeg;
        float y[3][4], acc[3][4], pv[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[c][e] = 0.f;
        load_y(jh, y);
        for (int p0 = 0; p0 < hcnt; p0 += G * GADM_BATCH) samples(p0 + slot, G, hcnt, hbeg, y, acc);
        // groups differ in lane bits log2(L) and up: add them pairwise
#pragma unroll
        for (int o = L; o < WAVE; o <<= 1)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[c][e] += __shfl_xor(acc[c][e], o, WAVE);
        float *hst = stage + wave * G * 6 * Q;   // slot 0 of the wavefront
        if (slot == 0) stage_column(jh, y, acc, hst, pv);
        wave_lds_sync();
        if (slot == 0) finish_column(jh, hst, pv);
        wave_lds_sync();
    }
    // the others side by side, G to a pass; the pass's first is its longest
    for (int pb = n_heavy + wave * G; pb < nloc; pb += NW * G) {
        const int sp = pb + slot;
        const bool in = sp < nloc;
        int j = 0, beg = 0, lc = 0;
        if (in) {
            j = c_beg + (order[sp] & 0xFF);
            beg = col_ptr[j];
            lc = col_ptr[j + 1] - beg;
        }
        const int mc = __builtin_amdgcn_readfirstlane(count_of_key(order[pb]));
        float *wst = stage + (wave * G + slot) * 6 * Q;
        float y[3][4], acc[3][4], pv[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) y[c][e] = acc[c][e] = 0.f;
        if (in) load_y(j, y);
        for (int p = 0; p < mc; p += GADM_BATCH) samples(p, 1, lc, beg, y, acc);
        if (in) stage_column(j, y, acc, wst, pv);
        wave_lds_sync();
        if (in) finish_column(j, wst, pv);
        // the next column's stage overwrites this slot
        wave_lds_sync();
    }
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_xsys(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    __shared__ AdmShared<Q> sh;
    constexpr int PCAP = (NW * Q * Q > 2 * 1024) ? NW * Q * Q : 2 * 1024;
    __shared__ float part[PCAP];
    __shared__ __align__(16) float stage[GADM_STAGE];
    const int s = __builtin_amdgcn_readfirstlane(a.ids[blockIdx.x]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const float *Y = a.Y_all + d.off_y;
    gram_rows<Q, PCAP, THREADS, GADM_STAGE>(sh, Y, 3 * d.n, part, stage);
    gadm_x_system<Q, THREADS>(sh, g, (double)a.alpha0 * (3.0 * d.n) / d.qr);
    (void)it;
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_final(GadmArgs a) {
    const int s = __builtin_amdgcn_readfirstlane(a.ids[blockIdx.x]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[3]) return;                  // all-zero slice: set by the init launch
    const SliceDesc d = a.desc[s];
    const int iters = g.state[1];
    const int t = threadIdx.x;
    if (iters & 1) {                          // the final X is in the second buffer
        const float *src = a.Xn_all + d.off_x;
        float *dst = a.X_all + d.off_x;
        for (int e = t; e < d.m * Q; e += THREADS) dst[e] = src[e];
    }
    if (t == 0) {
        int32_t *st = a.stats_all + 4 * s;
        st[0] = iters;
        if (!(a.mode & 1) && iters >= a.max_iter) st[1] |= VPLMC_SLICE_NOT_CONVERGED;
        st[2] = g.state[2];
    }
}

// the global-memory completion of group grp (odd: X in global memory): an
// init launch, four launches per iteration, a final launch
template <int Q, int THREADS>
int launch_gadm(hipStream_t st, const vplmc_plan &plan, int grp, const int32_t *ids, const int32_t *gblk_dev,
                char *gsys, double *ge2, const SliceDesc *desc, const vplmc_params &prm, const int32_t *row_ptr,
                const int32_t *csr_col, const float *csr_val, const int32_t *col_ptr, const int32_t *csc_row,
                const float *csc_val, float *X, float *Xn, float *Xp, float *Lam, float *Y, float *Yp, float *Pi,
                float *scale, int32_t *stats) {
    const size_t count = plan.groups[grp].size();
    if (count == 0) return VPLMC_OK;
    GadmArgs a;
    a.desc = desc;
    a.ids = ids;
    a.rowp = gblk_dev + plan.gblk_off[grp];
    a.colp = a.rowp + count + 1;
    a.count = (int32_t)count;
    a.seed = prm.seed;
    a.max_iter = prm.max_iter;
    a.mode = adm_mode(prm);
    a.tol = prm.tol;
    a.alpha0 = prm.alpha0;
    a.beta0 = prm.beta0;
    a.gamma = prm.gamma;
    a.row_ptr_all = row_ptr;
    a.csr_col_all = csr_col;
    a.csr_val_all = csr_val;
    a.col_ptr_all = col_ptr;
    a.csc_row_all = csc_row;
    a.csc_val_all = csc_val;
    a.X_all = X;
    a.Xn_all = Xn;
    a.Xp_all = Xp;
    a.Lam_all = Lam;
    a.Y_all = Y;
    a.Yp_all = Yp;
    a.Pi_all = Pi;
    a.scale_all = scale;
    a.stats_all = stats;
    a.gsys = gsys;
    a.ge2 = ge2 + plan.ge2_base[grp];
    const unsigned nr = (unsigned)plan.g_rows[grp], nc = (unsigned)plan.g_cols[grp];
    hipLaunchKernelGGL((k_gadm_init<Q, THREADS>), dim3((unsigned)count), dim3(THREADS), 0, st, a);
    VPLMC_HIP(hipGetLastError());
    for (int it = 0; it < prm.max_iter; ++it) {
        hipLaunchKernelGGL((k_gadm_rows<Q, THREADS>), dim3(nr), dim3(THREADS), 0, st, a, it);
        VPLMC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_gadm_ysys<Q, THREADS>), dim3((unsigned)count), dim3(THREADS), 0, st, a, it);
        VPLMC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_gadm_cols<Q, THREADS>), dim3(nc), dim3(THREADS), 0, st, a, it);
        VPLMC_HIP(hipGetLastError());
        if (it + 1 < prm.max_iter) {
            hipLaunchKernelGGL((k_gadm_xsys<Q, THREADS>), dim3((unsigned)count), dim3(THREADS), 0, st, a, it);
            VPLMC_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL((k_gadm_final<Q, THREADS>), dim3((unsigned)count), dim3(THREADS), 0, st, a);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace

int launch_gadm_group(hipStream_t st, int q, const vplmc_plan &plan, int grp, const int32_t *ids,
                      const int32_t *gblk_dev, char *gsys, double *ge2, const SliceDesc *desc,
                      const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
                      const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Xn,
                      float *Xp, float *Lam, float *Y, float *Yp, float *Pi, float *scale, int32_t *stats) {
#define VPLMC_GADM(QQ)                                                                                             \
    return launch_gadm<QQ, 256>(st, plan, grp, ids, gblk_dev, gsys, ge2, desc, prm, row_ptr, csr_col, csr_val,   \
                                col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats)
    switch (q) {
    case 4: VPLMC_GADM(4);
    case 8: VPLMC_GADM(8);
    case 16: VPLMC_GADM(16);
    case 32: VPLMC_GADM(32);
    default: return VPLMC_EINVAL;
    }
#undef VPLMC_GADM
}

}  // namespace vplmc
