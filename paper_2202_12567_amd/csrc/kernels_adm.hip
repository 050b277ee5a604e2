// Non-negative completion of each slice matrix by the alternating direction
// method (Appendix A), and the factorised column sum I(s) = X (Y e)
// (Sec. 3, step 5).
//
// A slice whose X fits in LDS is completed by one workgroup for all its
// iterations (k_adm_ell), so an iteration needs only workgroup barriers; the
// others (rank 32, tall slices) by a sequence of launches per iteration over
// all such slices (k_gadm_*, below).  The slice matrix is the stacked
// m' x 3n' matrix [M_R | M_G | M_B] known on the sampled entries; Y is
// stored cluster-major, Y[j][c][k] = the paper's Y(k, c n' + j).
//
// Iteration k (sparse-residual form of the appendix's updates, with
// R = P_Omega(M - X Y) and hence Z Y^T = X (Y Y^T) + R Y^T,
// X+^T Z = (X+^T X) Y + X+^T R):
//   phase A, one wavefront per row i, one lane per sampled entry (CSR):
//     r = M(i, j) - X_i . Y_j for the 3 channels, err += r^2,
//     RX_i = sum r Y_j;  X+_i = X_i GY (GY + aI)^-1 + (RX_i + a U_i - L_i)(GY + aI)^-1,
//     U_i = max(0, X+_i + L_i / a), L_i += g a (X+_i - U_i),
//     and the Grams X+^T X+ and X+^T X are accumulated;
//   stop test on ||R|| / ||P_Omega M|| (before any state is kept);
//   phase B, per column j (CSC): the residual again from (X_k, Y_k),
//     RY_j = sum r X+_i, Y+_j = (GX + bI)^-1 ((X+^T X) Y_j + RY_j + b V_j - P_j),
//     V_j = max(0, Y+_j + P_j / b), P_j += g b (Y+_j - V_j); a column of at
//     most GADM_LIGHT samples by one lane, a longer one by a wavefront;
//   GY = Y+ Y+^T for the next iteration, Y streamed through LDS tiles.
// The q x q systems are factored by Cholesky in FP64 and inverted once per
// iteration; phase A and the wavefront columns multiply by the FP64 inverse,
// the lane columns by its FP32 rounding.
// Every reduction has a fixed order: results are bitwise reproducible.

#include <algorithm>
#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
// columns with at most this many samples take the lane-per-column path of
// the global-memory completion, longer ones a wavefront each (measured on the
// rank-32 1080p frame: 2.00 s of completion at 64 against 2.13 s at 16)
constexpr int GADM_LIGHT = 64;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <int Q>
struct AdmShared {
    double A[Q * Q];      // Gram + shift, factored in place (lower)
    double Z[Q * Q];      // L^-1
    double Inv[Q * Q];    // (G + shift)^-1
    double F[Q * Q];      // X side: G Inv ; Y side: transpose of Inv C
    float G[Q * Q];       // current Gram (FP32)
    float C[Q * Q];       // X+^T X (C[a][b] = sum x+_a x_b)
    double red[32];
};

// LDS written by some lanes of a wavefront and then read by others: the
// wavefront's LDS operations complete, and the compiler keeps them in order
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// threadIdx.x behind an empty asm statement: what is derived from it is
// recomputed where it is used, not hoisted out of the iteration loop or
// shared between phases, where it would hold registers through every phase
__device__ __forceinline__ int fresh_tid() {
    int x = threadIdx.x;
    asm volatile("" : "+v"(x));
    return x;
}

// (G + shift I)^-1 in FP64 by Cholesky; result in sh.Inv.  All threads call.
template <int Q>
__device__ void spd_inverse(AdmShared<Q> &sh, double shift) {
    const int t = fresh_tid();
    for (int e = t; e < Q * Q; e += blockDim.x) {
        const int a = e / Q, b = e % Q;
        sh.A[e] = (double)sh.G[e] + (a == b ? shift : 0.0);
        sh.Z[e] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < Q; ++j) {          // right-looking Cholesky, lower triangle
        if (t == 0) sh.A[j * Q + j] = sqrt(sh.A[j * Q + j]);
        __syncthreads();
        const double djj = sh.A[j * Q + j];
        for (int i = j + 1 + t; i < Q; i += blockDim.x) sh.A[i * Q + j] /= djj;
        __syncthreads();
        for (int e = t; e < Q * Q; e += blockDim.x) {
            const int i = e / Q, k = e % Q;
            if (k > j && i >= k) sh.A[i * Q + k] -= sh.A[i * Q + j] * sh.A[k * Q + j];
        }
        __syncthreads();
    }
    if (t < Q) {                            // column t of L^-1 by forward substitution
        const int j = t;
        for (int i = j; i < Q; ++i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int l = j; l < i; ++l) s -= sh.A[i * Q + l] * sh.Z[l * Q + j];
            sh.Z[i * Q + j] = s / sh.A[i * Q + i];
        }
    }
    __syncthreads();
    for (int e = t; e < Q * Q; e += blockDim.x) {   // Inv = Z^T Z
        const int a = e / Q, b = e % Q;
        const int lo = a > b ? a : b;
        double s = 0.0;
        for (int i = lo; i < Q; ++i) s += sh.Z[i * Q + a] * sh.Z[i * Q + b];
        sh.Inv[e] = s;
    }
    __syncthreads();
}

// The same q x q system and F from it on one wavefront, with no workgroup
// barrier: the caller runs it on a wavefront of its own while the others
// work on what does not need Inv or F, and orders it with the workgroup's
// next barrier.  Cholesky with the reciprocal of each pivot, L^-1 by forward
// substitution, Inv = L^-T L^-1; XSIDE: F = G Inv, else F[b][a] = (Inv C)[a][b].
template <int Q, bool XSIDE>
__device__ void spd_solve_wave(AdmShared<Q> &sh, double shift, int lane) {
    for (int e = lane; e < Q * Q; e += WAVE) {
        const int a = e / Q, b = e % Q;
        sh.A[e] = (double)sh.G[e] + (a == b ? shift : 0.0);
    }
    wave_lds_sync();
    for (int j = 0; j < Q; ++j) {
        const double djj = sqrt(sh.A[j * Q + j]);
        const double rj = 1.0 / djj;
        for (int e = lane; e < Q * Q; e += WAVE) {
            const int i = e / Q, k = e % Q;
            if (k > j && i >= k) sh.A[e] -= (sh.A[i * Q + j] * rj) * (sh.A[k * Q + j] * rj);
        }
        wave_lds_sync();
        for (int i = j + 1 + lane; i < Q; i += WAVE) sh.A[i * Q + j] *= rj;
        if (lane == 0) sh.A[j * Q + j] = djj;
        wave_lds_sync();
    }
    for (int i = lane; i < Q; i += WAVE) sh.Z[i * Q + i] = 1.0 / sh.A[i * Q + i];   // reciprocal pivots
    wave_lds_sync();
    if (lane < Q) {                             // column lane of L^-1
        const int j = lane;
        for (int i = j + 1; i < Q; ++i) {
            double s = 0.0;
            for (int l = j; l < i; ++l) s -= sh.A[i * Q + l] * sh.Z[l * Q + j];
            sh.Z[i * Q + j] = s * sh.Z[i * Q + i];
        }
    }
    wave_lds_sync();
    for (int e = lane; e < Q * Q; e += WAVE) {  // Inv = Z^T Z
        const int a = e / Q, b = e % Q;
        const int lo = a > b ? a : b;
        double s = 0.0;
        for (int i = lo; i < Q; ++i) s += sh.Z[i * Q + a] * sh.Z[i * Q + b];
        sh.Inv[e] = s;
    }
    wave_lds_sync();
    for (int e = lane; e < Q * Q; e += WAVE) {
        const int a = e / Q, b = e % Q;
        double v = 0.0;
        if (XSIDE) {
            for (int l = 0; l < Q; ++l) v += (double)sh.G[a * Q + l] * sh.Inv[l * Q + b];
            sh.F[e] = v;
        } else {
            for (int l = 0; l < Q; ++l) v += sh.Inv[a * Q + l] * (double)sh.C[l * Q + b];
            sh.F[b * Q + a] = v;
        }
    }
}

// Gram G = M^T M of a (rows x Q) FP32 matrix into sh.G.  The rows stream
// through LDS in tiles of GRAM_STAGE floats (coalesced float4 loads, the next
// tile in flight while the current one is used); a thread owns a 4 x 4 block
// of G and every groups-th row of a tile.  The groups' partial blocks are then
// summed in group order, so the result does not depend on timing.  part holds
// PCAP floats.
constexpr int GRAM_STAGE = 16384;

template <int Q, int PCAP, int THREADS>
__device__ void gram_rows(AdmShared<Q> &sh, const float *__restrict__ M, int rows, float *part, float *stage) {
    constexpr int P = Q * Q, QB = Q / 4, NB = QB * QB;
    constexpr int TR = GRAM_STAGE / Q;                  // rows per tile
    constexpr int NL = GRAM_STAGE / 4 / THREADS;        // float4 per thread per tile
    static_assert(NL >= 1 && NL * 4 * THREADS == GRAM_STAGE, "tile split");
    const int t = fresh_tid();
    const int groups = min(THREADS / NB, PCAP / P);
    const int g = t / NB, blk = t % NB;
    const int a0 = 4 * (blk / QB), b0 = 4 * (blk % QB);
    const float4 *M4 = reinterpret_cast<const float4 *>(M);
    const int64_t tot4 = (int64_t)rows * (Q / 4);
    const int ntiles = (rows + TR - 1) / TR;
    float4 buf[NL];
    auto load = [&](int tile) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int64_t idx = (int64_t)tile * (GRAM_STAGE / 4) + u * THREADS + t;
            buf[u] = idx < tot4 ? M4[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    float acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.f;
    if (ntiles > 0) load(0);
    float4 *stage4 = reinterpret_cast<float4 *>(stage);
    for (int tile = 0; tile < ntiles; ++tile) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NL; ++u) stage4[u * THREADS + t] = buf[u];
        __syncthreads();
        if (tile + 1 < ntiles) load(tile + 1);
        const int rt = min(TR, rows - tile * TR);
        if (g < groups) {
            for (int r = g; r < rt; r += groups) {
                const float4 u = stage4[(r * Q + a0) / 4];
                const float4 v = stage4[(r * Q + b0) / 4];
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
        sh.G[e] = v;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Completion of the slices whose X does not fit in LDS (rank 32, or tall
// slices), with X and Y in global memory, as a sequence of launches per
// iteration over all such slices of a rank bucket, so that every phase has
// the whole GPU and the launch boundaries order the phases (no workgroup
// waits for another):
//   init    (workgroup per slice)  scale, initial factors, GY, X system
//   rows    (per 64-row block)     residuals of the row's samples, R_i Y^T,
//                                  X+_i = X_i F + T_i Inv, U, Lambda (a wavefront per row)
//   ysys    (workgroup per slice)  residual norm and the stop test, GX = X+^T X+,
//                                  C = X+^T X, Y system
//   cols    (per 256-column block) residuals again from X and Y, X+^T R_j,
//                                  Y+_j = F Y_j + Inv T_j, V, Pi (a lane per light
//                                  column, a wavefront per heavy one)
//   xsys    (workgroup per slice)  GY = Y+^T Y+, X system for the next iteration
//   final   (workgroup per slice)  the final X into the X region, statistics
// The two X buffers alternate by iteration parity.  The q x q systems (FP64,
// with FP32 copies for the light columns) and the slice's stop state live in
// GADM_SYS_BYTES per slice.  The arithmetic per row and per column is that of
// a single-workgroup completion; the Grams are sums in a fixed order.

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
    double *F, *Inv;                     // Q x Q (X side: F = G Inv; Y side: F stored transposed)
    float *Ff, *If;                      // Y side, FP32: Ff[a][b] = (Inv C)[a][b], If = Inv
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
    constexpr int HALF = GRAM_STAGE / 2;
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
    __shared__ __align__(16) float stage[GRAM_STAGE];
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


    gram_rows<Q, PCAP, THREADS>(sh, Y, 3 * n, part, stage);
    gadm_x_system<Q, THREADS>(sh, g, (double)a.alpha0 * (3.0 * n) / qr);
    (void)wave;
    (void)lane;
    (void)inv_s0;
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_rows(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    __shared__ double shF[Q * Q], shInv[Q * Q];
    __shared__ __align__(16) float stage[NW * 33 * Q];
    const int b = blockIdx.x;
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
    struct {
        double *F, *Inv;
    } sh = {shF, shInv};
    const bool nonneg = (a.mode & 4) == 0;
    const double s0 = g.dstate[1];
    const float inv_s0 = (float)(1.0 / s0);
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
    __syncthreads();
    float *wsa = stage + wave * (33 * Q);   // [32][q] partial rows, then T_i (q)
    double e2 = 0.0;
        for (int i = r_beg + wave; i < r_end; i += NW) {
            float xi[Q];
            const float4 *xr = reinterpret_cast<const float4 *>(X + (size_t)i * Q);
#pragma unroll
            for (int k = 0; k < Q; k += 4) {
                const float4 u = xr[k / 4];
                xi[k] = u.x; xi[k + 1] = u.y; xi[k + 2] = u.z; xi[k + 3] = u.w;
            }
            float acc[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) acc[k] = 0.f;
            const int beg = row_ptr[i], end = row_ptr[i + 1];
            for (int p = beg + lane; p < end; p += WAVE) {
                const int j = csr_col[p];
                const float m0 = csr_val[3 * p] * inv_s0;
                const float m1 = csr_val[3 * p + 1] * inv_s0;
                const float m2 = csr_val[3 * p + 2] * inv_s0;
                const float *yj = Y + (size_t)j * 3 * Q;
                float y0[Q], y1[Q], y2[Q];
#pragma unroll
                for (int k = 0; k < Q; k += 4) {
                    const float4 a = *(const float4 *)(yj + k);
                    const float4 b = *(const float4 *)(yj + Q + k);
                    const float4 c = *(const float4 *)(yj + 2 * Q + k);
                    y0[k] = a.x; y0[k + 1] = a.y; y0[k + 2] = a.z; y0[k + 3] = a.w;
                    y1[k] = b.x; y1[k + 1] = b.y; y1[k + 2] = b.z; y1[k + 3] = b.w;
                    y2[k] = c.x; y2[k + 1] = c.y; y2[k + 2] = c.z; y2[k + 3] = c.w;
                }
                float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    d0 = fmaf(xi[k], y0[k], d0);
                    d1 = fmaf(xi[k], y1[k], d1);
                    d2 = fmaf(xi[k], y2[k], d2);
                }
                const float r0 = m0 - d0, r1 = m1 - d1, r2 = m2 - d2;
                e2 += (double)(r0 * r0) + (double)(r1 * r1) + (double)(r2 * r2);
#pragma unroll
                for (int k = 0; k < Q; ++k) acc[k] = fmaf(r0, y0[k], fmaf(r1, y1[k], fmaf(r2, y2[k], acc[k])));
            }
            // R_i Y^T: lanes 32..63 folded onto 0..31, the 32 partial rows
            // transposed through the wavefront's LDS area, lane k summing element k
#pragma unroll
            for (int k = 0; k < Q; ++k) acc[k] += __shfl_xor(acc[k], 32, WAVE);
            if (lane < 32) {
                float4 *row = reinterpret_cast<float4 *>(wsa + lane * Q);
#pragma unroll
                for (int k = 0; k < Q; k += 4) row[k / 4] = make_float4(acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
            }
            wave_lds_sync();
            // X+_i (lane k < Q owns column k): T_k = (R_i Y^T)_k + a U_ik - L_ik staged
            // for the wavefront, then U and Lambda updates
            float lam = 0.f;
            if (lane < Q) {
                float sum = 0.f;
                for (int r = 0; r < 32; ++r) sum += wsa[r * Q + lane];
                lam = Lam[(size_t)i * Q + lane];
                wsa[32 * Q + lane] = sum + alpha_f * Xp[(size_t)i * Q + lane] - lam;
            }
            wave_lds_sync();
            float xn = 0.f;
            if (lane < Q) {
                const int k = lane;
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < Q; ++l)
                    v += (double)xi[l] * sh.F[l * Q + k] + (double)wsa[32 * Q + l] * sh.Inv[l * Q + k];
                xn = (float)v;
                const float u = nonneg ? fmaxf(0.f, xn + lam * inv_alpha) : xn + lam * inv_alpha;
                Xn[(size_t)i * Q + k] = xn;
                Xp[(size_t)i * Q + k] = u;
                Lam[(size_t)i * Q + k] = lam + ga * (xn - u);
            }
            // the next row's partial rows overwrite this area
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
    __shared__ __align__(16) float stage[GRAM_STAGE];
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
    gram_rows<Q, PCAP, THREADS>(sh, Xn, m, part, stage);
    gram_cross<Q, PCAP, THREADS>(sh, Xn, X, m, part, stage);
    const double beta = (double)a.beta0 * (double)m / qr;
    spd_inverse<Q>(sh, beta);
    for (int e = t; e < Q * Q; e += THREADS) {
        const int aa = e / Q, bb = e % Q;   // F[a][b] = sum_l Inv[a][l] C[l][b]; F^T at [b][a]
        double v = 0.0;
        for (int l = 0; l < Q; ++l) v += sh.Inv[aa * Q + l] * (double)sh.C[l * Q + bb];
        g.F[bb * Q + aa] = v;
        g.Inv[e] = sh.Inv[e];
        g.Ff[e] = (float)v;
        g.If[e] = (float)sh.Inv[e];
    }
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_cols(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    __shared__ double shF[Q * Q], shInv[Q * Q];
    __shared__ __align__(16) float Ff[Q * Q];
    __shared__ __align__(16) float If[Q * Q];
    __shared__ __align__(16) float stage[NW * 33 * 3 * Q];
    const int b = blockIdx.x;
    const int k = block_slice(a.colp, a.count, b);
    const int s = __builtin_amdgcn_readfirstlane(a.ids[k]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const int m = d.m, n = d.n, qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    const int c_beg = (b - a.colp[k]) * GADM_CB, c_end = min(n, c_beg + GADM_CB);
    for (int e = t; e < Q * Q; e += THREADS) {
        shF[e] = g.F[e];
        shInv[e] = g.Inv[e];
        Ff[e] = g.Ff[e];
        If[e] = g.If[e];
    }
    struct {
        double *F, *Inv;
    } sh = {shF, shInv};
    const bool nonneg = (a.mode & 4) == 0;
    const double s0 = g.dstate[1];
    const float inv_s0 = (float)(1.0 / s0);
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
    __syncthreads();
        // ---- phase B, light columns (at most GADM_LIGHT samples): lane per column ----
        // X+^T R_j over the column's samples, then per channel Y+_j = F Y_j + Inv T_j
        // with the FP32 copies of the system
        {
            const int j = c_beg + fresh_tid();
            int beg = 0, end = 0;
            if (j < c_end) {
                beg = col_ptr[j];
                end = col_ptr[j + 1];
            }
            if (j < c_end && end - beg <= GADM_LIGHT) {
                // an opaque zero offset keeps the system's LDS reads inside the loop
                // (hoisted, 2 Q^2 values would stay in registers)
                int z = 0;
                asm volatile("" : "+v"(z));
                float y[3][Q], acc[3][Q];
                const float4 *yj = reinterpret_cast<const float4 *>(Y + (size_t)j * 3 * Q);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < Q; k += 4) {
                        const float4 u = yj[(c * Q + k) / 4];
                        y[c][k] = u.x;
                        y[c][k + 1] = u.y;
                        y[c][k + 2] = u.z;
                        y[c][k + 3] = u.w;
                        acc[c][k] = acc[c][k + 1] = acc[c][k + 2] = acc[c][k + 3] = 0.f;
                    }
                for (int p = beg; p < end; ++p) {
                    const int i = csc_row[p];
                    const float m0 = csc_val[3 * p] * inv_s0;
                    const float m1 = csc_val[3 * p + 1] * inv_s0;
                    const float m2 = csc_val[3 * p + 2] * inv_s0;
                    const float4 *xo = reinterpret_cast<const float4 *>(X + (size_t)i * Q);
                    const float4 *xp = reinterpret_cast<const float4 *>(Xn + (size_t)i * Q);
                    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
                    for (int k = 0; k < Q; k += 4) {
                        const float4 u = xo[k / 4];
                        const float xa[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            d0 = fmaf(xa[e], y[0][k + e], d0);
                            d1 = fmaf(xa[e], y[1][k + e], d1);
                            d2 = fmaf(xa[e], y[2][k + e], d2);
                        }
                    }
                    const float r0 = m0 - d0, r1 = m1 - d1, r2 = m2 - d2;
#pragma unroll
                    for (int k = 0; k < Q; k += 4) {
                        const float4 v = xp[k / 4];
                        const float xb[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            acc[0][k + e] = fmaf(xb[e], r0, acc[0][k + e]);
                            acc[1][k + e] = fmaf(xb[e], r1, acc[1][k + e]);
                            acc[2][k + e] = fmaf(xb[e], r2, acc[2][k + e]);
                        }
                    }
                }
                float4 *ypj = reinterpret_cast<float4 *>(Yp + (size_t)j * 3 * Q);
                float4 *pij = reinterpret_cast<float4 *>(Pi + (size_t)j * 3 * Q);
                float4 *yw = reinterpret_cast<float4 *>(Y + (size_t)j * 3 * Q);
                // T_j = X+^T R_j + b V_j - P_j in place of the sums
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int l = 0; l < Q; l += 4) {
                        const float4 v = ypj[(c * Q + l) / 4], pp = pij[(c * Q + l) / 4];
                        acc[c][l] = acc[c][l] + beta_f * v.x - pp.x;
                        acc[c][l + 1] = acc[c][l + 1] + beta_f * v.y - pp.y;
                        acc[c][l + 2] = acc[c][l + 2] + beta_f * v.z - pp.z;
                        acc[c][l + 3] = acc[c][l + 3] + beta_f * v.w - pp.w;
                    }
                // outputs k..k+3 of the three channels; every read of Yp and P is
                // above, so they are stored at once
#pragma unroll 1
                for (int k = 0; k < Q; k += 4) {
                    float o[3][4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const float4 *fk = reinterpret_cast<const float4 *>(Ff + z + (k + kk) * Q);
                        const float4 *ik = reinterpret_cast<const float4 *>(If + z + (k + kk) * Q);
                        float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll
                        for (int l = 0; l < Q; l += 4) {
                            const float4 f = fk[l / 4], g = ik[l / 4];
                            const float fa[4] = {f.x, f.y, f.z, f.w}, ga[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                v0 = fmaf(fa[e], y[0][l + e], fmaf(ga[e], acc[0][l + e], v0));
                                v1 = fmaf(fa[e], y[1][l + e], fmaf(ga[e], acc[1][l + e], v1));
                                v2 = fmaf(fa[e], y[2][l + e], fmaf(ga[e], acc[2][l + e], v2));
                            }
                        }
                        o[0][kk] = v0;
                        o[1][kk] = v1;
                        o[2][kk] = v2;
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int w = (c * Q + k) / 4;
                        const float4 pv = pij[w];
                        const float pa[4] = {pv.x, pv.y, pv.z, pv.w};
                        float un[4], pn[4];
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            un[kk] = nonneg ? fmaxf(0.f, o[c][kk] + pa[kk] * inv_beta) : o[c][kk] + pa[kk] * inv_beta;
                            pn[kk] = pa[kk] + gb * (o[c][kk] - un[kk]);
                        }
                        ypj[w] = make_float4(un[0], un[1], un[2], un[3]);
                        pij[w] = make_float4(pn[0], pn[1], pn[2], pn[3]);
                        yw[w] = make_float4(o[c][0], o[c][1], o[c][2], o[c][3]);
                    }
                }
            }
        }

        // ---- phase B, heavy columns: wavefront per column ----
        float *wst = stage + wave * (33 * 3 * Q);   // [32][3q] partial rows, then T_j (3q)
        for (int jb = c_beg + wave * WAVE; jb < c_end; jb += NW * WAVE) {
            const int jl = jb + lane;
            const int cnt = jl < c_end ? col_ptr[jl + 1] - col_ptr[jl] : 0;
            uint64_t heavy = __ballot(cnt > GADM_LIGHT);
            while (heavy) {
                const int j = jb + __builtin_ctzll(heavy);
                heavy &= heavy - 1;
                float y0[Q], y1[Q], y2[Q];
                const float4 *yj = reinterpret_cast<const float4 *>(Y + (size_t)j * 3 * Q);
#pragma unroll
                for (int k = 0; k < Q; k += 4) {
                    const float4 u = yj[k / 4], v = yj[(Q + k) / 4], w = yj[(2 * Q + k) / 4];
                    y0[k] = u.x; y0[k + 1] = u.y; y0[k + 2] = u.z; y0[k + 3] = u.w;
                    y1[k] = v.x; y1[k + 1] = v.y; y1[k + 2] = v.z; y1[k + 3] = v.w;
                    y2[k] = w.x; y2[k + 1] = w.y; y2[k + 2] = w.z; y2[k + 3] = w.w;
                }
                float a0[Q], a1[Q], a2[Q];
#pragma unroll
                for (int k = 0; k < Q; ++k) a0[k] = a1[k] = a2[k] = 0.f;
                const int beg = col_ptr[j], end = col_ptr[j + 1];
                for (int p = beg + lane; p < end; p += WAVE) {
                    const int i = csc_row[p];
                    const float m0 = csc_val[3 * p] * inv_s0;
                    const float m1 = csc_val[3 * p + 1] * inv_s0;
                    const float m2 = csc_val[3 * p + 2] * inv_s0;
                    const float *xo = X + (size_t)i * Q;
                    const float *xp = Xn + (size_t)i * Q;
                    float xa[Q], xb[Q];
#pragma unroll
                    for (int k = 0; k < Q; k += 4) {
                        const float4 u = *(const float4 *)(xo + k);
                        const float4 v = *(const float4 *)(xp + k);
                        xa[k] = u.x; xa[k + 1] = u.y; xa[k + 2] = u.z; xa[k + 3] = u.w;
                        xb[k] = v.x; xb[k + 1] = v.y; xb[k + 2] = v.z; xb[k + 3] = v.w;
                    }
                    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        d0 = fmaf(xa[k], y0[k], d0);
                        d1 = fmaf(xa[k], y1[k], d1);
                        d2 = fmaf(xa[k], y2[k], d2);
                    }
                    const float r0 = m0 - d0, r1 = m1 - d1, r2 = m2 - d2;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        a0[k] = fmaf(xb[k], r0, a0[k]);
                        a1[k] = fmaf(xb[k], r1, a1[k]);
                        a2[k] = fmaf(xb[k], r2, a2[k]);
                    }
                }
                // X+^T R_j: lanes 32..63 folded onto 0..31, the 32 partial rows
                // transposed through the wavefront's LDS area, lane o summing element o
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    a0[k] += __shfl_xor(a0[k], 32, WAVE);
                    a1[k] += __shfl_xor(a1[k], 32, WAVE);
                    a2[k] += __shfl_xor(a2[k], 32, WAVE);
                }
                if (lane < 32) {
                    float4 *row = reinterpret_cast<float4 *>(wst + lane * 3 * Q);
#pragma unroll
                    for (int k = 0; k < Q; k += 4) {
                        row[k / 4] = make_float4(a0[k], a0[k + 1], a0[k + 2], a0[k + 3]);
                        row[(Q + k) / 4] = make_float4(a1[k], a1[k + 1], a1[k + 2], a1[k + 3]);
                        row[(2 * Q + k) / 4] = make_float4(a2[k], a2[k + 1], a2[k + 2], a2[k + 3]);
                    }
                }
                wave_lds_sync();
                // output o = (c, k), lanes o < 3q (two rounds when 3q > 64):
                // T_o = (X+^T R_j)_o + b V_o - P_o, staged for the whole wavefront
                float *ypj = Yp + (size_t)j * 3 * Q;
                float *pij = Pi + (size_t)j * 3 * Q;
                float pv[2];
#pragma unroll
                for (int rnd = 0; rnd < 2; ++rnd) {
                    const int o = lane + rnd * WAVE;
                    pv[rnd] = 0.f;
                    if (o < 3 * Q) {
                        float sum = 0.f;
                        for (int r = 0; r < 32; ++r) sum += wst[r * 3 * Q + o];
                        pv[rnd] = pij[o];
                        wst[32 * 3 * Q + o] = sum + beta_f * ypj[o] - pv[rnd];
                    }
                }
                wave_lds_sync();
                const float *tj = wst + 32 * 3 * Q;
#pragma unroll
                for (int rnd = 0; rnd < 2; ++rnd) {
                    const int o = lane + rnd * WAVE;
                    if (o < 3 * Q) {
                        const int c = o / Q, k = o % Q;
                        double v = 0.0;
#pragma unroll
                        for (int l = 0; l < Q; ++l) {
                            const float yl = c == 0 ? y0[l] : (c == 1 ? y1[l] : y2[l]);
                            v += sh.F[l * Q + k] * (double)yl + sh.Inv[l * Q + k] * (double)tj[c * Q + l];
                        }
                        const float yn = (float)v;
                        const float u = nonneg ? fmaxf(0.f, yn + pv[rnd] * inv_beta) : yn + pv[rnd] * inv_beta;
                        ypj[o] = u;
                        pij[o] = pv[rnd] + gb * (yn - u);
                        Y[(size_t)j * 3 * Q + o] = yn;
                    }
                }
                // the next column's partial rows overwrite this area
                wave_lds_sync();
            }
        }
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_gadm_xsys(GadmArgs a, int it) {
    constexpr int NW = THREADS / WAVE;
    __shared__ AdmShared<Q> sh;
    constexpr int PCAP = (NW * Q * Q > 2 * 1024) ? NW * Q * Q : 2 * 1024;
    __shared__ float part[PCAP];
    __shared__ __align__(16) float stage[GRAM_STAGE];
    const int s = __builtin_amdgcn_readfirstlane(a.ids[blockIdx.x]);
    const GSys g = gsys_of(a.gsys, s);
    if (g.state[0]) return;
    const SliceDesc d = a.desc[s];
    const float *Y = a.Y_all + d.off_y;
    gram_rows<Q, PCAP, THREADS>(sh, Y, 3 * d.n, part, stage);
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

// ---------------------------------------------------------------------------
// LDS-resident variant for ranks 4, 8, 16 (two LDS buffers of m (q + 1)
// words: X_k, and the R Y^T accumulator that then holds T and X+).  The
// samples are read from the slice's ELL copy, in which one lane walks one
// part of a column (at most ELL_LMAX samples; the parts of a 64-lane group
// have nearly equal lengths) and every load of a wavefront covers 64
// consecutive entries.
//   phase A, lane = part of column j: Y_j (3q floats) in registers, X_i from LDS;
//     the residual r is stored in the ELL copy and the q components of
//     sum_c r_c Y_j^c, times 2^S and rounded, are added into row i of a
//     fixed-point R Y^T accumulator with integer LDS atomics (LDS float
//     atomics serialise per lane on this chip).  Integer sums do not depend
//     on the order of the additions.  Word q of each row sums a ceil-rounded
//     bound of the row's L1 residual sum; the scale 2^S keeps every row sum
//     below 2^31 given that bound and |Y|max, and the phase runs again with
//     a smaller scale whenever an estimate taken from the previous iterate
//     fails, so no sum overflows.
//   X system, X update: Inv = (GY + a I)^-1 by FP64 Cholesky, T = R Y^T + a U - L,
//     then X+ = X (GY Inv) + T Inv as FP32 16 x 16 x 4 MFMA products per 16
//     rows (the FP64 factors rounded to FP32), with U, L and the Grams X+^T X+
//     and X+^T X fused on the product's output registers.
//   phase B, lane = part of column j: X+^T R over the part from the stored
//     residuals and X+ (LDS); T_j = X+^T R_j + W_j staged in global memory
//     (W = b V - P is what the Y update stores of V and P), the partial sums
//     of a column of several parts added in part order.
//   Y system, Y update: Inv = (GX + b I)^-1, Y+ = Y (Inv C)^T + T Inv as FP32
//     MFMA products per 16 rows of the 3n x q matrix, with P, W and the Gram
//     Y+^T Y+.
// Every phase issues a unit's loads before its stores: loads and stores retire
// through one in-order counter, so a load behind a store waits for the store.
// Rows of X in LDS keep their 4-float chunks rotated (xpos), which spreads the
// 128-bit reads of a wavefront over the banks.
// Per-wavefront partial Grams are summed in a fixed order through the
// slice's global scratch.  The run is reproducible bit for bit.

typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x4_f32 on one wavefront: lane l holds A[l % 16][l / 16] of
// the 16 x 4 left operand and B[l / 16][l % 16] of the 4 x 16 right one;
// register v of lane l of the result holds D[4 (l / 16) + v][l % 16].
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

// a value every lane holds alike, moved to scalar registers
__device__ __forceinline__ float uni(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uni(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// block-wide maximum of per-thread values; every thread calls it and gets the result
__device__ __forceinline__ float block_max(float v, float *red) {
    const int t = fresh_tid(), nw = blockDim.x / WAVE, lane = t % WAVE, w = t / WAVE;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    float r = red[0];
    for (int k = 1; k < nw; ++k) r = fmaxf(r, red[k]);
    __syncthreads();
    return uni(r);
}

// Sum over the wavefronts of two per-wavefront 16 x 16 partials (result
// layout of mfma16) in wavefront order, through global scratch `red`; the
// q x q corners land in out0 and out1 (out1 may be null).  All threads call.
template <int Q, int NW>
__device__ void sum_partials(const f4 &p0, const f4 &p1, float *red, float *out0, float *out1) {
    const int t = fresh_tid(), lane = t % WAVE, w = t / WAVE;
    const int rr = 4 * (lane / 16), cc = lane % 16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        red[(2 * w) * 256 + (rr + v) * 16 + cc] = p0[v];
        red[(2 * w + 1) * 256 + (rr + v) * 16 + cc] = p1[v];
    }
    __threadfence_block();
    __syncthreads();
    if (t < 2 * Q * Q) {
        const int which = t / (Q * Q), e = t % (Q * Q), a = e / Q, b = e % Q;
        float sum = 0.f;
        for (int k = 0; k < NW; ++k) sum += red[(2 * k + which) * 256 + a * 16 + b];
        if (which == 0) out0[e] = sum;
        else if (out1) out1[e] = sum;
    }
    __syncthreads();
}

// Word of X(i, k) in an LDS buffer of X: row i at i q, its 4-float chunks
// rotated by (i q) / 64, so that the 128-bit row reads of a wavefront (lanes
// with unrelated rows, same chunk) start on all 16 bank quadruples.
template <int Q>
__device__ __forceinline__ int xpos(int i, int k) {
    return i * Q + ((((k >> 2) + ((i * Q) >> 6)) % (Q / 4)) << 2) + (k & 3);
}
// the 16-byte chunk c of row i
template <int Q>
__device__ __forceinline__ const float4 *xchunk(const float *X, int i, int c) {
    return reinterpret_cast<const float4 *>(X + i * Q + (((c + ((i * Q) >> 6)) % (Q / 4)) << 2));
}
template <int Q>
__device__ __forceinline__ float4 *xchunk_w(float *X, int i, int c) {
    return reinterpret_cast<float4 *>(X + i * Q + (((c + ((i * Q) >> 6)) % (Q / 4)) << 2));
}

// elements of the fixed-point to float pass (m q <= ADM_CVT_ELEMS)
constexpr int ADM_CVT_ELEMS = 18 * 1024;
// ELL entries a lane loads at once in phase A (one more block of them in
// flight while a block is processed) and in phase B
constexpr int ADM_DA = 2;
constexpr int ADM_DB = 8;
// split-column sums a thread gathers before it stores them
constexpr int ADM_CMB = 4;

template <int Q, int THREADS>
__device__ void adm_ell_slice(
    int s, const SliceDesc *__restrict__ desc, uint64_t seed, int32_t max_iter,
    int32_t fixed_iters, float tol, float alpha0, float beta0, float gamma, const int32_t *__restrict__ col_ptr_all,
    EllView ell, float *X_all,
    float *Xp_all, float *Lam_all, float *Y_all, float *Yp_all, float *Pi_all, float *Yt_all, float *red_all,
    double *e2part_all, float *scale_all, int32_t *stats_all) {
    static_assert(Q % 4 == 0 && Q <= 16, "ranks 4, 8, 16");
    constexpr int NW = THREADS / WAVE;
    constexpr int QV = Q / 4;                         // MFMA steps over the rank
    extern __shared__ __align__(16) float dyn[];
    __shared__ AdmShared<Q> sh;
    __shared__ float redf[NW];

    const SliceDesc d = desc[s];
    const int m = d.m, n = d.n;
    // the slice's own rank qr <= Q: components qr .. Q-1 of X, Y and their
    // multipliers start at 0 and stay exactly 0 (their Gram block is alpha I
    // or beta I and every cross term is 0), so a rank-qr completion runs in
    // the rank-Q kernel
    const int qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    float *XA = dyn;                                  // X_k, row stride q
    float *XB = dyn + (size_t)m * (Q + 1);            // fixed-point R Y^T (stride q + 1); X+ replaces X in XA

    const int32_t *col_ptr = col_ptr_all + d.off_colptr;
    const int2 *part = ell.part + d.off_part;
    const int32_t *pbase = ell.pbase + d.off_colptr;
    const int32_t *grp = ell.grp + d.off_grp;
    float *partial = ell.partial + 48 * d.off_part;
    const uint16_t *erow = ell.row + d.off_ell;
    const float *eval = ell.val + 3 * d.off_ell;
    float *eres = ell.res + 3 * d.off_ell;
    float *Xg = X_all + d.off_x;
    float *Xp = Xp_all + d.off_x;
    float *Lam = Lam_all + d.off_x;
    float *Y = Y_all + d.off_y;
    float *W = Yp_all + d.off_y;          // W = b V - P: all that phase B needs of V and P
    float *Pi = Pi_all + d.off_y;
    float *Yt = Yt_all + d.off_y;
    float *red = red_all + d.off_red;
    double *e2part = e2part_all + 2 * d.off_part;   // per part: the two halves' sums
    int32_t *st = stats_all + 4 * s;
    const int nnz = col_ptr[n];
    const int P = pbase[n];               // parts
    const int G = (P + 63) / 64;          // groups of 64 parts
    const bool halves = G < NW - 1;       // phase A: two wavefronts per group
    const int R3 = 3 * n;

    // the slice's samples in the ELL copy: entries k < length of the part at
    // sorted position 64 g + lane lie at grp[g] + 64 k + lane
    auto for_each_entry = [&](auto &&f) {
        for (int g = wave; g < G; g += NW) {
            const int sp = 64 * g + lane;
            const int cl = sp < P ? (part[sp].x >> 16) & 0x7F : 0;
            const int base = grp[g];
            for (int k = 0; k < cl; ++k) f(base + 64 * k + lane);
        }
    };

    // ---- scale s0 = mean sampled value; ||P_Omega M|| ----
    double sum = 0.0, sumsq = 0.0;
    for_each_entry([&](int e) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = (double)eval[3 * e + c];
            sum += v;
            sumsq += v * v;
        }
    });
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
    tot = uni(tot);
    totsq = uni(totsq);
    __syncthreads();
    if (!(nnz > 0 && tot > 0.0)) {
        for (int e = t; e < m * Q; e += THREADS) Xg[e] = 0.f;
        for (int e = t; e < 3 * n * Q; e += THREADS) Y[e] = 0.f;
        if (t == 0) {
            scale_all[s] = 0.f;
            st[0] = 0;
            st[1] |= VPLMC_SLICE_ALL_ZERO;
            st[2] = __float_as_int(0.f);
        }
        return;
    }
    const double s0 = tot / (3.0 * (double)nnz);
    const float inv_s0 = (float)(1.0 / s0);
    const double normM = sqrt(totsq) / s0;
    if (t == 0) scale_all[s] = (float)s0;

    // ---- initial factors: fp32(u24(Philox) * fp32(2 / sqrt q)), or (mode bit 1)
    // the contents of the X and Y regions ----
    const float cq = (float)(2.0 / sqrt((double)qr));
    const bool given = (fixed_iters & 2) != 0;
    const bool nonneg = (fixed_iters & 4) == 0;    // mode bit 2: projections off
    for (int e = t; e < m * Q; e += THREADS) {
        const int i = e / Q, k = e % Q;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)i, (uint64_t)k, TAG_INITX, 0);
        const float v = k < qr ? (given ? Xg[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
        XA[xpos<Q>(i, k)] = v;
        Xp[e] = v;
        Lam[e] = 0.f;
    }
    float ym0 = 0.f;
    const float beta0_f = (float)((double)beta0 * (double)m / qr);
    for (int e = t; e < 3 * n * Q; e += THREADS) {
        const int j = e / (3 * Q), c = (e / Q) % 3, k = e % Q;
        const uint64_t col = (uint64_t)c * (uint64_t)n + (uint64_t)j;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)k, col, TAG_INITY, 0);
        const float v = k < qr ? (given ? Y[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
        Y[e] = v;
        W[e] = __fmul_rn(beta0_f, v);                 // b V_0 - P_0 with V_0 = Y_0, P_0 = 0
        Pi[e] = 0.f;
        ym0 = fmaxf(ym0, v);
    }
    __threadfence_block();
    __syncthreads();

    // ---- GY = Y0^T Y0 ----
    {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        const f4 zero = {0.f, 0.f, 0.f, 0.f};
        for (int r0 = 4 * wave; r0 < R3; r0 += 4 * NW) {
            const int r = r0 + lane / 16, c = lane % 16;
            const float v = (r < R3 && c < Q) ? Y[(size_t)r * Q + c] : 0.f;
            acc = mfma16(v, v, acc);
        }
        sum_partials<Q, NW>(acc, zero, red, sh.G, nullptr);
    }

    // ---- bounds for the fixed-point scale: K, the largest sum_c |M| of a
    // sample, the largest row 1-norm of X_0 ----
    int32_t *cntr = reinterpret_cast<int32_t *>(XB);
    for (int e = t; e < m; e += THREADS) cntr[e] = 0;
    __syncthreads();
    float msum = 0.f;
    for_each_entry([&](int e) {
        atomicAdd(cntr + erow[e], 1);
        msum = fmaxf(msum, fabsf(eval[3 * e]) + fabsf(eval[3 * e + 1]) + fabsf(eval[3 * e + 2]));
    });
    __syncthreads();
    float kmx = 0.f, x1 = 0.f;
    for (int i = t; i < m; i += THREADS) {
        kmx = fmaxf(kmx, (float)cntr[i]);
        float a = 0.f;
        for (int k = 0; k < Q; ++k) a += fabsf(XA[i * Q + k]);
        x1 = fmaxf(x1, a);
    }
    const double Krow = (double)block_max(kmx, redf);
    const double msum_max = (double)block_max(msum, redf) * (double)inv_s0;
    const double x1max = (double)block_max(x1, redf);
    double ymax = (double)block_max(ym0, redf);
    // Two fixed-point scales per iteration.  Word q of each accumulator row
    // sums ceil(2^Sr sum_c |r_c|) over the row's samples (an upper bound of
    // the row's L1 residual sum RS_i); words 0..q-1 sum round(2^S c_k) with
    // |c_k| <= sum_c |r_c| |Y|max.  Row sums fit in 32 bits when
    //   K (rs 2^Sr + 1) < 2^32 - 1      (rs = the largest sum_c |r_c|)
    //   RS |Y|max 2^S + K / 2 < 2^31 - 1 (RS = the largest RS_i),
    // the integer sums being exact modulo 2^32.  Estimates come from the
    // previous iterate (x2); phase A runs again if a bound fails.
    double rs_est = (msum_max + 3.0 * x1max * ymax) * (1.0 + 1e-5);   // a-priori bound for the first iterate
    double RS_est = Krow * rs_est;
    auto pow2_below = [](double lim, double b) {       // largest S in [-60, 60] with b 2^S <= lim
        // start one above floor(log2(lim / b)), read off the exponent bits
        // (no log2 call: its temporaries cost registers this kernel lacks)
        const double qt = lim / b;
        int S = b > 0.0 && qt < 1e300 ? (int)((__double_as_longlong(qt) >> 52) & 0x7FF) - 1023 + 1 : 60;
        S = S > 60 ? 60 : (S < -60 ? -60 : S);
        while (S > -60 && b * ldexp(1.0, S) > lim) --S;
        return S;
    };
    auto rs_fits = [&](int Sr, double rs) { return Krow * (rs * ldexp(1.0, Sr) + 1.0) < 4294967295.0; };
    auto rx_fits = [&](int S, double RS) {   // 1e-5: FP32 rounding of the contributions
        return RS * ymax * ldexp(1.0, S) * (1.0 + 1e-5) + 0.5 * Krow < 2147483647.0;
    };

    // uniform constants, kept in scalar registers
    const double alpha = uni((double)alpha0 * (3.0 * n) / qr);
    const double beta = uni((double)beta0 * (double)m / qr);
    const float alpha_f = uni((float)alpha), beta_f = uni((float)beta);
    const float ga = uni((float)((double)gamma * alpha)), gb = uni((float)((double)gamma * beta));
    const float inv_alpha = uni((float)(1.0 / alpha)), inv_beta = uni((float)(1.0 / beta));
    int iters = max_iter;
    double err = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        // a fresh thread index in every phase (fresh_tid)
        int t = fresh_tid(), lane = t % WAVE;
        // lane's part in group g (sorted position 64 g + lane): column j, its
        // length cnt, its number pc in column order, np = 1 for a column of one
        // part and 2 for a column of several
        auto part_of = [&](int g, int &j, int &cnt, int &pc, int &np) {
            const int sp = 64 * g + lane;
            j = 0;
            cnt = 0;
            pc = 0;
            np = 1;
            if (sp < P) {                    // one load: everything was packed by the part sort
                const int2 v = part[sp];
                j = v.x & 0xFFFF;
                cnt = (v.x >> 16) & 0x7F;
                np = (v.x >> 23) & 1 ? 2 : 1;
                pc = v.y;
            }
        };
        // right-hand operands of the dense updates: F[l][k] and Inv[l][k] (FP64),
        // zero outside q x q; lane holds row 4 v + lane / 16, column lane % 16
        auto load_rhs = [&](float *b1, float *b2) {
            const int c = lane % 16;
#pragma unroll
            for (int v = 0; v < QV; ++v) {
                const int l = 4 * v + lane / 16;
                b1[v] = c < Q ? (float)sh.F[l * Q + c] : 0.f;
                b2[v] = c < Q ? (float)sh.Inv[l * Q + c] : 0.f;
            }
        };
        // the same with the contraction index of MFMA step v at lane row
        // lane / 16 taken as QV (lane / 16) + v, so that a lane's operand
        // values of one row are contiguous
        auto load_rhs_c = [&](float *b1, float *b2) {
            const int c = lane % 16;
#pragma unroll
            for (int v = 0; v < QV; ++v) {
                const int l = QV * (lane / 16) + v;
                b1[v] = c < Q ? (float)sh.F[l * Q + c] : 0.f;
                b2[v] = c < Q ? (float)sh.Inv[l * Q + c] : 0.f;
            }
        };
        // ---- phase A: residuals, 2^S R Y^T into XB ----
        int32_t *RXI = reinterpret_cast<int32_t *>(XB);
        int Sr = pow2_below(2147483648.0, Krow * rs_est);
        int S = pow2_below(1073741824.0, RS_est * ymax);
        double e2t = 0.0, RSc = 0.0;
        float rsc = 0.f;
        bool xsys = false;
        for (;;) {
            const float fxs = ldexpf(1.f, S), fxr = ldexpf(1.f, Sr);
            for (int e = t; e < m * (Q + 1); e += THREADS) RXI[e] = 0;
            __syncthreads();
            float rsm = 0.f;
            // the last wavefront solves the X system (Inv, F for the X update),
            // which needs only GY, while the others take the parts
            if (wave == NW - 1) {
                if (!xsys) {
                    spd_solve_wave<Q, true>(sh, alpha, lane);
                    xsys = true;
                }
            } else {
            // with fewer part groups than working wavefronts, two wavefronts
            // share a group, the first taking entries [0, kh) of every part,
            // the second [kh, length)
            const int items = halves ? 2 * G : G;
            for (int item = wave; item < items; item += NW - 1) {
                const int g = halves ? item >> 1 : item, h = halves ? item & 1 : 0;
                int j, cnt, pc, np;
                part_of(g, j, cnt, pc, np);
                const int base = grp[g];
                const int len = (grp[g + 1] - base) >> 6;
                const int kh = halves ? (len + 2 * ADM_DA - 1) / (2 * ADM_DA) * ADM_DA : len;
                const int kb = h ? kh : 0, ke = h ? len : kh;
                const int ce = cnt < ke ? cnt : ke;          // the lane's entries: [kb, ce)
                double e2 = 0.0;
                float y[3 * Q];
                const float4 *y4 = reinterpret_cast<const float4 *>(Y + (size_t)j * 3 * Q);
#pragma unroll
                for (int v = 0; v < 3 * Q / 4; ++v) {
                    const float4 a = ce > kb ? y4[v] : make_float4(0.f, 0.f, 0.f, 0.f);
                    y[4 * v] = a.x;
                    y[4 * v + 1] = a.y;
                    y[4 * v + 2] = a.z;
                    y[4 * v + 3] = a.w;
                }
                // entries k0 .. k0 + ADM_DA - 1 of the lane's part; the next block
                // is loaded before this block's residuals are stored
                auto load_block = [&](int k0, int *ib, float *mb0, float *mb1, float *mb2) {
#pragma unroll
                    for (int u = 0; u < ADM_DA; ++u) {
                        const bool act = k0 + u < ce;
                        const int e = base + 64 * (k0 + u) + lane;
                        ib[u] = act ? (int)erow[e] : -1;
                        mb0[u] = act ? eval[3 * e] : 0.f;
                        mb1[u] = act ? eval[3 * e + 1] : 0.f;
                        mb2[u] = act ? eval[3 * e + 2] : 0.f;
                    }
                };
                int ib[ADM_DA];
                float mb0[ADM_DA], mb1[ADM_DA], mb2[ADM_DA];
                if (kb < ke) load_block(kb, ib, mb0, mb1, mb2);
                for (int k0 = kb; k0 < ke; k0 += ADM_DA) {
                    int ibn[ADM_DA];
                    float mn0[ADM_DA], mn1[ADM_DA], mn2[ADM_DA];
                    if (k0 + ADM_DA < ke) load_block(k0 + ADM_DA, ibn, mn0, mn1, mn2);
#pragma unroll
                    for (int u = 0; u < ADM_DA; ++u) {
                        mb0[u] *= inv_s0;
                        mb1[u] *= inv_s0;
                        mb2[u] *= inv_s0;
                    }
#pragma unroll
                    for (int u = 0; u < ADM_DA; ++u) {
                        const int i = ib[u];
                        if (i >= 0) {
                            float x[Q];
#pragma unroll
                            for (int v = 0; v < QV; ++v) {
                                const float4 a4 = *xchunk<Q>(XA, i, v);
                                x[4 * v] = a4.x;
                                x[4 * v + 1] = a4.y;
                                x[4 * v + 2] = a4.z;
                                x[4 * v + 3] = a4.w;
                            }
                            float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
                            for (int kk = 0; kk < Q; ++kk) {
                                d0 = fmaf(x[kk], y[kk], d0);
                                d1 = fmaf(x[kk], y[Q + kk], d1);
                                d2 = fmaf(x[kk], y[2 * Q + kk], d2);
                            }
                            const float r0 = mb0[u] - d0, r1 = mb1[u] - d1, r2 = mb2[u] - d2;
                            e2 += (double)(r0 * r0) + (double)(r1 * r1) + (double)(r2 * r2);
                            const int e = base + 64 * (k0 + u) + lane;
                            eres[3 * e] = r0;
                            eres[3 * e + 1] = r1;
                            eres[3 * e + 2] = r2;
                            const float rsa = fabsf(r0) + fabsf(r1) + fabsf(r2);
                            rsm = fmaxf(rsm, rsa);
                            const float s0r = r0 * fxs, s1r = r1 * fxs, s2r = r2 * fxs;
                            int32_t *row = RXI + i * (Q + 1);
#pragma unroll
                            for (int kk = 0; kk < Q; ++kk)
                                atomicAdd(row + kk,
                                          __float2int_rn(fmaf(s0r, y[kk], fmaf(s1r, y[Q + kk], s2r * y[2 * Q + kk]))));
                            atomicAdd(reinterpret_cast<uint32_t *>(row + Q), __float2uint_ru(rsa * fxr));
                        }
                    }
#pragma unroll
                    for (int u = 0; u < ADM_DA; ++u) {
                        ib[u] = ibn[u];
                        mb0[u] = mn0[u];
                        mb1[u] = mn1[u];
                        mb2[u] = mn2[u];
                    }
                }
                if (64 * g + lane < P) e2part[2 * pc + h] = e2;
            }
            }
            // sum of the parts' squared residuals in column order (and half order)
            __threadfence_block();
            __syncthreads();
            double e2 = 0.0;
            for (int u = t; u < P; u += THREADS) e2 += halves ? e2part[2 * u] + e2part[2 * u + 1] : e2part[2 * u];
            uint32_t rsw = 0;
            for (int i = t; i < m; i += THREADS) rsw = max(rsw, reinterpret_cast<const uint32_t *>(RXI)[i * (Q + 1) + Q]);
            e2 = wave_sum_d(e2);
            rsm = wave_max(rsm);
            const float rswf = wave_max((float)rsw);
            if (lane == 0) {
                sh.red[wave] = e2;
                redf[wave] = rsm;
                sh.red[16 + wave] = (double)rswf;
            }
            __syncthreads();
            e2t = 0.0;
            rsc = 0.f;
            double rsw_max = 0.0;
            for (int w = 0; w < NW; ++w) {
                e2t += sh.red[w];
                rsc = fmaxf(rsc, redf[w]);
                rsw_max = fmax(rsw_max, sh.red[16 + w]);
            }
            e2t = uni(e2t);
            rsc = uni(rsc);
            rsw_max = uni(rsw_max);
            __syncthreads();
            // every integer sum provably fits, or the residuals are not finite
            const double rsb = (double)rsc * (1.0 + 1e-5);
            if (!(rsb < 1e300)) break;
            if (!rs_fits(Sr, rsb)) {                  // row L1 sums may have wrapped: redo with safe scales
                Sr = pow2_below(2147483648.0, Krow * rsb);
                S = pow2_below(1073741824.0, Krow * rsb * ymax);
                if (Sr <= -60) break;
                continue;
            }
            // (float) of the 32-bit word rounds by at most 2^-24 relative
            RSc = rsw_max * (1.0 + 1e-6) * ldexp(1.0, -Sr);
            if (rx_fits(S, RSc) || S <= -60) break;
            S = pow2_below(1073741824.0, RSc * ymax);
        }
        rs_est = 2.0 * (double)rsc;
        RS_est = 2.0 * RSc;
        err = sqrt(e2t) / normM;
        if (!(fixed_iters & 1) && err < (double)tol) {
            iters = it;
            break;
        }

        // (the X system was solved during phase A; the integer sums are complete)
        // ---- X+ = X F + T Inv (FP32 MFMA on FP32 copies of the FP64 q x q factors), U, L, Grams X+^T X+ and X+^T X ----
        t = fresh_tid();
        lane = t % WAVE;
        {
            // as in the Y update: operands of row lane % 16 with contiguous
            // components, the product plain (Grams) and transposed (a lane
            // writes components 4 (lane / 16) .. + 3 of one row of X+, U, L)
            const float ifx = ldexpf(1.f, -S);
            float b1[QV], b2[QV];
            load_rhs_c(b1, b2);
            f4 gx = {0.f, 0.f, 0.f, 0.f}, cx = {0.f, 0.f, 0.f, 0.f};
            for (int r0 = 16 * wave; r0 < m; r0 += 16 * NW) {
                const int ra = r0 + lane % 16;
                const bool rok = ra < m;
                const int rc = rok ? ra : m - 1;
                // operands: X (row rc) and T = 2^-S R Y^T + a U - L, formed
                // here from the integer sums (read-only in XB now)
                float a1[QV], a2[QV];
                const int kb = QV * (lane / 16);
                const int32_t *rxi = RXI + rc * (Q + 1) + kb;
                const size_t eo = (size_t)rc * Q + kb;
                const int cb = 4 * (lane / 16);
                float4 lam4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if constexpr (QV == 4) {
                    const float4 x4 = *xchunk<Q>(XA, rc, lane / 16);
                    const float4 u4 = *reinterpret_cast<const float4 *>(Xp + eo);
                    lam4 = *reinterpret_cast<const float4 *>(Lam + eo);   // kb == cb: also the update's
                    a1[0] = x4.x; a1[1] = x4.y; a1[2] = x4.z; a1[3] = x4.w;
                    a2[0] = (float)rxi[0] * ifx + (alpha_f * u4.x - lam4.x);
                    a2[1] = (float)rxi[1] * ifx + (alpha_f * u4.y - lam4.y);
                    a2[2] = (float)rxi[2] * ifx + (alpha_f * u4.z - lam4.z);
                    a2[3] = (float)rxi[3] * ifx + (alpha_f * u4.w - lam4.w);
                } else {
#pragma unroll
                    for (int v = 0; v < QV; ++v) {
                        a1[v] = XA[xpos<Q>(rc, kb + v)];
                        a2[v] = (float)rxi[v] * ifx + (alpha_f * Xp[eo + v] - Lam[eo + v]);
                    }
                    if (rok && cb < Q) lam4 = *reinterpret_cast<const float4 *>(Lam + (size_t)ra * Q + cb);
                }
                f4 D = {0.f, 0.f, 0.f, 0.f}, Dt = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int v = 0; v < QV; ++v) {
                    const float x = rok ? a1[v] : 0.f, tt = rok ? a2[v] : 0.f;
                    D = mfma16(x, b1[v], D);
                    D = mfma16(tt, b2[v], D);
                    Dt = mfma16(b1[v], x, Dt);
                    Dt = mfma16(b2[v], tt, Dt);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 4 * (lane / 16) + v, c = lane % 16;   // FP32 result layout
                    const bool ok = r < m && c < Q;
                    const float xn = ok ? D[v] : 0.f;
                    const float xk = ok ? XA[xpos<Q>(r, c)] : 0.f;
                    gx = mfma16(xn, xn, gx);
                    cx = mfma16(xn, xk, cx);
                }
                if (rok && cb < Q) {
                    const float li[4] = {lam4.x, lam4.y, lam4.z, lam4.w};
                    float uo[4], lo[4], xo[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float xn = Dt[v];
                        const float u = nonneg ? fmaxf(0.f, xn + li[v] * inv_alpha) : xn + li[v] * inv_alpha;
                        uo[v] = u;
                        lo[v] = li[v] + ga * (xn - u);
                        xo[v] = xn;
                    }
                    const size_t e = (size_t)ra * Q + cb;
                    *reinterpret_cast<float4 *>(Xp + e) = make_float4(uo[0], uo[1], uo[2], uo[3]);
                    *reinterpret_cast<float4 *>(Lam + e) = make_float4(lo[0], lo[1], lo[2], lo[3]);
                    *xchunk_w<Q>(XA, ra, lane / 16) = make_float4(xo[0], xo[1], xo[2], xo[3]);   // X+ in place
                }
            }
            sum_partials<Q, NW>(gx, cx, red, sh.G, sh.C);
        }
        // ---- phase B: T_j = X+^T R_j + b V_j - P_j (columns of several parts: partial sums) ----
        // the last wavefront meanwhile solves the Y system (Inv = (GX + b I)^-1,
        // F[l][k] = (Inv C)[k][l]), which the Y update needs and phase B does not
        t = fresh_tid();
        lane = t % WAVE;
        if (wave == NW - 1)
            spd_solve_wave<Q, false>(sh, beta, lane);
        else
        for (int g = wave; g < G; g += NW - 1) {
            int j, cnt, pc, np;
            part_of(g, j, cnt, pc, np);
            const int base = grp[g];
            const int len = (grp[g + 1] - base) >> 6;
            float acc[3 * Q];
#pragma unroll
            for (int kk = 0; kk < 3 * Q; ++kk) acc[kk] = 0.f;
            // the part's entries are loaded ADM_DB at a time, all in flight together
            for (int k0 = 0; k0 < len; k0 += ADM_DB) {
                int ib[ADM_DB];
                float rb0[ADM_DB], rb1[ADM_DB], rb2[ADM_DB];
#pragma unroll
                for (int u = 0; u < ADM_DB; ++u) {
                    const bool act = k0 + u < cnt;
                    const int e = base + 64 * (k0 + u) + lane;
                    ib[u] = act ? (int)erow[e] : -1;
                    rb0[u] = act ? eres[3 * e] : 0.f;
                    rb1[u] = act ? eres[3 * e + 1] : 0.f;
                    rb2[u] = act ? eres[3 * e + 2] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < ADM_DB; ++u) {
                    if (ib[u] >= 0) {
#pragma unroll
                        for (int v = 0; v < QV; ++v) {
                            const float4 a = *xchunk<Q>(XA, ib[u], v);
                            const float xs[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
                            for (int w = 0; w < 4; ++w) {
                                acc[4 * v + w] = fmaf(rb0[u], xs[w], acc[4 * v + w]);
                                acc[Q + 4 * v + w] = fmaf(rb1[u], xs[w], acc[Q + 4 * v + w]);
                                acc[2 * Q + 4 * v + w] = fmaf(rb2[u], xs[w], acc[2 * Q + 4 * v + w]);
                            }
                        }
                    }
                }
            }
            if (64 * g + lane < P) {
                if (np == 1) {
                    // every load before the first store: loads and stores share
                    // one in-order counter, so a load after a store waits for it.
                    // W is added into acc one channel (q values) at a time, so
                    // that at most q loaded values are held at once.
                    const size_t o = (size_t)j * 3 * Q;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float4 wv[QV];
#pragma unroll
                        for (int v = 0; v < QV; ++v) wv[v] = reinterpret_cast<const float4 *>(W + o)[c * QV + v];
#pragma unroll
                        for (int v = 0; v < QV; ++v) {
                            const int k = 4 * (c * QV + v);
                            acc[k] += wv[v].x;
                            acc[k + 1] += wv[v].y;
                            acc[k + 2] += wv[v].z;
                            acc[k + 3] += wv[v].w;
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 3 * Q / 4; ++v)
                        reinterpret_cast<float4 *>(Yt + o)[v] =
                            make_float4(acc[4 * v], acc[4 * v + 1], acc[4 * v + 2], acc[4 * v + 3]);
                } else {
                    float4 *pp = reinterpret_cast<float4 *>(partial + (size_t)pc * 3 * Q);
#pragma unroll
                    for (int v = 0; v < 3 * Q / 4; ++v)
                        pp[v] = make_float4(acc[4 * v], acc[4 * v + 1], acc[4 * v + 2], acc[4 * v + 3]);
                }
            }
        }
        __threadfence_block();
        __syncthreads();
        // columns of several parts: sum their partials in part order
        t = fresh_tid();
        lane = t % WAVE;
        const int nsplit = ell.nsplit[s];
        const int ncmb = nsplit * (3 * Q / 4);
        for (int e0 = t; e0 < ncmb; e0 += ADM_CMB * THREADS) {
            float4 a[ADM_CMB];
            size_t o[ADM_CMB];
#pragma unroll
            for (int b = 0; b < ADM_CMB; ++b) {
                const int e = e0 + b * THREADS;
                a[b] = make_float4(0.f, 0.f, 0.f, 0.f);
                o[b] = 0;
                if (e < ncmb) {
                    const int j = ell.split[d.off_col + e / (3 * Q / 4)], v = e % (3 * Q / 4);
                    const int p0 = pbase[j], p1 = pbase[j + 1];
                    a[b] = reinterpret_cast<const float4 *>(partial + (size_t)p0 * 3 * Q)[v];
                    for (int u = p0 + 1; u < p1; ++u) {
                        const float4 c = reinterpret_cast<const float4 *>(partial + (size_t)u * 3 * Q)[v];
                        a[b].x += c.x;
                        a[b].y += c.y;
                        a[b].z += c.z;
                        a[b].w += c.w;
                    }
                    o[b] = (size_t)j * 3 * Q + 4 * v;
                    const float4 w = *reinterpret_cast<const float4 *>(W + o[b]);
                    a[b].x += w.x;
                    a[b].y += w.y;
                    a[b].z += w.z;
                    a[b].w += w.w;
                }
            }
#pragma unroll
            for (int b = 0; b < ADM_CMB; ++b)
                if (e0 + b * THREADS < ncmb) *reinterpret_cast<float4 *>(Yt + o[b]) = a[b];
        }
        __threadfence_block();
        __syncthreads();
        // ---- Y+ = Y F + T Inv (FP32 MFMA on FP32 copies of the FP64 q x q factors) over the 3n rows, V, P, Gram Y+^T Y+ ----
        t = fresh_tid();
        lane = t % WAVE;
        {
            float b1[QV], b2[QV];
            load_rhs_c(b1, b2);
            f4 gy = {0.f, 0.f, 0.f, 0.f};
            const f4 zero = {0.f, 0.f, 0.f, 0.f};
            float ymx = 0.f;
            // tile r0 of the 3n rows.  Y and T enter as MFMA operands of row
            // lane % 16, components QV (lane / 16) .. + QV - 1 (one vector
            // load each).  The product is formed twice: transposed, so that a
            // lane holds components 4 (lane / 16) .. + 3 of row r0 + lane % 16
            // (P read, Y, W and P written as float4), and plain (result layout)
            // for the Gram Y+^T Y+.  Indices are clamped into the slice and
            // values outside it masked at use.
            auto load_tile = [&](int r0, float *ya, float *ta, float4 &pa) {
                const int ra = min(r0 + lane % 16, R3 - 1);
                const size_t e = (size_t)ra * Q + QV * (lane / 16);
                if constexpr (QV == 4) {
                    const float4 y4 = *reinterpret_cast<const float4 *>(Y + e);
                    const float4 t4 = *reinterpret_cast<const float4 *>(Yt + e);
                    ya[0] = y4.x; ya[1] = y4.y; ya[2] = y4.z; ya[3] = y4.w;
                    ta[0] = t4.x; ta[1] = t4.y; ta[2] = t4.z; ta[3] = t4.w;
                } else if constexpr (QV == 2) {
                    const float2 y2 = *reinterpret_cast<const float2 *>(Y + e);
                    const float2 t2 = *reinterpret_cast<const float2 *>(Yt + e);
                    ya[0] = y2.x; ya[1] = y2.y;
                    ta[0] = t2.x; ta[1] = t2.y;
                } else {
                    ya[0] = Y[e];
                    ta[0] = Yt[e];
                }
                const int cb = min(4 * (lane / 16), Q - 4);
                pa = *reinterpret_cast<const float4 *>(Pi + (size_t)ra * Q + cb);
            };
            auto do_tile = [&](int r0, const float *ya, const float *ta, const float4 &pa) {
                const bool rok = r0 + lane % 16 < R3;
                f4 D = {0.f, 0.f, 0.f, 0.f}, Dt = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int v = 0; v < QV; ++v) {
                    const float y = rok ? ya[v] : 0.f, tt = rok ? ta[v] : 0.f;
                    D = mfma16(y, b1[v], D);
                    D = mfma16(tt, b2[v], D);
                    Dt = mfma16(b1[v], y, Dt);
                    Dt = mfma16(b2[v], tt, Dt);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 4 * (lane / 16) + v, c = lane % 16;   // FP32 result layout
                    const float yn = r < R3 && c < Q ? D[v] : 0.f;
                    gy = mfma16(yn, yn, gy);
                }
                const int cb = 4 * (lane / 16);
                if (rok && cb < Q) {
                    const float pin[4] = {pa.x, pa.y, pa.z, pa.w};
                    float wo[4], po[4], yo[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float yn = Dt[v], pi = pin[v];
                        const float u = nonneg ? fmaxf(0.f, yn + pi * inv_beta) : yn + pi * inv_beta;
                        const float pn = pi + gb * (yn - u);
                        wo[v] = fmaf(beta_f, u, -pn);
                        po[v] = pn;
                        yo[v] = yn;
                        ymx = fmaxf(ymx, fabsf(yn));
                    }
                    const size_t e = (size_t)(r0 + lane % 16) * Q + cb;
                    *reinterpret_cast<float4 *>(W + e) = make_float4(wo[0], wo[1], wo[2], wo[3]);
                    *reinterpret_cast<float4 *>(Pi + e) = make_float4(po[0], po[1], po[2], po[3]);
                    *reinterpret_cast<float4 *>(Y + e) = make_float4(yo[0], yo[1], yo[2], yo[3]);
                }
            };
            for (int r0 = 16 * wave; r0 < R3; r0 += 16 * NW) {
                float ya[QV], ta[QV];
                float4 pa;
                load_tile(r0, ya, ta, pa);
                do_tile(r0, ya, ta, pa);
            }
            __threadfence_block();
            sum_partials<Q, NW>(gy, zero, red, sh.G, nullptr);
            ymax = (double)block_max(ymx, redf);
        }
    }
    for (int e = t; e < m * Q; e += THREADS) Xg[e] = XA[xpos<Q>(e / Q, e % Q)];
    if (t == 0) {
        st[0] = iters;
        if (!(fixed_iters & 1) && iters >= max_iter) st[1] |= VPLMC_SLICE_NOT_CONVERGED;
        st[2] = __float_as_int((float)err);
    }
}


// The slices of slice_list[0 .. count): one workgroup per slice, or, with a
// queue counter (zero at launch), a fixed number of workgroups that take the
// next slice from the counter until the list is exhausted (the list is
// ordered by decreasing cost, so the queue runs longest-first).
__device__ __forceinline__ bool next_slice(int32_t *queue, int32_t count, int &k, int &state) {
    __shared__ int32_t taken;
    if (!queue) {
        k = blockIdx.x;
        return state++ == 0 && k < count;
    }
    if (threadIdx.x == 0) taken = atomicAdd(queue, 1);
    __syncthreads();
    k = __builtin_amdgcn_readfirstlane(taken);     // uniform: descriptors and pointers stay scalar
    __syncthreads();
    return k < count;
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_adm_ell(
    const SliceDesc *__restrict__ desc, const int32_t *__restrict__ slice_list, int32_t count, int32_t *queue,
    uint64_t seed, int32_t max_iter, int32_t fixed_iters, float tol, float alpha0, float beta0, float gamma,
    const int32_t *__restrict__ col_ptr_all, EllView ell, float *X_all, float *Xp_all, float *Lam_all, float *Y_all,
    float *Yp_all, float *Pi_all, float *Yt_all, float *red_all, double *e2part_all, float *scale_all,
    int32_t *stats_all) {
    int k, state = 0;
    while (next_slice(queue, count, k, state)) {
        adm_ell_slice<Q, THREADS>(__builtin_amdgcn_readfirstlane(slice_list[k]), desc, seed, max_iter, fixed_iters, tol, alpha0, beta0, gamma,
                                  col_ptr_all, ell, X_all, Xp_all, Lam_all, Y_all, Yp_all,
                                  Pi_all, Yt_all, red_all, e2part_all, scale_all, stats_all);
        __syncthreads();
    }
}

// I^c_i = s0 sum_k X_ik (sum_j Y[j][c][k]), FP64 accumulation; one workgroup per slice.
__global__ __launch_bounds__(256) void k_reduce(const SliceDesc *__restrict__ desc,
                                                 const int32_t *__restrict__ pt_ids,
                                                 const float *__restrict__ X_all,
                                                 const float *__restrict__ Y_all,
                                                 const float *__restrict__ scale, int32_t n_points,
                                                 float *__restrict__ radiance) {
    __shared__ double w[3 * VPLMC_MAX_RANK];
    __shared__ double part[256 / 32 * 3 * VPLMC_MAX_RANK];
    const int s = blockIdx.x;
    const SliceDesc d = desc[s];
    const int q = d.q, n = d.n, m = d.m;
    const float *X = X_all + d.off_x;
    const float *Y = Y_all + d.off_y;
    const int t = threadIdx.x;
    // w[c][k] = sum_j Y[j][c][k]: 3q outputs, threads split j into 256 / (3q) groups
    const int outs = 3 * q;
    const int groups = 256 / outs;          // >= 2 since 3q <= 96
    const int o = t % outs, g = t / outs;
    double acc = 0.0;
    if (g < groups)
        for (int j = g; j < n; j += groups) acc += (double)Y[(size_t)j * outs + o];
    if (g < groups) part[g * outs + o] = acc;
    __syncthreads();
    if (t < outs) {
        double v = 0.0;
        for (int gg = 0; gg < groups; ++gg) v += part[gg * outs + t];
        w[t] = v;
    }
    __syncthreads();
    const double s0 = (double)scale[s];
    for (int i = t; i < m; i += 256) {
        double r = 0.0, gg = 0.0, b = 0.0;
        for (int k = 0; k < q; ++k) {
            const double x = (double)X[(size_t)i * q + k];
            r += x * w[k];
            gg += x * w[q + k];
            b += x * w[2 * q + k];
        }
        const int pid = clamp_index(pt_ids[d.pt_off + i], n_points);
        radiance[3 * (size_t)pid] = (float)(s0 * r);
        radiance[3 * (size_t)pid + 1] = (float)(s0 * gg);
        radiance[3 * (size_t)pid + 2] = (float)(s0 * b);
    }
}

// mode word of the completion kernels: bit 0 a fixed iteration count, bit 1
// initial factors given in the X and Y regions, bit 2 no non-negativity
// (U = X+ + Lambda / alpha, V = Y+ + Pi / beta without the projection)
inline int32_t adm_mode(const vplmc_params &prm) {
    return ((prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0) | ((prm.flags & VPLMC_GIVEN_INIT) ? 2 : 0) |
           ((prm.flags & VPLMC_NO_NONNEG) ? 4 : 0);
}

// grid of a launch over `count` slices: one workgroup per slice, or with a
// queue as many workgroups as fit on the device at once (at most count)
template <typename K>
int adm_grid(K kern, int threads, size_t dyn, int n_cu, bool queue, size_t count, unsigned &grid) {
    grid = (unsigned)count;
    if (!queue) return VPLMC_OK;
    int per_cu = 0;
    VPLMC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, dyn));
    const size_t g = (size_t)std::max(per_cu, 1) * (size_t)std::max(n_cu, 1);
    grid = (unsigned)std::min(count, g);
    return VPLMC_OK;
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

template <int Q, int T>
int launch_adm_ell_t(hipStream_t st, size_t count, int max_m, const int32_t *ids_dev, int32_t *queue, int n_cu,
                     const SliceDesc *desc, const vplmc_params &prm, const int32_t *col_ptr, const EllView &ell,
                     float *X, float *Xp, float *Lam, float *Y, float *Yp,
                     float *Pi, float *Yt, float *red, double *e2part, float *scale, int32_t *stats) {
    const size_t dyn = adm_lds_dynamic_bytes(Q, max_m);
    auto kern = k_adm_ell<Q, T>;
    VPLMC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    unsigned grid;
    int rc;
    if ((rc = adm_grid(kern, T, dyn, n_cu, queue != nullptr, count, grid))) return rc;
    if (queue && (rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(queue), 1, 0u))) return rc;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(T), dyn, st, desc, ids_dev, (int32_t)count, queue, prm.seed,
                       prm.max_iter, adm_mode(prm), prm.tol, prm.alpha0, prm.beta0,
                       prm.gamma, col_ptr, ell, X, Xp, Lam, Y, Yp, Pi, Yt, red, e2part, scale,
                       stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

template <int Q>
int launch_adm_ell(hipStream_t st, int threads, size_t count, int max_m, const int32_t *ids_dev, int32_t *queue,
                   int n_cu, const SliceDesc *desc, const vplmc_params &prm, const int32_t *col_ptr,
                   const EllView &ell, float *X, float *Xp, float *Lam,
                   float *Y, float *Yp, float *Pi, float *Yt, float *red, double *e2part, float *scale,
                   int32_t *stats) {
    if (count == 0) return VPLMC_OK;
    if (threads == 512)
        return launch_adm_ell_t<Q, 512>(st, count, max_m, ids_dev, queue, n_cu, desc, prm, col_ptr, ell, X, Xp, Lam,
                                        Y, Yp, Pi, Yt, red, e2part, scale, stats);
    return launch_adm_ell_t<Q, 1024>(st, count, max_m, ids_dev, queue, n_cu, desc, prm, col_ptr, ell, X, Xp, Lam, Y,
                                     Yp, Pi, Yt, red, e2part, scale, stats);
}

}  // namespace

int launch_adm(hipStream_t st, const AdmStreams *ss, const vplmc_plan &plan, int n_cu, const SliceDesc *desc,
               const int32_t *ids_dev, const int32_t *gblk_dev, char *gsys, double *ge2,
               int32_t *queues, const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col,
               const float *csr_val, const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val,
               const EllView &ell, float *X, float *Xn, float *Xp, float *Lam, float *Y, float *Yp, float *Pi,
               float *Yt, float *red, double *e2part, float *scale, int32_t *stats) {
    // ids_dev holds the slice ids of groups 0..7 in order (2 * rank bucket + variant)
    size_t base[9] = {0};
    for (int g = 0; g < 8; ++g) base[g + 1] = base[g] + plan.groups[g].size();
    const int32_t *id[8];
    for (int g = 0; g < 8; ++g) id[g] = ids_dev + base[g];
    const bool qm = plan.tune.adm_queue != 0;
    auto qp = [&](int g) { return qm ? queues + g : nullptr; };
    const int thr = plan.tune.adm_threads;
    // The rank buckets touch disjoint slices: with more than one bucket present,
    // ranks 4, 8 and 16 run on streams forked from st while rank 32 (the
    // longest slices) runs on st, so that one bucket's tail of large slices
    // overlaps the others.  Every stream is joined back into st.
    int buckets = 0;
    for (int b = 0; b < 4; ++b) buckets += (plan.groups[2 * b].size() + plan.groups[2 * b + 1].size()) > 0;
    const bool fork = ss != nullptr && buckets > 1;
    hipStream_t sb[4] = {st, st, st, st};
    if (fork) {
        VPLMC_HIP(hipEventRecord(ss->fork, st));
        for (int k = 0; k < 3; ++k) {
            VPLMC_HIP(hipStreamWaitEvent(ss->side[k], ss->fork, 0));
            sb[k] = ss->side[k];
        }
    }
    // rank 32 never fits in LDS (group 6 is empty)
    int rc = launch_gadm<32, 256>(sb[3], plan, 7, id[7], gblk_dev, gsys, ge2, desc, prm, row_ptr, csr_col, csr_val,
                                  col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
#define VPLMC_ADM_PAIR(B, Q, TG)                                                                                      \
    if (!rc)                                                                                                          \
        rc = launch_adm_ell<Q>(sb[B], thr, plan.groups[2 * B].size(), plan.group_max_m[2 * B], id[2 * B], qp(2 * B), \
                               n_cu, desc, prm, col_ptr, ell, X, Xp, Lam, Y, Yp, Pi, Yt, red, e2part, scale, stats); \
    if (!rc)                                                                                                          \
        rc = launch_gadm<Q, 256>(sb[B], plan, 2 * B + 1, id[2 * B + 1], gblk_dev, gsys, ge2, desc, prm, row_ptr,    \
                                 csr_col, csr_val, col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    VPLMC_ADM_PAIR(2, 16, 512)
    VPLMC_ADM_PAIR(1, 8, 512)
    VPLMC_ADM_PAIR(0, 4, 1024)
#undef VPLMC_ADM_PAIR
    if (fork) {
        // joined even after a failed launch, so that no stream is left forked
        for (int k = 0; k < 3; ++k) {
            hipError_t e = hipEventRecord(ss->join[k], ss->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, ss->join[k], 0);
            if (e != hipSuccess && !rc) rc = hip_error(e, "joining the completion streams");
        }
    }
    return rc;
}

int launch_reduce(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *pt_ids,
                  const float *X, const float *Y, const float *scale, int32_t n_points, float *radiance) {
    if (plan.n_slices == 0 || n_points < 1) return VPLMC_OK;
    hipLaunchKernelGGL(k_reduce, dim3(plan.n_slices), dim3(256), 0, st, desc, pt_ids, X, Y, scale, n_points,
                       radiance);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
