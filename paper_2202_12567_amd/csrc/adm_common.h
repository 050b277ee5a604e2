// Device helpers of the two completion kernels (the LDS-resident k_adm_ell
// and the global-memory k_gadm_* launches): wavefront sums, the LDS state of
// a q x q system with its FP64 Cholesky inverse and solve, and the Gram of a
// row-major matrix streamed through LDS.
#pragma once

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
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
// through LDS in tiles of STAGE floats (coalesced float4 loads, the next
// tile in flight while the current one is used); a thread owns a 4 x 4 block
// of G and every groups-th row of a tile.  The groups' partial blocks are then
// summed in group order, so the result does not depend on timing.  part holds
// PCAP floats.
constexpr int GRAM_STAGE = 16384;

template <int Q, int PCAP, int THREADS, int STAGE = GRAM_STAGE>
__device__ void gram_rows(AdmShared<Q> &sh, const float *__restrict__ M, int rows, float *part, float *stage) {
    constexpr int P = Q * Q, QB = Q / 4, NB = QB * QB;
    constexpr int TR = STAGE / Q;                       // rows per tile
    constexpr int NL = STAGE / 4 / THREADS;             // float4 per thread per tile
    static_assert(NL >= 1 && NL * 4 * THREADS == STAGE, "tile split");
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
            const int64_t idx = (int64_t)tile * (STAGE / 4) + u * THREADS + t;
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

// mode word of the completion kernels: bit 0 a fixed iteration count, bit 1
// initial factors given in the X and Y regions, bit 2 no non-negativity
// (U = X+ + Lambda / alpha, V = Y+ + Pi / beta without the projection)
inline int32_t adm_mode(const vplmc_params &prm) {
    return ((prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0) | ((prm.flags & VPLMC_GIVEN_INIT) ? 2 : 0) |
           ((prm.flags & VPLMC_NO_NONNEG) ? 4 : 0);
}

}  // namespace
}  // namespace vplmc
