// Non-negative completion of each slice matrix by the alternating direction
// method (Appendix A), and the factorised column sum I(s) = X (Y e)
// (Sec. 3, step 5).
//
// One workgroup owns one slice for the whole iteration, so an iteration
// needs only workgroup barriers.  The slice matrix is the stacked
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
//   phase B, one wavefront per column j (CSC): the residual again from
//     (X_k, Y_k), RY_j = sum r X+_i, Y+_j = (GX + bI)^-1 ((X+^T X) Y_j + RY_j + b V_j - P_j),
//     V_j = max(0, Y+_j + P_j / b), P_j += g b (Y+_j - V_j);
//   GY = Y+ Y+^T for the next iteration.
// The q x q systems are factored by Cholesky in FP64 and inverted once per
// iteration; rows and columns are then multiplied by the FP64 inverse.
// Every reduction has a fixed order: results are bitwise reproducible.

#include <type_traits>

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
// a wavefront-uniform value kept in a scalar register
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
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

// (G + shift I)^-1 in FP64 by Cholesky; result in sh.Inv.  All threads call.
template <int Q>
__device__ void spd_inverse(AdmShared<Q> &sh, double shift) {
    const int t = threadIdx.x;
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

// Gram G = M^T M of a (rows x Q) FP32 matrix into sh.G, fixed summation order.
template <int Q>
__device__ void gram_rows(AdmShared<Q> &sh, const float *__restrict__ M, int rows, float *part) {
    const int t = threadIdx.x;
    const int T = blockDim.x;
    constexpr int P = Q * Q;
    if (T >= P) {
        const int groups = T / P, g = t / P, p = t % P;
        if (g < groups) {
            float acc = 0.f;
            for (int r = g; r < rows; r += groups)
                acc = fmaf(M[(size_t)r * Q + p / Q], M[(size_t)r * Q + p % Q], acc);
            part[g * P + p] = acc;
        }
        __syncthreads();
        for (int e = t; e < P; e += T) {
            float v = 0.f;
            for (int gg = 0; gg < groups; ++gg) v += part[gg * P + e];
            sh.G[e] = v;
        }
    } else {
        for (int e = t; e < P; e += T) {
            float acc = 0.f;
            for (int r = 0; r < rows; ++r) acc = fmaf(M[(size_t)r * Q + e / Q], M[(size_t)r * Q + e % Q], acc);
            sh.G[e] = acc;
        }
    }
    __syncthreads();
}

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_adm(
    const SliceDesc *__restrict__ desc, const int32_t *__restrict__ slice_list, uint64_t seed,
    int32_t max_iter, int32_t fixed_iters, float tol, float alpha0, float beta0, float gamma,
    const int32_t *__restrict__ row_ptr_all, const int32_t *__restrict__ csr_col_all,
    const float *__restrict__ csr_val_all, const int32_t *__restrict__ col_ptr_all,
    const int32_t *__restrict__ csc_row_all, const float *__restrict__ csc_val_all, float *X_all,
    float *Xn_all, float *Xp_all, float *Lam_all, float *Y_all, float *Yp_all, float *Pi_all,
    float *scale_all, int32_t *stats_all) {
    constexpr int NW = THREADS / WAVE;
    __shared__ AdmShared<Q> sh;
    __shared__ float part[(NW * Q * Q > 2 * 1024) ? NW * Q * Q : 2 * 1024];

    const int s = slice_list[blockIdx.x];
    const SliceDesc d = desc[s];
    const int m = d.m, n = d.n;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);

    const int32_t *row_ptr = row_ptr_all + d.off_row;
    const int32_t *col_ptr = col_ptr_all + d.off_colptr;
    const int32_t *csr_col = csr_col_all + d.off_omega;
    const float *csr_val = csr_val_all + 3 * d.off_omega;
    const int32_t *csc_row = csc_row_all + d.off_omega;
    const float *csc_val = csc_val_all + 3 * d.off_omega;
    float *Xa = X_all + d.off_x;
    float *Xb = Xn_all + d.off_x;
    float *Xp = Xp_all + d.off_x;
    float *Lam = Lam_all + d.off_x;
    float *Y = Y_all + d.off_y;
    float *Yp = Yp_all + d.off_y;
    float *Pi = Pi_all + d.off_y;
    int32_t *st = stats_all + 4 * s;
    const int nnz = row_ptr[m];

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
        }
        return;
    }
    const double s0 = tot / (3.0 * (double)nnz);
    const float inv_s0 = (float)(1.0 / s0);
    const double normM = sqrt(totsq) / s0;
    if (t == 0) scale_all[s] = (float)s0;

    // ---- initial factors: fp32(u24(Philox) * fp32(2 / sqrt q)) ----
    const float cq = (float)(2.0 / sqrt((double)Q));
    for (int e = t; e < m * Q; e += THREADS) {
        const int i = e / Q, k = e % Q;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)i, (uint64_t)k, TAG_INITX, 0);
        const float v = __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq);
        Xa[e] = v;
        Xp[e] = v;
        Lam[e] = 0.f;
    }
    for (int e = t; e < 3 * n * Q; e += THREADS) {
        const int j = e / (3 * Q), c = (e / Q) % 3, k = e % Q;
        const uint64_t col = (uint64_t)c * (uint64_t)n + (uint64_t)j;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)k, col, TAG_INITY, 0);
        const float v = __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq);
        Y[e] = v;
        Yp[e] = v;
        Pi[e] = 0.f;
    }
    __threadfence_block();
    __syncthreads();

    const double alpha = (double)alpha0 * (3.0 * n) / Q;
    const double beta = (double)beta0 * (double)m / Q;
    const float alpha_f = (float)alpha, beta_f = (float)beta;
    const float ga = (float)((double)gamma * alpha), gb = (float)((double)gamma * beta);
    const float inv_alpha = (float)(1.0 / alpha), inv_beta = (float)(1.0 / beta);

    gram_rows<Q>(sh, Y, 3 * n, part);

    float *X = Xa, *Xn = Xb;
    int iters = max_iter;
    double err = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        // ---- X system: Inv = (GY + a I)^-1, F = GY Inv ----
        spd_inverse<Q>(sh, alpha);
        for (int e = t; e < Q * Q; e += THREADS) {
            const int a = e / Q, b = e % Q;
            double v = 0.0;
            for (int l = 0; l < Q; ++l) v += (double)sh.G[a * Q + l] * sh.Inv[l * Q + b];
            sh.F[e] = v;
        }
        __syncthreads();

        // ---- phase A: rows ----
        double e2 = 0.0;
        float gx[Q], cx[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) gx[k] = cx[k] = 0.f;
        for (int i = wave; i < m; i += NW) {
            float xi[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) xi[k] = X[(size_t)i * Q + k];
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
#pragma unroll
            for (int k = 0; k < Q; ++k) acc[k] = wave_sum(acc[k]);
            // X+_i (lane k < Q owns column k), U and Lambda updates
            float xn = 0.f;
            if (lane < Q) {
                const int k = lane;
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < Q; ++l) {
                    const float tl = acc[l] + alpha_f * Xp[(size_t)i * Q + l] - Lam[(size_t)i * Q + l];
                    v += (double)xi[l] * sh.F[l * Q + k] + (double)tl * sh.Inv[l * Q + k];
                }
                xn = (float)v;
                const float lam = Lam[(size_t)i * Q + k];
                const float u = fmaxf(0.f, xn + lam * inv_alpha);
                Xn[(size_t)i * Q + k] = xn;
                Xp[(size_t)i * Q + k] = u;
                Lam[(size_t)i * Q + k] = lam + ga * (xn - u);
            }
            // Grams: lane k accumulates GX[l][k] = sum x+_l x+_k and C[l][k] = sum x+_l x_k
            float xk = 0.f;
#pragma unroll
            for (int k = 0; k < Q; ++k) xk = (lane == k) ? xi[k] : xk;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                const float xl = __shfl(xn, l, WAVE);
                gx[l] = fmaf(xl, xn, gx[l]);
                cx[l] = fmaf(xl, xk, cx[l]);
            }
        }
        e2 = wave_sum_d(e2);
        if (lane == 0) sh.red[wave] = e2;
        if (lane < Q) {
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                part[(wave * Q + l) * Q + lane] = gx[l];
            }
        }
        __syncthreads();
        double e2t = 0.0;
        for (int w = 0; w < NW; ++w) e2t += sh.red[w];
        err = sqrt(e2t) / normM;
        for (int e = t; e < Q * Q; e += THREADS) {
            float v = 0.f;
            for (int w = 0; w < NW; ++w) v += part[w * Q * Q + e];
            sh.G[e] = v;
        }
        __syncthreads();
        if (lane < Q) {
#pragma unroll
            for (int l = 0; l < Q; ++l) part[(wave * Q + l) * Q + lane] = cx[l];
        }
        __syncthreads();
        for (int e = t; e < Q * Q; e += THREADS) {
            float v = 0.f;
            for (int w = 0; w < NW; ++w) v += part[w * Q * Q + e];
            sh.C[e] = v;
        }
        __syncthreads();
        if (!fixed_iters && err < (double)tol) {
            iters = it;
            break;
        }

        // ---- Y system: Inv = (GX + b I)^-1, F^T = (Inv C)^T ----
        spd_inverse<Q>(sh, beta);
        for (int e = t; e < Q * Q; e += THREADS) {
            const int a = e / Q, b = e % Q;   // F[a][b] = sum_l Inv[a][l] C[l][b]; store F^T at [b][a]
            double v = 0.0;
            for (int l = 0; l < Q; ++l) v += sh.Inv[a * Q + l] * (double)sh.C[l * Q + b];
            sh.F[b * Q + a] = v;
        }
        __syncthreads();

        // ---- phase B: columns ----
        for (int j = wave; j < n; j += NW) {
            float y0[Q], y1[Q], y2[Q];
            const float *yj = Y + (size_t)j * 3 * Q;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                y0[k] = yj[k];
                y1[k] = yj[Q + k];
                y2[k] = yj[2 * Q + k];
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
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                a0[k] = wave_sum(a0[k]);
                a1[k] = wave_sum(a1[k]);
                a2[k] = wave_sum(a2[k]);
            }
            // Y+ for output o = (c, k): lanes o < 3Q (two rounds when 3Q > 64)
            float *ypj = Yp + (size_t)j * 3 * Q;
            float *pij = Pi + (size_t)j * 3 * Q;
            float outv[2];
            int outo[2];
#pragma unroll
            for (int rnd = 0; rnd < 2; ++rnd) {
                const int o = lane + rnd * WAVE;
                outo[rnd] = o;
                outv[rnd] = 0.f;
                if (o < 3 * Q) {
                    const int c = o / Q, k = o % Q;
                    double v = 0.0;
#pragma unroll
                    for (int l = 0; l < Q; ++l) {
                        const float yl = c == 0 ? y0[l] : (c == 1 ? y1[l] : y2[l]);
                        const float rl = c == 0 ? a0[l] : (c == 1 ? a1[l] : a2[l]);
                        const float tl = rl + beta_f * ypj[c * Q + l] - pij[c * Q + l];
                        v += sh.F[l * Q + k] * (double)yl + sh.Inv[l * Q + k] * (double)tl;
                    }
                    outv[rnd] = (float)v;
                }
            }
            // all reads of Yp/Pi/Y for this column are done by every lane
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int rnd = 0; rnd < 2; ++rnd) {
                const int o = outo[rnd];
                if (o < 3 * Q) {
                    const float yn = outv[rnd];
                    const float pv = pij[o];
                    const float v = fmaxf(0.f, yn + pv * inv_beta);
                    ypj[o] = v;
                    pij[o] = pv + gb * (yn - v);
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int rnd = 0; rnd < 2; ++rnd)
                if (outo[rnd] < 3 * Q) Y[(size_t)j * 3 * Q + outo[rnd]] = outv[rnd];
        }
        __threadfence_block();
        __syncthreads();
        gram_rows<Q>(sh, Y, 3 * n, part);
        float *tmp = X;
        X = Xn;
        Xn = tmp;
    }
    // final X lives in X; make it the X region
    if (X != Xa) {
        for (int e = t; e < m * Q; e += THREADS) Xa[e] = X[e];
    }
    if (t == 0) {
        st[0] = iters;
        if (!fixed_iters && iters >= max_iter) st[1] |= VPLMC_SLICE_NOT_CONVERGED;
        st[2] = __float_as_int((float)err);
    }
}

// ---------------------------------------------------------------------------
// LDS-resident variant for ranks 4, 8, 16: both X buffers live in LDS and
// both phases stream the slice's samples in column-major (CSC) order, so the
// only gathers are LDS reads and reads of Y rows that neighbouring lanes
// share.
//   phase A, one lane per sampled entry: X_i (LDS) and Y_j (global, 3q
//     floats) in registers, the three dots X_i . Y_j^c, the residual r,
//     which is also stored for phase B, and the q components of
//     sum_c r_c Y_j^c added into the R Y^T accumulator in the other LDS
//     buffer with LDS float atomics.  The accumulator's rows are rotated by
//     their index, (i, k) at i q + (k + i) mod q, so that the lanes of one
//     atomic instruction (same k, random i) spread over the banks;
//   X update, one thread per row: t = R Y^T + a U - L un-rotated in place,
//     X+ = X (GY Inv) + t Inv in FP64, written through a global staging buffer;
//   phase B, a wavefront is four groups of 16 lanes (one DPP row each); a
//     group owns one column at a time and lane k owns rank component k.
//     The stored residuals of the column arrive 16 at a time, one per lane,
//     and are handed to the group by DPP row broadcasts; X+^T R is
//     accumulated in lane k, Y+_j solved in FP64 with the inverse applied
//     across the group by DPP broadcasts, and Y+ Y+^T accumulated per lane
//     and added into the Gram with LDS atomics.
// The LDS atomics make the FP summation order, and hence the last bits of
// the result, vary between runs.
constexpr int GRP = 16;   // lanes per column group = one DPP row
constexpr int PBK = 1;    // samples per lane in one batch

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_mov_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
// sum over the 16 lanes of a DPP row, result in every lane of the row
__device__ __forceinline__ float row_sum16(float v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}
// value of lane S of the row, in every lane of the row (row_newbcast)
template <int S>
__device__ __forceinline__ float row_bcast(float v) { return dpp_mov<0x150 + S>(v); }
template <int S>
__device__ __forceinline__ int row_bcast_i(int v) { return dpp_mov_i<0x150 + S>(v); }

template <int S, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (S < N) {
        f(std::integral_constant<int, S>{});
        static_for<S + 1, N>(f);
    }
}

struct Batch {
    int i[PBK];
    float m0[PBK], m1[PBK], m2[PBK];
};

__device__ __forceinline__ void load_batch(const int32_t *__restrict__ csc_row, const float *__restrict__ resid,
                                           int p0, int end, int gl, Batch &b) {
#pragma unroll
    for (int u = 0; u < PBK; ++u) {
        const int p = p0 + u * GRP + gl;
        const bool ok = p < end;
        const int pc = ok ? p : 0;
        b.i[u] = ok ? csc_row[pc] : 0;
        b.m0[u] = ok ? resid[3 * pc] : 0.f;
        b.m1[u] = ok ? resid[3 * pc + 1] : 0.f;
        b.m2[u] = ok ? resid[3 * pc + 2] : 0.f;
    }
}

// phase A for sampled entry p = (i, j) with scaled values m0..m2.  The
// q components of sum_c r_c Y_j^c, times 2^S, are rounded to integers and
// added into row i of the fixed-point accumulator (row stride q + 1, so the
// lanes' rows fall in different banks); integer sums do not depend on the
// order of the additions.
template <int Q>
__device__ __forceinline__ void entryA(int p, int i, int j, float m0, float m1, float m2, const float *XA,
                                       int32_t *RXI, const float *__restrict__ Y, float *__restrict__ resid,
                                       float fxs, double &e2, float &rsmax) {
    float y[3 * Q], x[Q];
    const float4 *y4 = reinterpret_cast<const float4 *>(Y + (size_t)j * 3 * Q);
#pragma unroll
    for (int v = 0; v < 3 * Q / 4; ++v) {
        const float4 a = y4[v];
        y[4 * v] = a.x;
        y[4 * v + 1] = a.y;
        y[4 * v + 2] = a.z;
        y[4 * v + 3] = a.w;
    }
    const float4 *x4 = reinterpret_cast<const float4 *>(XA + i * Q);
#pragma unroll
    for (int v = 0; v < Q / 4; ++v) {
        const float4 a = x4[v];
        x[4 * v] = a.x;
        x[4 * v + 1] = a.y;
        x[4 * v + 2] = a.z;
        x[4 * v + 3] = a.w;
    }
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        d0 = fmaf(x[k], y[k], d0);
        d1 = fmaf(x[k], y[Q + k], d1);
        d2 = fmaf(x[k], y[2 * Q + k], d2);
    }
    const float r0 = m0 - d0, r1 = m1 - d1, r2 = m2 - d2;
    e2 += (double)(r0 * r0) + (double)(r1 * r1) + (double)(r2 * r2);
    rsmax = fmaxf(rsmax, fabsf(r0) + fabsf(r1) + fabsf(r2));
    resid[3 * p] = r0;
    resid[3 * p + 1] = r1;
    resid[3 * p + 2] = r2;
    const float s0 = r0 * fxs, s1 = r1 * fxs, s2 = r2 * fxs;
    int32_t *row = RXI + i * (Q + 1);
#pragma unroll
    for (int k = 0; k < Q; ++k) atomicAdd(row + k, __float2int_rn(fmaf(s0, y[k], fmaf(s1, y[Q + k], s2 * y[2 * Q + k]))));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
    return v;
}

// one batch of phase B: cnt valid samples (uniform in the group); the batch
// holds the stored residuals
template <int Q>
__device__ __forceinline__ void batchB(const Batch &b, int cnt, int kk, const float *XB, float &a0, float &a1,
                                       float &a2) {
    const bool kact = kk < Q;
    const int kc = kact ? kk : 0;
#pragma unroll
    for (int u = 0; u < PBK; ++u) {
        static_for<0, GRP>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            if (u * GRP + S < cnt) {
                const int i = row_bcast_i<S>(b.i[u]);
                const float r0 = row_bcast<S>(b.m0[u]), r1 = row_bcast<S>(b.m1[u]), r2 = row_bcast<S>(b.m2[u]);
                const float xn = kact ? XB[i * Q + kc] : 0.f;
                a0 = fmaf(xn, r0, a0);
                a1 = fmaf(xn, r1, a1);
                a2 = fmaf(xn, r2, a2);
            }
        });
    }
}

// block-wide maximum of per-thread values; every thread calls it and gets the result
__device__ __forceinline__ float block_max(float v, float *red) {
    const int nw = blockDim.x / WAVE, lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    float r = red[0];
    for (int k = 1; k < nw; ++k) r = fmaxf(r, red[k]);
    __syncthreads();
    return r;
}

// elements per thread of the fixed-point to float pass (m q <= ADM_CVT_MAX * threads)
constexpr int ADM_CVT_MAX = 18;

template <int Q, int THREADS>
__global__ __launch_bounds__(THREADS) void k_adm_lds(
    const SliceDesc *__restrict__ desc, const int32_t *__restrict__ slice_list, uint64_t seed,
    int32_t max_iter, int32_t fixed_iters, float tol, float alpha0, float beta0, float gamma,
    const int32_t *__restrict__ col_ptr_all, const int32_t *__restrict__ csc_row_all,
    const int32_t *__restrict__ csc_col_all, const float *__restrict__ csc_val_all, float *resid_all, float *X_all,
    float *Xn_all, float *Xp_all, float *Lam_all, float *Y_all, float *Yp_all, float *Pi_all, float *scale_all,
    int32_t *stats_all) {
    static_assert(Q <= GRP, "one lane per rank component");
    constexpr int NW = THREADS / WAVE;
    constexpr int NG = THREADS / GRP;                  // column groups per workgroup
    constexpr int BS = PBK * GRP;                      // samples per group batch
    extern __shared__ __align__(16) float dyn[];
    __shared__ AdmShared<Q> sh;
    __shared__ float red2[THREADS];

    const int s = slice_list[blockIdx.x];
    const SliceDesc d = desc[s];
    const int m = d.m, n = d.n;
    const int t = threadIdx.x, lane = t % WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(t / WAVE);
    const int gl = lane % GRP;                         // lane in its group = rank component
    const int grp = t / GRP;
    const bool kact = gl < Q;
    const int kc = kact ? gl : 0;
    // two buffers of m (q + 1) words: X_k (row stride q) and the other one,
    // which holds the fixed-point R Y^T (row stride q + 1) in phase A and X+
    // (row stride q) from the X update on; they swap every iteration
    float *XA = dyn;
    float *XB = dyn + (size_t)m * (Q + 1);
    __shared__ float redf[NW];

    const int32_t *col_ptr = col_ptr_all + d.off_colptr;
    const int32_t *csc_row = csc_row_all + d.off_omega;
    const int32_t *csc_col = csc_col_all + d.off_omega;
    const float *csc_val = csc_val_all + 3 * d.off_omega;
    float *resid = resid_all + 3 * d.off_omega;
    float *Xg = X_all + d.off_x;
    float *Xs = Xn_all + d.off_x;     // staging of X+
    float *Xp = Xp_all + d.off_x;
    float *Lam = Lam_all + d.off_x;
    float *Y = Y_all + d.off_y;
    float *Yp = Yp_all + d.off_y;
    float *Pi = Pi_all + d.off_y;
    int32_t *st = stats_all + 4 * s;
    const int nnz = col_ptr[n];

    double sum = 0.0, sumsq = 0.0;
    for (int p = t; p < 3 * nnz; p += THREADS) {
        const double v = (double)csc_val[p];
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

    const float cq = (float)(2.0 / sqrt((double)Q));
    float ym0 = 0.f;
    for (int e = t; e < m * Q; e += THREADS) {
        const int i = e / Q, k = e % Q;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)i, (uint64_t)k, TAG_INITX, 0);
        const float v = __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq);
        XA[e] = v;
        Xp[e] = v;
        Lam[e] = 0.f;
    }
    for (int e = t; e < 3 * n * Q; e += THREADS) {
        const int j = e / (3 * Q), c = (e / Q) % 3, k = e % Q;
        const uint64_t col = (uint64_t)c * (uint64_t)n + (uint64_t)j;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)k, col, TAG_INITY, 0);
        const float v = __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq);
        Y[e] = v;
        Yp[e] = v;
        Pi[e] = 0.f;
        ym0 = fmaxf(ym0, v);
    }
    __threadfence_block();
    __syncthreads();
    gram_rows<Q>(sh, Y, 3 * n, red2);

    // bounds for the fixed-point scale: K = most samples in one row, the
    // largest sum_c |M| of a sample, the largest row 1-norm of X_0
    int32_t *cntr = reinterpret_cast<int32_t *>(XB);
    for (int e = t; e < m; e += THREADS) cntr[e] = 0;
    __syncthreads();
    float msum = 0.f;
    for (int p = t; p < nnz; p += THREADS) {
        atomicAdd(cntr + csc_row[p], 1);
        msum = fmaxf(msum, fabsf(csc_val[3 * p]) + fabsf(csc_val[3 * p + 1]) + fabsf(csc_val[3 * p + 2]));
    }
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
    // a-priori bound on sum_c |r_c| for the first iteration
    double rs_est = (msum_max + 3.0 * x1max * ymax) * (1.0 + 1e-5);
    // scale 2^S with K (rs ymax 2^S + 1/2) < 2^31 - 1, taken near 2^30 / (K rs ymax)
    auto fits = [&](int S, double rs) {
        return Krow * (rs * ymax * ldexp(1.0, S) + 0.5) < 2147483647.0;
    };
    auto pick_scale = [&](double rs) {
        const double b = Krow * rs * ymax;
        int S = b > 0.0 ? (int)floor(log2(1073741824.0 / b)) : 60;
        S = S > 60 ? 60 : (S < -60 ? -60 : S);
        while (S > -60 && !fits(S, rs)) --S;
        return S;
    };

    const double alpha = (double)alpha0 * (3.0 * n) / Q;
    const double beta = (double)beta0 * (double)m / Q;
    const float alpha_f = (float)alpha, beta_f = (float)beta;
    const float ga = (float)((double)gamma * alpha), gb = (float)((double)gamma * beta);
    const float inv_alpha = (float)(1.0 / alpha), inv_beta = (float)(1.0 / beta);

    // column metadata of a group's round: j = rd * NG + grp
    auto col_range = [&](int j, int &b, int &e) {
        if (j < n) {
            b = col_ptr[j];
            e = col_ptr[j + 1];
        } else {
            b = e = 0;
        }
    };
    auto load_y = [&](int j, float &y0, float &y1, float &y2) {
        const float *yj = Y + (size_t)(j < n ? j : 0) * 3 * Q;
        y0 = (kact && j < n) ? yj[kc] : 0.f;
        y1 = (kact && j < n) ? yj[Q + kc] : 0.f;
        y2 = (kact && j < n) ? yj[2 * Q + kc] : 0.f;
    };

    int iters = max_iter;
    double err = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        // ---- phase A: residuals, 2^S R Y^T added into XB (fixed point) ----
        int32_t *RXI = reinterpret_cast<int32_t *>(XB);
        int S = pick_scale(rs_est);
        double e2t = 0.0;
        float rsc = 0.f;
        for (;;) {
            const float fxs = ldexpf(1.f, S);
            for (int e = t; e < m * (Q + 1); e += THREADS) RXI[e] = 0;
            __syncthreads();
            double e2 = 0.0;
            float rsm = 0.f;
            int p = t;
            int i = 0, j = 0;
            float m0 = 0.f, m1 = 0.f, m2 = 0.f;
            if (p < nnz) {
                i = csc_row[p];
                j = csc_col[p];
                m0 = csc_val[3 * p] * inv_s0;
                m1 = csc_val[3 * p + 1] * inv_s0;
                m2 = csc_val[3 * p + 2] * inv_s0;
            }
            while (p < nnz) {
                const int pn = p + THREADS;
                int in = 0, jn = 0;
                float n0 = 0.f, n1 = 0.f, n2 = 0.f;
                if (pn < nnz) {
                    in = csc_row[pn];
                    jn = csc_col[pn];
                    n0 = csc_val[3 * pn] * inv_s0;
                    n1 = csc_val[3 * pn + 1] * inv_s0;
                    n2 = csc_val[3 * pn + 2] * inv_s0;
                }
                entryA<Q>(p, i, j, m0, m1, m2, XA, RXI, Y, resid, fxs, e2, rsm);
                p = pn;
                i = in;
                j = jn;
                m0 = n0;
                m1 = n1;
                m2 = n2;
            }
            e2 = wave_sum_d(e2);
            rsm = wave_max(rsm);
            if (lane == 0) {
                sh.red[wave] = e2;
                redf[wave] = rsm;
            }
            __syncthreads();
            e2t = 0.0;
            rsc = 0.f;
            for (int w = 0; w < NW; ++w) {
                e2t += sh.red[w];
                rsc = fmaxf(rsc, redf[w]);
            }
            __syncthreads();
            // every integer sum provably fits, or the residuals are not finite
            const double rsb = (double)rsc * (1.0 + 1e-5);
            if (!(rsb < 1e300) || fits(S, rsb) || S <= -60) break;
            S = pick_scale(rsb);
        }
        rs_est = 2.0 * (double)rsc;
        err = sqrt(e2t) / normM;
        if (!fixed_iters && err < (double)tol) {
            iters = it;
            break;
        }

        // ---- X update: t = RX + a U - L (in XB, row stride q), X+ = X (GY Inv) + t Inv ----
        {
            const float ifx = ldexpf(1.f, -S);
            float tv[ADM_CVT_MAX];
#pragma unroll
            for (int u = 0; u < ADM_CVT_MAX; ++u) {
                const int e = t + u * THREADS;
                tv[u] = 0.f;
                if (e < m * Q) {
                    const int i = e / Q, k = e % Q;
                    tv[u] = (float)RXI[i * (Q + 1) + k] * ifx + (alpha_f * Xp[e] - Lam[e]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < ADM_CVT_MAX; ++u) {
                const int e = t + u * THREADS;
                if (e < m * Q) XB[e] = tv[u];
            }
        }
        spd_inverse<Q>(sh, alpha);           // begins and ends with a barrier
        for (int e = t; e < Q * Q; e += THREADS) {
            const int a = e / Q, b = e % Q;
            double v = 0.0;
            for (int l = 0; l < Q; ++l) v += (double)sh.G[a * Q + l] * sh.Inv[l * Q + b];
            sh.F[e] = v;
        }
        __syncthreads();
        for (int e = t; e < m * Q; e += THREADS) {
            const int i = e / Q, k = e % Q;
            const float *xa = XA + i * Q;
            const float *tb = XB + i * Q;
            double v = 0.0;
#pragma unroll 4
            for (int l = 0; l < Q; ++l) v += (double)xa[l] * sh.F[l * Q + k] + (double)tb[l] * sh.Inv[l * Q + k];
            Xs[e] = (float)v;
        }
        __threadfence_block();
        __syncthreads();
        for (int e = t; e < m * Q; e += THREADS) {
            const float xn = Xs[e];
            const float lam = Lam[e];
            const float u = fmaxf(0.f, xn + lam * inv_alpha);
            Xp[e] = u;
            Lam[e] = lam + ga * (xn - u);
            XB[e] = xn;
        }
        __syncthreads();
        // Grams GX = X+^T X+ and C = X+^T X over the rows (fixed order)
        {
            constexpr int P = Q * Q;
            const int groups = THREADS / P, g = t / P, pp = t % P;
            const int a = pp / Q, b = pp % Q;
            float gx = 0.f, cc = 0.f;
            for (int r = g; r < m; r += groups) {
                const float xa = XB[r * Q + a];
                gx = fmaf(xa, XB[r * Q + b], gx);
                cc = fmaf(xa, XA[r * Q + b], cc);
            }
            red2[t] = gx;
            __syncthreads();
            if (t < P) {
                float v = 0.f;
                for (int gg = 0; gg < groups; ++gg) v += red2[gg * P + t];
                sh.G[t] = v;
            }
            __syncthreads();
            red2[t] = cc;
            __syncthreads();
            if (t < P) {
                float v = 0.f;
                for (int gg = 0; gg < groups; ++gg) v += red2[gg * P + t];
                sh.C[t] = v;
            }
        }
        // ---- Y system: Inv = (GX + b I)^-1, F^T = (Inv C)^T ----
        spd_inverse<Q>(sh, beta);
        for (int e = t; e < Q * Q; e += THREADS) {
            const int a = e / Q, b = e % Q;
            double v = 0.0;
            for (int l = 0; l < Q; ++l) v += sh.Inv[a * Q + l] * (double)sh.C[l * Q + b];
            sh.F[b * Q + a] = v;
        }
        for (int e = t; e < Q * Q; e += THREADS) sh.G[e] = 0.f;
        __syncthreads();

        // ---- phase B ----
        float ymx = 0.f;
        float gyrow[Q];
#pragma unroll
        for (int b = 0; b < Q; ++b) gyrow[b] = 0.f;
        {
            int j = grp, beg, end, begn, endn;
            float y0, y1, y2, z0, z1, z2;
            Batch bc, bn, bx;
            col_range(j, beg, end);
            load_y(j, y0, y1, y2);
            load_batch(csc_row, resid, beg, end, gl, bc);
            for (; j < n; j += NG) {
                const int jn = j + NG;
                col_range(jn, begn, endn);
                load_y(jn, z0, z1, z2);
                load_batch(csc_row, resid, begn, endn, gl, bn);
                float a0 = 0.f, a1 = 0.f, a2 = 0.f;
                for (int p0 = beg; p0 < end; p0 += BS) {
                    const bool more = p0 + BS < end;
                    if (more) load_batch(csc_row, resid, p0 + BS, end, gl, bx);
                    batchB<Q>(bc, end - p0, gl, XB, a0, a1, a2);
                    if (more) bc = bx;
                }
                // Y+ (c, k) = sum_l F[k][l] y(c, l) + Inv[k][l] t(c, l), lane k of the group
                float *ypj = Yp + (size_t)j * 3 * Q;
                float *pij = Pi + (size_t)j * 3 * Q;
                const float p0v = kact ? pij[kc] : 0.f, p1v = kact ? pij[Q + kc] : 0.f, p2v = kact ? pij[2 * Q + kc] : 0.f;
                const float t0 = kact ? a0 + beta_f * ypj[kc] - p0v : 0.f;
                const float t1 = kact ? a1 + beta_f * ypj[Q + kc] - p1v : 0.f;
                const float t2 = kact ? a2 + beta_f * ypj[2 * Q + kc] - p2v : 0.f;
                double v0 = 0.0, v1 = 0.0, v2 = 0.0;
                static_for<0, Q>([&](auto lc) {
                    constexpr int L = decltype(lc)::value;
                    const double f = sh.F[L * Q + kc], iv = sh.Inv[L * Q + kc];
                    v0 += f * (double)row_bcast<L>(y0) + iv * (double)row_bcast<L>(t0);
                    v1 += f * (double)row_bcast<L>(y1) + iv * (double)row_bcast<L>(t1);
                    v2 += f * (double)row_bcast<L>(y2) + iv * (double)row_bcast<L>(t2);
                });
                const float n0 = kact ? (float)v0 : 0.f, n1 = kact ? (float)v1 : 0.f, n2 = kact ? (float)v2 : 0.f;
                if (kact) {
                    const float u0 = fmaxf(0.f, n0 + p0v * inv_beta);
                    const float u1 = fmaxf(0.f, n1 + p1v * inv_beta);
                    const float u2 = fmaxf(0.f, n2 + p2v * inv_beta);
                    ypj[kc] = u0;
                    ypj[Q + kc] = u1;
                    ypj[2 * Q + kc] = u2;
                    pij[kc] = p0v + gb * (n0 - u0);
                    pij[Q + kc] = p1v + gb * (n1 - u1);
                    pij[2 * Q + kc] = p2v + gb * (n2 - u2);
                    float *yw = Y + (size_t)j * 3 * Q;
                    yw[kc] = n0;
                    yw[Q + kc] = n1;
                    yw[2 * Q + kc] = n2;
                    ymx = fmaxf(ymx, fmaxf(fabsf(n0), fmaxf(fabsf(n1), fabsf(n2))));
                }
                // row kc of Y+ Y+^T for this column
                static_for<0, Q>([&](auto bc2) {
                    constexpr int B = decltype(bc2)::value;
                    gyrow[B] = fmaf(n0, row_bcast<B>(n0), fmaf(n1, row_bcast<B>(n1), fmaf(n2, row_bcast<B>(n2), gyrow[B])));
                });
                bc = bn;
                y0 = z0; y1 = z1; y2 = z2;
                beg = begn;
                end = endn;
            }
        }
        if (kact) {
#pragma unroll
            for (int b = 0; b < Q; ++b) atomicAdd(&sh.G[kc * Q + b], gyrow[b]);
        }
        __threadfence_block();
        ymax = (double)block_max(ymx, redf);   // ends with a barrier
        float *tmp = XA;
        XA = XB;
        XB = tmp;
    }
    for (int e = t; e < m * Q; e += THREADS) Xg[e] = XA[e];
    if (t == 0) {
        st[0] = iters;
        if (!fixed_iters && iters >= max_iter) st[1] |= VPLMC_SLICE_NOT_CONVERGED;
        st[2] = __float_as_int((float)err);
    }
}

// I^c_i = s0 sum_k X_ik (sum_j Y[j][c][k]), FP64 accumulation; one workgroup per slice.
__global__ __launch_bounds__(256) void k_reduce(const SliceDesc *__restrict__ desc,
                                                 const int32_t *__restrict__ pt_ids,
                                                 const float *__restrict__ X_all,
                                                 const float *__restrict__ Y_all,
                                                 const float *__restrict__ scale,
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
        const int pid = pt_ids[d.pt_off + i];
        radiance[3 * (size_t)pid] = (float)(s0 * r);
        radiance[3 * (size_t)pid + 1] = (float)(s0 * gg);
        radiance[3 * (size_t)pid + 2] = (float)(s0 * b);
    }
}

template <int Q, int THREADS>
int launch_adm_global(hipStream_t st, size_t count, const int32_t *ids_dev, const SliceDesc *desc,
                      const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
                      const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Xn,
                      float *Xp, float *Lam, float *Y, float *Yp, float *Pi, float *scale, int32_t *stats) {
    if (count == 0) return VPLMC_OK;
    hipLaunchKernelGGL((k_adm<Q, THREADS>), dim3((unsigned)count), dim3(THREADS), 0, st, desc, ids_dev, prm.seed,
                       prm.max_iter, (prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0, prm.tol, prm.alpha0, prm.beta0,
                       prm.gamma, row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi,
                       scale, stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

template <int Q>
int launch_adm_lds(hipStream_t st, size_t count, int max_m, const int32_t *ids_dev, const SliceDesc *desc,
                   const vplmc_params &prm, const int32_t *col_ptr, const int32_t *csc_row, const int32_t *csc_col,
                   const float *csc_val, float *resid, float *X, float *Xn, float *Xp, float *Lam, float *Y, float *Yp,
                   float *Pi, float *scale, int32_t *stats) {
    if (count == 0) return VPLMC_OK;
    constexpr int T = adm_lds_threads(Q);
    const size_t dyn = adm_lds_dynamic_bytes(Q, max_m);
    auto kern = k_adm_lds<Q, T>;
    VPLMC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    hipLaunchKernelGGL(kern, dim3((unsigned)count), dim3(T), dyn, st, desc, ids_dev, prm.seed, prm.max_iter,
                       (prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0, prm.tol, prm.alpha0, prm.beta0, prm.gamma, col_ptr,
                       csc_row, csc_col, csc_val, resid, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace

int launch_adm(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *ids_dev,
               const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
               const int32_t *col_ptr, const int32_t *csc_row, const int32_t *csc_col, const float *csc_val,
               float *resid, float *X, float *Xn, float *Xp, float *Lam, float *Y, float *Yp, float *Pi, float *scale,
               int32_t *stats) {
    // ids_dev holds the slice ids of groups 0..7 in order (2 * rank bucket + variant)
    size_t base[9] = {0};
    for (int g = 0; g < 8; ++g) base[g + 1] = base[g] + plan.groups[g].size();
    const int32_t *id[8];
    for (int g = 0; g < 8; ++g) id[g] = ids_dev + base[g];
    int rc;
#define VPLMC_ADM_PAIR(B, Q, TG)                                                                                   \
    if ((rc = launch_adm_lds<Q>(st, plan.groups[2 * B].size(), plan.group_max_m[2 * B], id[2 * B], desc, prm,       \
                                col_ptr, csc_row, csc_col, csc_val, resid, X, Xn, Xp, Lam, Y, Yp, Pi, scale,      \
                                stats)))                                                                           \
        return rc;                                                                                                 \
    if ((rc = launch_adm_global<Q, TG>(st, plan.groups[2 * B + 1].size(), id[2 * B + 1], desc, prm, row_ptr,      \
                                       csr_col, csr_val, col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi,      \
                                       scale, stats)))                                                             \
        return rc;
    VPLMC_ADM_PAIR(0, 4, 1024)
    VPLMC_ADM_PAIR(1, 8, 512)
    VPLMC_ADM_PAIR(2, 16, 512)
    if ((rc = launch_adm_global<32, 256>(st, plan.groups[6].size() + plan.groups[7].size(), id[6], desc, prm, row_ptr,
                                         csr_col, csr_val, col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi,
                                         scale, stats)))
        return rc;
#undef VPLMC_ADM_PAIR
    return VPLMC_OK;
}

int launch_reduce(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *pt_ids,
                  const float *X, const float *Y, const float *scale, float *radiance) {
    if (plan.n_slices == 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_reduce, dim3(plan.n_slices), dim3(256), 0, st, desc, pt_ids, X, Y, scale, radiance);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
