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
int launch_adm_q(hipStream_t st, const std::vector<int32_t> &ids, const int32_t *ids_dev,
                 const SliceDesc *desc, const vplmc_params &prm, const int32_t *row_ptr,
                 const int32_t *csr_col, const float *csr_val, const int32_t *col_ptr,
                 const int32_t *csc_row, const float *csc_val, float *X, float *Xn, float *Xp,
                 float *Lam, float *Y, float *Yp, float *Pi, float *scale, int32_t *stats) {
    if (ids.empty()) return VPLMC_OK;
    hipLaunchKernelGGL((k_adm<Q, THREADS>), dim3((unsigned)ids.size()), dim3(THREADS), 0, st, desc,
                       ids_dev, prm.seed, prm.max_iter, (prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0,
                       prm.tol, prm.alpha0, prm.beta0, prm.gamma, row_ptr, csr_col, csr_val, col_ptr,
                       csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace

int launch_adm(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *ids_dev,
               const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
               const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Xn,
               float *Xp, float *Lam, float *Y, float *Yp, float *Pi, float *scale, int32_t *stats) {
    // ids_dev holds the slice ids grouped by rank bucket 4, 8, 16, 32 (in that order)
    size_t base = 0;
    int rc;
    const std::vector<int32_t> *b = plan.slices_by_q;
    rc = launch_adm_q<4, 1024>(st, b[0], ids_dev + base, desc, prm, row_ptr, csr_col, csr_val, col_ptr,
                               csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    if (rc) return rc;
    base += b[0].size();
    rc = launch_adm_q<8, 512>(st, b[1], ids_dev + base, desc, prm, row_ptr, csr_col, csr_val, col_ptr,
                               csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    if (rc) return rc;
    base += b[1].size();
    rc = launch_adm_q<16, 512>(st, b[2], ids_dev + base, desc, prm, row_ptr, csr_col, csr_val, col_ptr,
                               csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
    if (rc) return rc;
    base += b[2].size();
    return launch_adm_q<32, 256>(st, b[3], ids_dev + base, desc, prm, row_ptr, csr_col, csr_val, col_ptr,
                                 csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
}

int launch_reduce(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *pt_ids,
                  const float *X, const float *Y, const float *scale, float *radiance) {
    if (plan.n_slices == 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_reduce, dim3(plan.n_slices), dim3(256), 0, st, desc, pt_ids, X, Y, scale, radiance);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
