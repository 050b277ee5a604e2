// Per-row masked alternating least squares: a completion variant of the
// slice matrix beside the ADM (Appendix A).  Every row of X, then every
// column of Y, is the ridge least-squares fit to its own observed entries
// (weighted regularisation, Zhou et al. 2008):
//
//   x_i = (sum_{c in Omega_i} y_c y_c^T + lam max(1, n_i) I)^-1 sum_{c in Omega_i} M_ic y_c
//   y_c = (sum_{i in Omega^c} x_i x_i^T + lam max(1, n_c) I)^-1 sum_{i in Omega^c} M_ic x_i
//
// on the stacked m' x 3n' matrix (a sample (i, j) observes columns j, n + j
// and 2n + j, so n_i is three times the row's samples and the three channel
// columns of j share one Gram matrix).  Same scale s0, initial factors,
// residual test and iteration cap as the ADM; components past the slice's
// rank stay 0 (their Gram block is lam max(1, n) I and their right-hand side
// 0).
//
// One workgroup per slice, X and Y in global memory (each slice's factors
// stay in the caches of its CU).  One wavefront per row (then per column):
// the wavefront stages a block of the row's samples' Y vectors in its LDS
// area, each lane accumulates its share of the q x q Gram (FP32) and lanes
// below q the right-hand side; the system is solved in FP64 by a
// right-looking Cholesky in the wavefront's LDS area.  Rows and columns are
// owned by fixed wavefronts and summed in a fixed order, so results are
// bit-reproducible.

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
constexpr int ALS_THREADS = 512;
constexpr int ALS_NW = ALS_THREADS / WAVE;
constexpr int ALS_B = 4;          // samples staged per round

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Solves A x = b for nrhs right-hand sides (b[r * Q + k]) in place, A the
// Q x Q SPD matrix in the wavefront's LDS area (full matrix written; the lower
// triangle is factored).
template <int Q>
__device__ void wave_chol_solve(double *A, double *b, int nrhs, int lane) {
    for (int j = 0; j < Q; ++j) {
        if (lane == 0) A[j * Q + j] = sqrt(A[j * Q + j]);
        wave_lds_sync();
        const double d = A[j * Q + j];
        for (int i = j + 1 + lane; i < Q; i += WAVE) A[i * Q + j] /= d;
        wave_lds_sync();
        for (int e = lane; e < Q * Q; e += WAVE) {
            const int i = e / Q, k = e % Q;
            if (k > j && i >= k) A[i * Q + k] -= A[i * Q + j] * A[k * Q + j];
        }
        wave_lds_sync();
    }
    if (lane < nrhs) {
        double *x = b + lane * Q;
        for (int i = 0; i < Q; ++i) {
            double s = x[i];
            for (int l = 0; l < i; ++l) s -= A[i * Q + l] * x[l];
            x[i] = s / A[i * Q + i];
        }
        for (int i = Q - 1; i >= 0; --i) {
            double s = x[i];
            for (int l = i + 1; l < Q; ++l) s -= A[l * Q + i] * x[l];
            x[i] = s / A[i * Q + i];
        }
    }
    wave_lds_sync();
}

template <int Q>
struct AlsWave {
    double A[Q * Q];
    double b[3 * Q];
    float stage[ALS_B * 3 * Q];
};

// sum over the block of one double per thread, in a fixed order
__device__ __forceinline__ double block_sum_d(double v, double *red) {
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    v = wave_sum_d(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < ALS_NW; ++k) s += red[k];
    __syncthreads();
    return s;
}

template <int Q>
__global__ __launch_bounds__(ALS_THREADS) void k_als(
    const SliceDesc *__restrict__ desc, const int32_t *__restrict__ slice_list, uint64_t seed, int32_t max_iter,
    int32_t mode, float tol, float lam, const int32_t *__restrict__ row_ptr_all,
    const int32_t *__restrict__ csr_col_all, const float *__restrict__ csr_val_all,
    const int32_t *__restrict__ col_ptr_all, const int32_t *__restrict__ csc_row_all,
    const float *__restrict__ csc_val_all, float *X_all, float *Y_all, float *scale_all, int32_t *stats_all) {
    constexpr int EPL = (Q * Q + WAVE - 1) / WAVE;     // Gram entries per lane
    __shared__ AlsWave<Q> wv[ALS_NW];
    __shared__ double red[ALS_NW];
    const int s = __builtin_amdgcn_readfirstlane(slice_list[blockIdx.x]);
    const SliceDesc d = desc[s];
    const int m = d.m, n = d.n, qr = d.qr;
    const int t = threadIdx.x, lane = t % WAVE;
    const int w = __builtin_amdgcn_readfirstlane(t / WAVE);
    AlsWave<Q> &my = wv[w];
    const int32_t *row_ptr = row_ptr_all + d.off_row;
    const int32_t *col_ptr = col_ptr_all + d.off_colptr;
    const int32_t *csr_col = csr_col_all + d.off_omega;
    const float *csr_val = csr_val_all + 3 * d.off_omega;
    const int32_t *csc_row = csc_row_all + d.off_omega;
    const float *csc_val = csc_val_all + 3 * d.off_omega;
    float *X = X_all + d.off_x;
    float *Y = Y_all + d.off_y;
    int32_t *st = stats_all + 4 * s;
    const int nnz = row_ptr[m];

    // ---- scale s0 = mean sampled value; ||P_Omega M|| of M / s0 ----
    double sum = 0.0, sumsq = 0.0;
    for (int p = t; p < 3 * nnz; p += ALS_THREADS) {
        const double v = (double)csr_val[p];
        sum += v;
        sumsq += v * v;
    }
    sum = block_sum_d(sum, red);
    sumsq = block_sum_d(sumsq, red);
    if (nnz == 0 || !(sumsq > 0.0)) {
        for (int e = t; e < m * Q; e += ALS_THREADS) X[e] = 0.f;
        for (int e = t; e < 3 * n * Q; e += ALS_THREADS) Y[e] = 0.f;
        if (t == 0) {
            scale_all[s] = 0.f;
            st[0] = 0;
            st[1] |= VPLMC_SLICE_ALL_ZERO;
            st[2] = __float_as_int(0.f);
        }
        return;
    }
    const double s0 = sum / (3.0 * (double)nnz);
    const float inv_s0 = (float)(1.0 / s0);
    const double normM = sqrt(sumsq) / s0;
    if (t == 0) scale_all[s] = (float)s0;

    // ---- initial factors, as the ADM's ----
    const float cq = (float)(2.0 / sqrt((double)qr));
    const bool given = (mode & 2) != 0;
    for (int e = t; e < m * Q; e += ALS_THREADS) {
        const int i = e / Q, k = e % Q;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)i, (uint64_t)k, TAG_INITX, 0);
        X[e] = k < qr ? (given ? X[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
    }
    for (int e = t; e < 3 * n * Q; e += ALS_THREADS) {
        const int j = e / (3 * Q), c = (e / Q) % 3, k = e % Q;
        const uint64_t col = (uint64_t)c * (uint64_t)n + (uint64_t)j;
        const U64x4 r = philox(seed, (uint64_t)s, (uint64_t)k, col, TAG_INITY, 0);
        Y[e] = k < qr ? (given ? Y[e] : __fmul_rn((float)(r.a >> 40) * 0x1p-24f, cq)) : 0.f;
    }
    __threadfence_block();
    __syncthreads();

    int iters = max_iter;
    double err = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        // ---- relative residual on Omega: one wavefront per row, lanes over its samples ----
        double r2 = 0.0;
        for (int i = w; i < m; i += ALS_NW) {
            const float *xi = X + (size_t)i * Q;
            for (int p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += WAVE) {
                const float *yj = Y + (size_t)csr_col[p] * 3 * Q;
                float d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    const float x = xi[k];
                    d0 = fmaf(x, yj[k], d0);
                    d1 = fmaf(x, yj[Q + k], d1);
                    d2 = fmaf(x, yj[2 * Q + k], d2);
                }
                const float e0 = csr_val[3 * p] * inv_s0 - d0, e1 = csr_val[3 * p + 1] * inv_s0 - d1;
                const float e2 = csr_val[3 * p + 2] * inv_s0 - d2;
                r2 += (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
            }
        }
        r2 = block_sum_d(r2, red);
        err = sqrt(r2) / normM;
        if (!(mode & 1) && err < (double)tol) {
            iters = it;
            break;
        }
        // ---- rows: x_i from the row's samples ----
        for (int i = w; i < m; i += ALS_NW) {
            float g[EPL];
#pragma unroll
            for (int u = 0; u < EPL; ++u) g[u] = 0.f;
            float rhs = 0.f;
            const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
            for (int pb = p0; pb < p1; pb += ALS_B) {
                const int nb = min(ALS_B, p1 - pb);
                for (int e = lane; e < nb * 3 * Q; e += WAVE) {
                    const int b = e / (3 * Q), o = e % (3 * Q);
                    my.stage[e] = Y[(size_t)csr_col[pb + b] * 3 * Q + o];
                }
                wave_lds_sync();
                for (int b = 0; b < nb; ++b) {
                    const float *ys = my.stage + b * 3 * Q;
#pragma unroll
                    for (int u = 0; u < EPL; ++u) {
                        const int e = lane + u * WAVE;
                        if (e < Q * Q) {
                            const int a = e / Q, c = e % Q;
                            g[u] += ys[a] * ys[c] + ys[Q + a] * ys[Q + c] + ys[2 * Q + a] * ys[2 * Q + c];
                        }
                    }
                    if (lane < Q) {
                        const float *v = csr_val + 3 * (pb + b);
                        rhs += (v[0] * inv_s0) * ys[lane] + (v[1] * inv_s0) * ys[Q + lane] +
                               (v[2] * inv_s0) * ys[2 * Q + lane];
                    }
                }
                wave_lds_sync();
            }
            const double shift = (double)lam * (double)max(1, 3 * (p1 - p0));
#pragma unroll
            for (int u = 0; u < EPL; ++u) {
                const int e = lane + u * WAVE;
                if (e < Q * Q) my.A[e] = (double)g[u] + (e / Q == e % Q ? shift : 0.0);
            }
            if (lane < Q) my.b[lane] = (double)rhs;
            wave_lds_sync();
            wave_chol_solve<Q>(my.A, my.b, 1, lane);
            if (lane < Q) X[(size_t)i * Q + lane] = lane < qr ? (float)my.b[lane] : 0.f;
            wave_lds_sync();
        }
        __threadfence_block();
        __syncthreads();
        // ---- columns: y_{c, j} for the three channels of column j ----
        for (int j = w; j < n; j += ALS_NW) {
            float g[EPL];
#pragma unroll
            for (int u = 0; u < EPL; ++u) g[u] = 0.f;
            float r0 = 0.f, r1 = 0.f, r2c = 0.f;
            const int p0 = col_ptr[j], p1 = col_ptr[j + 1];
            for (int pb = p0; pb < p1; pb += ALS_B) {
                const int nb = min(ALS_B, p1 - pb);
                for (int e = lane; e < nb * Q; e += WAVE) {
                    const int b = e / Q, o = e % Q;
                    my.stage[e] = X[(size_t)csc_row[pb + b] * Q + o];
                }
                wave_lds_sync();
                for (int b = 0; b < nb; ++b) {
                    const float *xs = my.stage + b * Q;
#pragma unroll
                    for (int u = 0; u < EPL; ++u) {
                        const int e = lane + u * WAVE;
                        if (e < Q * Q) g[u] += xs[e / Q] * xs[e % Q];
                    }
                    if (lane < Q) {
                        const float *v = csc_val + 3 * (pb + b);
                        const float x = xs[lane];
                        r0 += (v[0] * inv_s0) * x;
                        r1 += (v[1] * inv_s0) * x;
                        r2c += (v[2] * inv_s0) * x;
                    }
                }
                wave_lds_sync();
            }
            const double shift = (double)lam * (double)max(1, p1 - p0);
#pragma unroll
            for (int u = 0; u < EPL; ++u) {
                const int e = lane + u * WAVE;
                if (e < Q * Q) my.A[e] = (double)g[u] + (e / Q == e % Q ? shift : 0.0);
            }
            if (lane < Q) {
                my.b[lane] = (double)r0;
                my.b[Q + lane] = (double)r1;
                my.b[2 * Q + lane] = (double)r2c;
            }
            wave_lds_sync();
            wave_chol_solve<Q>(my.A, my.b, 3, lane);
            if (lane < Q) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Y[(size_t)j * 3 * Q + c * Q + lane] = lane < qr ? (float)my.b[c * Q + lane] : 0.f;
            }
            wave_lds_sync();
        }
        __threadfence_block();
        __syncthreads();
    }
    if (t == 0) {
        st[0] = iters;
        if (!(mode & 1) && iters >= max_iter) st[1] |= VPLMC_SLICE_NOT_CONVERGED;
        st[2] = __float_as_int((float)err);
    }
}

template <int Q>
int launch_als_q(hipStream_t st, size_t count, const int32_t *ids, const SliceDesc *desc, const vplmc_params &prm,
                 const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val, const int32_t *col_ptr,
                 const int32_t *csc_row, const float *csc_val, float *X, float *Y, float *scale, int32_t *stats) {
    if (count == 0) return VPLMC_OK;
    const int32_t mode = ((prm.flags & VPLMC_FIXED_ITERS) ? 1 : 0) | ((prm.flags & VPLMC_GIVEN_INIT) ? 2 : 0);
    hipLaunchKernelGGL(k_als<Q>, dim3((unsigned)count), dim3(ALS_THREADS), 0, st, desc, ids, prm.seed, prm.max_iter,
                       mode, prm.tol, prm.lam, row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, X, Y, scale,
                       stats);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace

int launch_als(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *ids_dev,
               const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
               const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Y, float *scale,
               int32_t *stats) {
    // with ALS every slice is in its rank bucket's global-memory group (2 b + 1)
    size_t base[9] = {0};
    for (int g = 0; g < 8; ++g) base[g + 1] = base[g] + plan.groups[g].size();
    int rc = VPLMC_OK;
#define VPLMC_ALS_BUCKET(B, Q)                                                                                   \
    if (!rc)                                                                                                     \
        rc = launch_als_q<Q>(st, plan.groups[2 * B + 1].size(), ids_dev + base[2 * B + 1], desc, prm, row_ptr,   \
                             csr_col, csr_val, col_ptr, csc_row, csc_val, X, Y, scale, stats);
    VPLMC_ALS_BUCKET(3, 32)
    VPLMC_ALS_BUCKET(2, 16)
    VPLMC_ALS_BUCKET(1, 8)
    VPLMC_ALS_BUCKET(0, 4)
#undef VPLMC_ALS_BUCKET
    return rc;
}

}  // namespace vplmc
