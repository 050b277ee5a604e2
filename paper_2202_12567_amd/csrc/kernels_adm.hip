// Non-negative completion of each slice matrix by the alternating direction
// method (Appendix A), and the factorised column sum I(s) = X (Y e)
// (Sec. 3, step 5).
//
// A slice whose X fits in LDS is completed by one workgroup for all its
// iterations (k_adm_ell), so an iteration needs only workgroup barriers; the
// others (rank 32, tall slices) by a sequence of launches per iteration over
// all such slices (k_gadm_*, kernels_gadm.hip).  The slice matrix is the stacked
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
//     V_j = max(0, Y+_j + P_j / b), P_j += g b (Y+_j - V_j);
//   GY = Y+ Y+^T for the next iteration, Y streamed through LDS tiles.
// The q x q systems are factored by Cholesky in FP64 and inverted once per
// iteration; phase A multiplies by the FP64 inverse, phase B by its FP32
// rounding.
// Every reduction has a fixed order: results are bitwise reproducible.

#include <algorithm>
#include "adm_common.h"

namespace vplmc {
namespace {

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
    int rc = launch_gadm_group(sb[3], 32, plan, 7, id[7], gblk_dev, gsys, ge2, desc, prm, row_ptr, csr_col,
                               csr_val, col_ptr, csc_row, csc_val, X, Xn, Xp, Lam, Y, Yp, Pi, scale, stats);
#define VPLMC_ADM_PAIR(B, Q, TG)                                                                                      \
    if (!rc)                                                                                                          \
        rc = launch_adm_ell<Q>(sb[B], thr, plan.groups[2 * B].size(), plan.group_max_m[2 * B], id[2 * B], qp(2 * B), \
                               n_cu, desc, prm, col_ptr, ell, X, Xp, Lam, Y, Yp, Pi, Yt, red, e2part, scale, stats); \
    if (!rc)                                                                                                          \
        rc = launch_gadm_group(sb[B], Q, plan, 2 * B + 1, id[2 * B + 1], gblk_dev, gsys, ge2, desc, prm, row_ptr,  \
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
