// Learned second-pass proposal: per-(slice, column) features from the first
// pass, a 12 -> 128 -> 128 -> 1 GELU network predicting the log of a column
// sampling density, its training (softmax-KL loss, backward, Adam) and the
// training targets from fully evaluated slices.  The paper samples columns by
// g(j) = max C_j - min C_j because columns whose results vary are important
// (Sec. 5) and names image-space-guided sampling as future work (Sec. 7);
// the network estimates that importance from the same sparse observations.
//
// Weights are used rounded to bfloat16 (round to nearest even) and the two
// hidden activations are rounded to bfloat16; accumulation is FP32.  The
// 128 x 128 layer of inference runs on MFMA (v_mfma_f32_32x32x8 bf16): one
// wavefront owns 32 rows, computes their layer-1 activations directly in
// the MFMA A-operand layout, and reduces the output layer across lanes.
// Training uses FP32 VALU kernels with the same rounding points.

#include <type_traits>

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr int WAVE = 64;
constexpr float SQRT_2_OVER_PI = 0.7978845608028654f;

// parameter offsets in the flat FP32 vector (W1 b1 W2 b2 W3 b3)
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + MLP_HID * MLP_IN;
constexpr int P_W2 = P_B1 + MLP_HID;
constexpr int P_B2 = P_W2 + MLP_HID * MLP_HID;
constexpr int P_W3 = P_B2 + MLP_HID;
constexpr int P_B3 = P_W3 + MLP_HID;

__device__ __forceinline__ float bf16r(float x) {
    uint32_t u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint16_t bf16bits(float x) { return (uint16_t)(__float_as_uint(bf16r(x)) >> 16); }

__device__ __forceinline__ float gelu(float x) {
    return 0.5f * x * (1.0f + tanhf(SQRT_2_OVER_PI * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float u = SQRT_2_OVER_PI * (x + 0.044715f * x * x * x);
    const float th = tanhf(u);
    const float du = SQRT_2_OVER_PI * (1.0f + 3.0f * 0.044715f * x * x);
    return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * du;
}

// ---------------------------------------------------------------------------
// features: one workgroup per slice
//   mu = first-pass mean of t; per column j:
//   0 log1p(mean/mu) 1 log1p(std/mu) 2 log1p((max-min)/mu) 3 count/(N1/n)
//   4 zero fraction 5 log1p(cluster bbox diag / dist) 6 log1p(dist / slice diag)
//   7 cos(slice mean normal, slice->cluster) 8 cos(cluster normal, cluster->slice)
//   9 log1p(I_c / mean I over the cut) 10 log(members) 11 1 - |slice mean normal|
// Member counts come from the cut's offsets, or (light coarsening: columns
// are tree nodes) from node_members.
__global__ __launch_bounds__(256) void k_features(const SliceDesc *__restrict__ desc, vplmc_points pts,
                                                  const int32_t *__restrict__ pt_ids,
                                                  const int32_t *__restrict__ cl_ids, const float *__restrict__ lights,
                                                  int32_t nc, const float *__restrict__ bbox, vplmc_cut cut,
                                                  const int32_t *__restrict__ node_members,
                                                  const int32_t *__restrict__ cnt, const float *__restrict__ mn,
                                                  const float *__restrict__ mx, const double *__restrict__ sum,
                                                  const double *__restrict__ sumsq, const int32_t *__restrict__ zeros,
                                                  float *__restrict__ geo_out, float *__restrict__ F) {
    __shared__ double red[8][256];
    __shared__ float geo[8];
    __shared__ double mu_s, imean_s;
    const int s = blockIdx.x;
    const SliceDesc d = desc[s];
    const int t = threadIdx.x;
    const size_t N = (size_t)nc;
    // slice geometry and first-pass mean, fixed-order reductions
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = t; i < d.m; i += 256) {
        const int p = clamp_index(pt_ids[d.pt_off + i], pts.m);
        const float x = pts.px[p], y = pts.py[p], z = pts.pz[p];
        a[0] += x; a[1] += y; a[2] += z;
        a[3] += pts.nx[p]; a[4] += pts.ny[p]; a[5] += pts.nz[p];
        lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
        hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
    }
    for (int j = t; j < d.n; j += 256) {
        a[6] += sum[d.off_col + j];
        const int c = clamp_index(cl_ids[d.cl_off + j], nc);
        a[7] += (double)((lights[6 * N + c] + lights[7 * N + c]) + lights[8 * N + c]);
    }
    for (int k = 0; k < 8; ++k) red[k][t] = a[k];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 8; ++k) red[k][t] += red[k][t + w];
        __syncthreads();
    }
    // bbox: reuse the reduction for min / max (as doubles)
    double bl[3] = {lo[0], lo[1], lo[2]}, bh[3] = {hi[0], hi[1], hi[2]};
    double tot[8];
    for (int k = 0; k < 8; ++k) tot[k] = red[k][0];
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        red[k][t] = bl[k];
        red[3 + k][t] = bh[k];
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 3; ++k) {
                red[k][t] = fmin(red[k][t], red[k][t + w]);
                red[3 + k][t] = fmax(red[3 + k][t], red[3 + k][t + w]);
            }
        __syncthreads();
    }
    if (t == 0) {
        const double im = 1.0 / (double)d.m;
        const double dx = red[3][0] - red[0][0], dy = red[4][0] - red[1][0], dz = red[5][0] - red[2][0];
        geo[0] = (float)(tot[0] * im);
        geo[1] = (float)(tot[1] * im);
        geo[2] = (float)(tot[2] * im);
        geo[3] = (float)sqrt(dx * dx + dy * dy + dz * dz);
        geo[4] = (float)(tot[3] * im);
        geo[5] = (float)(tot[4] * im);
        geo[6] = (float)(tot[5] * im);
        geo[7] = 0.f;
        const double mu = tot[6] / (double)(d.N1 > 0 ? d.N1 : 1);
        mu_s = mu > 0.0 ? mu : 1e-30;
        imean_s = tot[7] / (double)d.n;
        for (int k = 0; k < 8; ++k) geo_out[8 * s + k] = geo[k];
    }
    __syncthreads();
    const float cx = geo[0], cy = geo[1], cz = geo[2];
    const float diag = geo[3] + 1e-6f;
    const float mnx = geo[4], mny = geo[5], mnz = geo[6];
    const float nn = sqrtf(mnx * mnx + mny * mny + mnz * mnz) + 1e-12f;
    const double mu = mu_s;
    const float per = (float)d.N1 / (float)d.n;
    for (int j = t; j < d.n; j += 256) {
        const int64_t o = d.off_col + j;
        const int c = clamp_index(cl_ids[d.cl_off + j], nc);
        const float k = (float)cnt[o];
        const float safe = k > 0.f ? k : 1.f;
        const double mean = sum[o] / (double)safe;
        const double var = fmax(0.0, sumsq[o] / (double)safe - mean * mean);
        float *f = F + 12 * o;
        f[0] = (float)log1p(mean / mu);
        f[1] = (float)log1p(sqrt(var) / mu);
        f[2] = (float)log1p((double)(k > 0.f ? mx[o] - mn[o] : 0.f) / mu);
        f[3] = k / (per > 0.f ? per : 1.f);
        f[4] = k > 0.f ? (float)zeros[o] / safe : 0.f;
        const float px = lights[c] - cx, py = lights[N + c] - cy, pz = lights[2 * N + c] - cz;
        const float dist = sqrtf(px * px + py * py + pz * pz) + 1e-6f;
        const float ux = px / dist, uy = py / dist, uz = pz / dist;
        const float bx = bbox[3 * N + c] - bbox[c], by = bbox[4 * N + c] - bbox[N + c], bz = bbox[5 * N + c] - bbox[2 * N + c];
        f[5] = log1pf(sqrtf(bx * bx + by * by + bz * bz) / dist);
        f[6] = log1pf(dist / diag);
        f[7] = (ux * mnx + uy * mny + uz * mnz) / nn;
        f[8] = -(lights[3 * N + c] * ux + lights[4 * N + c] * uy + lights[5 * N + c] * uz);
        const double is = (double)((lights[6 * N + c] + lights[7 * N + c]) + lights[8 * N + c]);
        f[9] = (float)log1p(is / (imean_s + 1e-30));
        f[10] = logf((float)(node_members ? node_members[c] : cut.offsets[c + 1] - cut.offsets[c]));
        f[11] = 1.0f - nn;
    }
}

// ---------------------------------------------------------------------------
// inference: one wavefront = 32 rows; layer 2 on MFMA 32x32x8 bf16
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ P, int64_t rows,
                                                     const float *__restrict__ F, float *__restrict__ y) {
    __shared__ float w1s[MLP_HID * MLP_IN];
    __shared__ float b1s[MLP_HID];
    __shared__ uint16_t w2s[MLP_HID * MLP_HID];   // bf16 bits, [h][k]
    __shared__ float b2s[MLP_HID], w3s[MLP_HID];
    const int t = threadIdx.x;
    for (int e = t; e < MLP_HID * MLP_IN; e += 256) w1s[e] = bf16r(P[P_W1 + e]);
    for (int e = t; e < MLP_HID; e += 256) {
        b1s[e] = P[P_B1 + e];
        b2s[e] = P[P_B2 + e];
        w3s[e] = bf16r(P[P_W3 + e]);
    }
    for (int e = t; e < MLP_HID * MLP_HID; e += 256) w2s[e] = bf16bits(P[P_W2 + e]);
    __syncthreads();
    const float b3 = P[P_B3];
    const int lane = t % WAVE, wave = t / WAVE;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
    if (r0 >= rows) return;
    const int i = lane % 32;          // A-operand row of this lane
    const int kh = lane / 32;         // which 4-wide k half of each 8-wide step
    const int64_t row = r0 + i;
    float f[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) f[q] = row < rows ? F[12 * row + q] : 0.f;
    // layer 1 in the A layout: step ks covers k = 8 ks + 4 kh + {0..3}
    short4_t A[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        short4_t v;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = 8 * ks + 4 * kh + c;
            float z = b1s[k];
#pragma unroll
            for (int q = 0; q < MLP_IN; ++q) z = fmaf(w1s[k * MLP_IN + q], f[q], z);
            v[c] = (short)bf16bits(gelu(z));
        }
        A[ks] = v;
    }
    // layer 2 (MFMA) and the output layer, four 32-column tiles of hidden units
    float part[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) part[v] = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int h = nt * 32 + (lane % 32);  // B-operand column / C column of this lane
        float16_t acc = {};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            short4_t b;
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = (short)w2s[h * MLP_HID + 8 * ks + 4 * kh + c];
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[ks], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float h2 = bf16r(gelu(acc[v] + b2s[h]));
            part[v] = fmaf(w3s[h], h2, part[v]);
        }
    }
    // sum over the 32 hidden-unit lanes of each half-wave
#pragma unroll
    for (int v = 0; v < 16; ++v) {
#pragma unroll
        for (int o = 16; o >= 1; o >>= 1) part[v] += __shfl_xor(part[v], o, WAVE);
    }
    if (lane % 32 == 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = (v / 4) * 8 + kh * 4 + (v % 4);   // C row of accumulator v
            if (r0 + r < rows) y[r0 + r] = part[v] + b3;
        }
    }
}

// ---------------------------------------------------------------------------
// training: FP32 VALU, tiles of TR rows, one thread per hidden unit
constexpr int TR = 32;

__global__ __launch_bounds__(128) void k_train_forward(const float *__restrict__ P, int64_t rows,
                                                       const float *__restrict__ F, float *__restrict__ y,
                                                       float *__restrict__ cache) {
    __shared__ float fs[TR][MLP_IN];
    __shared__ float h1s[TR][MLP_HID];
    __shared__ float part[TR][2];
    const int h = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TR;
    for (int e = h; e < TR * MLP_IN; e += 128) {
        const int64_t r = r0 + e / MLP_IN;
        fs[e / MLP_IN][e % MLP_IN] = r < rows ? F[12 * r + e % MLP_IN] : 0.f;
    }
    __syncthreads();
    float w1[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) w1[q] = bf16r(P[P_W1 + h * MLP_IN + q]);
    const float b1 = P[P_B1 + h], b2 = P[P_B2 + h], w3 = bf16r(P[P_W3 + h]);
    for (int r = 0; r < TR; ++r) {
        float z = b1;
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) z = fmaf(w1[q], fs[r][q], z);
        const float a = bf16r(gelu(z));
        h1s[r][h] = a;
        const int64_t rr = r0 + r;
        if (rr < rows) {
            cache[(rr * 4 + 0) * MLP_HID + h] = z;
            cache[(rr * 4 + 1) * MLP_HID + h] = a;
        }
    }
    __syncthreads();
    for (int r = 0; r < TR; ++r) {
        float z = b2;
        for (int k = 0; k < MLP_HID; ++k) z = fmaf(bf16r(P[P_W2 + h * MLP_HID + k]), h1s[r][k], z);
        const float a = bf16r(gelu(z));
        const int64_t rr = r0 + r;
        if (rr < rows) {
            cache[(rr * 4 + 2) * MLP_HID + h] = z;
            cache[(rr * 4 + 3) * MLP_HID + h] = a;
        }
        float pv = w3 * a;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) pv += __shfl_xor(pv, o, WAVE);
        if (h % WAVE == 0) part[r][h / WAVE] = pv;
    }
    __syncthreads();
    if (h < TR && r0 + h < rows) y[r0 + h] = (part[h][0] + part[h][1]) + P[P_B3];
}

// per group (slice): q = softmax(y), loss += KL(p* || q), dy = q - p*
__global__ __launch_bounds__(256) void k_softmax_kl(const float *__restrict__ y, const float *__restrict__ pstar,
                                                    const int32_t *__restrict__ goff, float *__restrict__ dy,
                                                    float *__restrict__ loss) {
    __shared__ float red[256];
    const int g = blockIdx.x, t = threadIdx.x;
    const int b = goff[g], e = goff[g + 1];
    float mxv = -INFINITY;
    for (int r = b + t; r < e; r += 256) mxv = fmaxf(mxv, y[r]);
    red[t] = mxv;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] = fmaxf(red[t], red[t + w]);
        __syncthreads();
    }
    const float ym = red[0];
    __syncthreads();
    float se = 0.f;
    for (int r = b + t; r < e; r += 256) se += expf(y[r] - ym);
    red[t] = se;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const float lse = ym + logf(red[0]);
    __syncthreads();
    float l = 0.f;
    for (int r = b + t; r < e; r += 256) {
        const float lq = y[r] - lse;
        const float p = pstar[r];
        if (p > 0.f) l += p * (logf(p) - lq);
        dy[r] = expf(lq) - p;
    }
    red[t] = l;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) atomicAdd(loss, red[0]);
}

// gradients of sum(dy * y); straight-through at the bf16 rounding points
__global__ __launch_bounds__(128) void k_train_backward(const float *__restrict__ P, int64_t rows,
                                                        const float *__restrict__ F, const float *__restrict__ dy,
                                                        const float *__restrict__ cache, float *__restrict__ G) {
    __shared__ float fs[TR][MLP_IN];
    __shared__ float h1s[TR][MLP_HID];
    __shared__ float dz2s[TR][MLP_HID];
    __shared__ float dys[TR];
    const int h = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TR;
    for (int e = h; e < TR * MLP_IN; e += 128) {
        const int64_t r = r0 + e / MLP_IN;
        fs[e / MLP_IN][e % MLP_IN] = r < rows ? F[12 * r + e % MLP_IN] : 0.f;
    }
    if (h < TR) dys[h] = r0 + h < rows ? dy[r0 + h] : 0.f;
    const float w3 = bf16r(P[P_W3 + h]);
    float gw3 = 0.f, gb2 = 0.f;
    for (int r = 0; r < TR; ++r) {
        const int64_t rr = r0 + r;
        const bool ok = rr < rows;
        const float z2 = ok ? cache[(rr * 4 + 2) * MLP_HID + h] : 0.f;
        const float a2 = ok ? cache[(rr * 4 + 3) * MLP_HID + h] : 0.f;
        h1s[r][h] = ok ? cache[(rr * 4 + 1) * MLP_HID + h] : 0.f;
        __syncthreads();
        const float d = dys[r];
        const float dz2 = d * w3 * gelu_grad(z2);
        dz2s[r][h] = dz2;
        gw3 = fmaf(d, a2, gw3);
        gb2 += dz2;
    }
    __syncthreads();
    atomicAdd(G + P_W3 + h, gw3);
    atomicAdd(G + P_B2 + h, gb2);
    if (h == 0) {
        float s = 0.f;
        for (int r = 0; r < TR; ++r) s += dys[r];
        atomicAdd(G + P_B3, s);
    }
    // dW2[h][k] = sum_r dz2[r][h] h1[r][k]
    for (int k = 0; k < MLP_HID; ++k) {
        float s = 0.f;
        for (int r = 0; r < TR; ++r) s = fmaf(dz2s[r][h], h1s[r][k], s);
        atomicAdd(G + P_W2 + h * MLP_HID + k, s);
    }
    // thread h now plays hidden unit k = h of layer 1: dh1[r][k] = sum_j dz2[r][j] W2[j][k]
    const int k = h;
    float gb1 = 0.f, gw1[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) gw1[q] = 0.f;
    for (int r = 0; r < TR; ++r) {
        const int64_t rr = r0 + r;
        float dh1 = 0.f;
        for (int j = 0; j < MLP_HID; ++j) dh1 = fmaf(dz2s[r][j], bf16r(P[P_W2 + j * MLP_HID + k]), dh1);
        const float z1 = rr < rows ? cache[(rr * 4 + 0) * MLP_HID + k] : 0.f;
        const float dz1 = dh1 * gelu_grad(z1);
        gb1 += dz1;
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) gw1[q] = fmaf(dz1, fs[r][q], gw1[q]);
    }
    atomicAdd(G + P_B1 + k, gb1);
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) atomicAdd(G + P_W1 + k * MLP_IN + q, gw1[q]);
}

// Adam (Kingma & Ba) with bias correction; step counts from 1
__global__ void k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M,
                       float *__restrict__ V, int32_t step, float lr) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MLP_PARAMS) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = G[e];
    const float m = b1 * M[e] + (1.f - b1) * g;
    const float v = b2 * V[e] + (1.f - b2) * g * g;
    M[e] = m;
    V[e] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    P[e] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_zero(float *p, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.f;
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

int launch_features(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const vplmc_points &pts,
                    const int32_t *pt_ids, const int32_t *cl_ids, const float *lights, const float *bbox,
                    const vplmc_cut &cut, const int32_t *node_members, const int32_t *cnt, const float *mn,
                    const float *mx, const double *sum, const double *sumsq, const int32_t *zeros, float *slice_geo,
                    float *features) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_features, dim3(plan.n_slices), dim3(256), 0, st, desc, pts, pt_ids, cl_ids, lights,
                       plan.n_lights, bbox, cut, node_members, cnt, mn, mx, sum, sumsq, zeros, slice_geo, features);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_mlp_forward(hipStream_t st, const float *params, int64_t rows, const float *features, float *y) {
    if (rows <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(rows, 128)), dim3(256), 0, st, params, rows, features, y);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_mlp_grad(hipStream_t st, const float *params, int64_t rows, const float *features, const float *dy,
                    float *grad, float *y, float *cache) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(MLP_PARAMS, 256)), dim3(256), 0, st, grad, MLP_PARAMS);
    VPLMC_HIP(hipGetLastError());
    if (rows <= 0) return VPLMC_OK;
    hipLaunchKernelGGL(k_train_forward, dim3(blocks_for(rows, TR)), dim3(128), 0, st, params, rows, features, y, cache);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_train_backward, dim3(blocks_for(rows, TR)), dim3(128), 0, st, params, rows, features, dy,
                       cache, grad);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_mlp_train_step(hipStream_t st, float *params, float *m, float *v, int32_t step, float lr, int64_t rows,
                          const float *features, const float *pstar, int32_t n_groups, const int32_t *group_off,
                          float *y, float *dy, float *grad, float *loss, float *cache) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(MLP_PARAMS, 256)), dim3(256), 0, st, grad, MLP_PARAMS);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(32), 0, st, loss, 1);
    VPLMC_HIP(hipGetLastError());
    if (rows > 0) {
        hipLaunchKernelGGL(k_train_forward, dim3(blocks_for(rows, TR)), dim3(128), 0, st, params, rows, features, y,
                           cache);
        hipLaunchKernelGGL(k_softmax_kl, dim3(n_groups), dim3(256), 0, st, y, pstar, group_off, dy, loss);
        hipLaunchKernelGGL(k_train_backward, dim3(blocks_for(rows, TR)), dim3(128), 0, st, params, rows, features, dy,
                           cache, grad);
        VPLMC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(MLP_PARAMS, 256)), dim3(256), 0, st, params, grad, m, v, step, lr);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_mlp_adam(hipStream_t st, float *params, const float *grad, float *m, float *v, int32_t step, float lr) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(MLP_PARAMS, 256)), dim3(256), 0, st, params, grad, m, v, step, lr);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
