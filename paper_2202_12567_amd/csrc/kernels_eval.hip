// Lighting-matrix entries A(i, j) (Sec. 3): the contribution of a point
// light to a surface point, with a shadow ray against the occluder BVH
// (visibility is the most expensive part of an entry, Sec. 2 and Sec. 6).
//
//   d = y - x, w = d / |d|, c_x = n_x . w, c_y = -n_y . w (0, no ray, if either <= 0)
//   G = c_x c_y / max(|d|^2, r_min^2)
//   f = kd / pi + ks (e + 2) / (2 pi) max(0, w_r . w_o)^e,  w_r = 2 c_x n_x - w
//   A = f * I * G * V
// V = 0 iff the segment from x + eps n_x to y passes within the radius of a
// sphere (closest point of the segment to the centre), found by an any-hit
// traversal of a bounding-volume hierarchy in depth-first order with skip
// indices (no stack).

#include <algorithm>

#include "vplmc_internal.h"
#include "shading.h"

namespace vplmc {
namespace {

// The BVH as read by a traversal: from global memory, or from a copy staged
// in LDS (nodes as pairs of float4, then the spheres).
// KIND: 0 spheres, 1 triangles (Bvh::kind), fixed per kernel instance so that
// the sphere traversal carries no triangle code.
template <int KIND>
struct BvhGlobal {
    static constexpr int kind = KIND;
    const Bvh &b;
    __device__ BvhNode node(int k) const { return b.nodes[k]; }
    __device__ float4 sphere(int k) const { return b.spheres[k]; }
};
template <int KIND>
struct BvhStaged {
    static constexpr int kind = KIND;
    const float4 *lds;   // LDS: 2 n_nodes float4 of nodes, then the spheres or triangles
    int n_nodes;
    __device__ BvhNode node(int k) const {
        const float4 a = lds[2 * k], c = lds[2 * k + 1];
        BvhNode nd;
        nd.lo[0] = a.x;
        nd.lo[1] = a.y;
        nd.lo[2] = a.z;
        nd.leaf = __float_as_int(a.w);
        nd.hi[0] = c.x;
        nd.hi[1] = c.y;
        nd.hi[2] = c.z;
        nd.skip = __float_as_int(c.w);
        return nd;
    }
    __device__ float4 sphere(int k) const { return lds[2 * n_nodes + k]; }
};

// does a triangle reference of a leaf meet the open segment o + t D,
// t in (0, 1): barycentric u, v >= 0, u + v <= 1 of the crossing with the
// triangle's plane (Moller-Trumbore), none for a segment parallel to it
template <typename B>
__device__ __forceinline__ bool leaf_occludes_tri(const B &bvh, int first, int cnt, P3 o, P3 D) {
    bool any = false;
    for (int k = 0; k < cnt; ++k) {
        const float4 a4 = bvh.sphere(3 * (first + k)), b4 = bvh.sphere(3 * (first + k) + 1);
        const float4 c4 = bvh.sphere(3 * (first + k) + 2);
        const P3 e1 = {b4.x, b4.y, b4.z}, e2 = {c4.x, c4.y, c4.z};
        const P3 p = {D.y * e2.z - D.z * e2.y, D.z * e2.x - D.x * e2.z, D.x * e2.y - D.y * e2.x};
        const float det = dot(e1, p);
        const float inv = 1.0f / det;
        const P3 s = {o.x - a4.x, o.y - a4.y, o.z - a4.z};
        const float u = dot(s, p) * inv;
        const P3 q = {s.y * e1.z - s.z * e1.y, s.z * e1.x - s.x * e1.z, s.x * e1.y - s.y * e1.x};
        const float v = dot(D, q) * inv;
        const float t = dot(e2, q) * inv;
        any = any || (det != 0.0f && u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && t < 1.0f);
    }
    return any;
}

// does a sphere of a leaf (first << 4 | count) come closer to the segment
// o + t D, t in [0, 1], than its radius (or, for triangle occluders, does a
// triangle of the leaf meet it)
template <typename B>
__device__ __forceinline__ bool leaf_occludes(const B &bvh, int leaf, P3 o, P3 D, float inv_dd) {
    const int first = leaf >> 4, cnt = leaf & 15;
    if constexpr (B::kind == 1) return leaf_occludes_tri(bvh, first, cnt, o, D);
    bool any = false;
    for (int k = 0; k < cnt; ++k) {
        const float4 sp4 = bvh.sphere(first + k);
        const P3 oc = {sp4.x - o.x, sp4.y - o.y, sp4.z - o.z};
        const float t = fminf(fmaxf(dot(oc, D) * inv_dd, 0.0f), 1.0f);
        const P3 p = {oc.x - t * D.x, oc.y - t * D.y, oc.z - t * D.z};
        any = any || dot(p, p) < sp4.w * sp4.w;
    }
    return any;
}

// any hit on the open segment o + t D, t in (0, 1)
template <typename B>
__device__ __forceinline__ bool occluded_in(const B &bvh, int n_nodes, P3 o, P3 D) {
    if (n_nodes == 0) return false;
    const float dd = dot(D, D);
    const float inv_dd = 1.0f / dd;
    const float ix = 1.0f / (fabsf(D.x) > 1e-20f ? D.x : copysignf(1e-20f, D.x));
    const float iy = 1.0f / (fabsf(D.y) > 1e-20f ? D.y : copysignf(1e-20f, D.y));
    const float iz = 1.0f / (fabsf(D.z) > 1e-20f ? D.z : copysignf(1e-20f, D.z));
    int node = 0;
    while (node < n_nodes) {
        const BvhNode nd = bvh.node(node);
        const float tx0 = (nd.lo[0] - o.x) * ix, tx1 = (nd.hi[0] - o.x) * ix;
        const float ty0 = (nd.lo[1] - o.y) * iy, ty1 = (nd.hi[1] - o.y) * iy;
        const float tz0 = (nd.lo[2] - o.z) * iz, tz1 = (nd.hi[2] - o.z) * iz;
        const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
        const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), 1.0f));
        const bool hit = tmin <= tmax;
        if (hit && nd.leaf != 0 && leaf_occludes(bvh, nd.leaf, o, D, inv_dd)) return true;
        // an inner node that is hit descends to its left child; anything else
        // continues after its subtree
        node = hit && nd.leaf == 0 ? node + 1 : nd.skip;
    }
    return false;
}


// entry of one (point, light) pair (zero when the pair faces away or is
// occluded); bvh is a BVH view (BvhGlobal or BvhStaged) of n_nodes nodes.
// Returns whether a shadow ray was cast (both cosines positive).
template <typename B>
__device__ __forceinline__ bool shade_in(const B &bvh, int n_nodes, const PointData &q, const Light &L,
                                         float r_min2, float eps, float &o0, float &o1, float &o2) {
    o0 = o1 = o2 = 0.0f;
    const P3 d = sub(L.y, q.x);
    const float r2 = dot(d, d);
    const float inv_r = 1.0f / sqrtf(r2);
    const P3 w = {d.x * inv_r, d.y * inv_r, d.z * inv_r};
    const float cx = dot(q.n, w);
    const float cy = -dot(L.n, w);
    if (!(cx > 0.0f && cy > 0.0f)) return false;
    const float G = cx * cy / fmaxf(r2, r_min2);
    float spec = 0.0f;
    if (q.ks > 0.0f) {
        const P3 wr = {2.0f * cx * q.n.x - w.x, 2.0f * cx * q.n.y - w.y, 2.0f * cx * q.n.z - w.z};
        const float cr = fmaxf(0.0f, dot(wr, q.wo));
        spec = q.ks * (q.e + 2.0f) * (0.5f * INV_PI) * powf(cr, q.e);
    }
    const P3 o = {fmaf(eps, q.n.x, q.x.x), fmaf(eps, q.n.y, q.x.y), fmaf(eps, q.n.z, q.x.z)};
    if (occluded_in(bvh, n_nodes, o, sub(L.y, o))) return true;
    o0 = fmaf(q.kd0, INV_PI, spec) * L.i0 * G;
    o1 = fmaf(q.kd1, INV_PI, spec) * L.i1 * G;
    o2 = fmaf(q.kd2, INV_PI, spec) * L.i2 * G;
    return true;
}

template <int KIND>
__device__ __forceinline__ bool shade(const Bvh &bvh, const PointData &q, const Light &L, float r_min2,
                                      float eps, float &o0, float &o1, float &o2) {
    return shade_in(BvhGlobal<KIND>{bvh}, bvh.n_nodes, q, L, r_min2, eps, o0, o1, o2);
}

// adds a per-thread count into a device total: one atomic per wavefront
__device__ __forceinline__ void add_count(unsigned long long *total, uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(total, (unsigned long long)v);
}

__device__ __forceinline__ int slice_of_off(const SliceDesc *__restrict__ desc, int S, int64_t g, int which) {
    int lo = 0, hi = S;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const int64_t o = which ? desc[mid].off2 : desc[mid].off1;
        if (o <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// entry of sample g of one pass (nothing for slots past the slice's first-pass
// count or its accepted second-pass count)
template <bool STAGED, int KIND>
__device__ __forceinline__ uint32_t eval_one(const Bvh &bvh, const BvhStaged<KIND> &staged, const vplmc_points &pts,
                                         const float *__restrict__ lights, int32_t n_lights,
                                         const SliceDesc *__restrict__ desc, int S, const int32_t *__restrict__ pt_ids,
                                         const int32_t *__restrict__ cl_ids, const uint32_t *__restrict__ keys,
                                         int64_t g, int which, const int32_t *__restrict__ stats, float r_min2,
                                         float eps, float *__restrict__ vals) {
    const int s = slice_of_off(desc, S, g, which);
    const SliceDesc d = desc[s];
    if (which ? g - d.off2 >= stats[4 * s + 3] : g - d.off1 >= d.N1) return 0;
    const uint32_t key = keys[g];
    const int i = (int)(key >> 16), j = (int)(key & 0xFFFFu);
    const int pid = pt_ids[d.pt_off + i];
    const int c = clamp_index(cl_ids[d.cl_off + j], n_lights);
    const size_t N = (size_t)n_lights;
    const Light L = {{lights[c], lights[N + c], lights[2 * N + c]},
                     {lights[3 * N + c], lights[4 * N + c], lights[5 * N + c]},
                     lights[6 * N + c], lights[7 * N + c], lights[8 * N + c]};
    const PointData q = load_point(pts, pid);
    float o0, o1, o2;
    bool ray;
    if (STAGED)
        ray = shade_in(staged, bvh.n_nodes, q, L, r_min2, eps, o0, o1, o2);
    else
        ray = shade<KIND>(bvh, q, L, r_min2, eps, o0, o1, o2);
    vals[3 * g] = o0;
    vals[3 * g + 1] = o1;
    vals[3 * g + 2] = o2;
    return ray ? 1u : 0u;
}

// BVH bytes (nodes and spheres) an entry kernel stages in LDS; larger ones are
// read from global memory
constexpr int EVAL_LDS_BYTES = 48 * 1024;
// workgroups per compute unit of an entry launch
constexpr int EVAL_GRID_PER_CU = 16;

// entries of one pass's samples (draw order), lights = cluster table planes;
// a fixed grid walks the samples, each workgroup first copying the BVH to LDS
// when STAGED
template <bool STAGED, int KIND>
__global__ __launch_bounds__(256) void k_eval_omega(Bvh bvh, vplmc_points pts, const float *__restrict__ lights,
                                                    int32_t n_lights, const SliceDesc *__restrict__ desc, int S,
                                                    const int32_t *__restrict__ pt_ids,
                                                    const int32_t *__restrict__ cl_ids,
                                                    const uint32_t *__restrict__ keys, int64_t n_keys,
                                                    int which, const int32_t *__restrict__ stats, float r_min2,
                                                    float eps, float *__restrict__ vals,
                                                    unsigned long long *__restrict__ rays) {
    extern __shared__ float4 stage[];
    if (STAGED) {
        const int nn = 2 * bvh.n_nodes, ns = bvh.n_spheres;
        const float4 *nodes4 = reinterpret_cast<const float4 *>(bvh.nodes);
        for (int k = threadIdx.x; k < nn + ns; k += blockDim.x) stage[k] = k < nn ? nodes4[k] : bvh.spheres[k - nn];
        __syncthreads();
    }
    const BvhStaged<KIND> staged{stage, bvh.n_nodes};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t traced = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_keys; g += stride) {
        traced += eval_one<STAGED, KIND>(bvh, staged, pts, lights, n_lights, desc, S, pt_ids, cl_ids, keys, g, which, stats,
                                   r_min2, eps, vals);
    }
    if (rays) add_count(rays, traced);
}

// Merge errors of the per-slice light coarsening (Sec. 4).  One thread per
// row draw (slice s, draw r; r < kpre[n_g]): the draw belongs to leaf x
// (kpre[x] <= r < kpre[x + 1]) and is its k-th, k = r - kpre[x] < m'; its row
// is the k-th image of leaf x's keyed permutation of [0, m') (4-round
// Feistel, round function Philox(key = (seed, s), ctr = (R, round, TAG_ZETA,
// x)) & mask, cycle-walked).  Walking from x to the root, the thread carries
// S(i, rep of the current node) at unit intensity; at each split node f
// (kept child a, dropped b) one new entry gives the other child's, and
// I_b |S(i, rep_b) - S(i, rep_a)| (max over channels) goes into eps(f) by an
// integer max (non-negative floats order as their bits).  A node's light is
// its kept child's, so the carried value becomes S(i, rep_a).  Every node's
// eps is thus the max over the union of its leaves' draws, each pixel
// evaluated once per level (the reuse Sec. 4 describes).
__device__ __forceinline__ uint64_t feistel_zeta(uint64_t v, uint64_t seed, uint64_t s, uint64_t x, int h) {
    const uint64_t mask = (1ull << h) - 1ull;
    uint64_t L = v >> h, R = v & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t F = philox(seed, s, R, (uint64_t)r, TAG_ZETA, x).a & mask;
        const uint64_t nL = R;
        R = L ^ F;
        L = nL;
    }
    return (L << h) | R;
}


// six wavefronts per SIMD (80 VGPRs): the walk's latency needs the occupancy;
// at 83 VGPRs (five) the kernel ran 14% slower on the 1080p frame
template <bool STAGED, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_coarsen_eps(Bvh bvh, vplmc_points pts, const float *__restrict__ lights,
                                                     const SliceDesc *__restrict__ desc, int64_t total, int64_t K,
                                                     const int32_t *__restrict__ pt_ids, CoarsenTree tr,
                                                     CoarsenSlices cs, uint64_t seed, float r_min2, float eps,
                                                     unsigned long long *__restrict__ counts) {
    extern __shared__ float4 stage[];
    if (STAGED) {
        const int nn = 2 * bvh.n_nodes, ns = bvh.n_spheres;
        const float4 *nodes4 = reinterpret_cast<const float4 *>(bvh.nodes);
        for (int k = threadIdx.x; k < nn + ns; k += blockDim.x) stage[k] = k < nn ? nodes4[k] : bvh.spheres[k - nn];
        __syncthreads();
    }
    const BvhStaged<KIND> staged{stage, bvh.n_nodes};
    const int ng = tr.n_leaves;
    const size_t N = (size_t)(2 * ng - 1);
    const int64_t kt = cs.kpre[ng];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t n_eval = 0, n_ray = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += stride) {
        const int s = (int)(g / K);
        const int64_t r = g - (int64_t)s * K;
        if (r >= kt) continue;
        const SliceDesc d = desc[s];
        int lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cs.kpre[mid] <= r) lo = mid; else hi = mid;
        }
        const int x = lo;
        const int64_t k = r - cs.kpre[x];
        if (k >= d.m) continue;
        // row of the draw
        const uint64_t m = (uint64_t)d.m;
        int b = m > 1 ? 64 - __clzll((long long)(m - 1)) : 0;
        b = b < 2 ? 2 : b;
        const int h = (b + 1) / 2;
        uint64_t e = feistel_zeta((uint64_t)k, seed, (uint64_t)s, (uint64_t)x, h);
        while (e >= m) e = feistel_zeta(e, seed, (uint64_t)s, (uint64_t)x, h);
        const int i = (int)e;
        cs.zeta[g] = (uint16_t)i;
        const PointData q = load_point(pts, pt_ids[d.pt_off + i]);
        float c0, c1, c2;
        bool ray;
        if (STAGED)
            ray = shade_in(staged, bvh.n_nodes, q, node_light(lights, N, x, true), r_min2, eps, c0, c1, c2);
        else
            ray = shade<KIND>(bvh, q, node_light(lights, N, x, true), r_min2, eps, c0, c1, c2);
        n_eval += 1;
        n_ray += ray ? 1u : 0u;
        float *node_eps = cs.eps + (size_t)s * (ng - 1);
        int c = x;
        for (int f = tr.parent[x]; f >= 0; c = f, f = tr.parent[f]) {
            const int kk = f - ng;
            const int a = cs.kept[kk], bb = cs.dropped[kk];
            const int other = c == a ? bb : a;
            float o0, o1, o2;
            if (STAGED)
                ray = shade_in(staged, bvh.n_nodes, q, node_light(lights, N, other, true), r_min2, eps, o0, o1, o2);
            else
                ray = shade<KIND>(bvh, q, node_light(lights, N, other, true), r_min2, eps, o0, o1, o2);
            n_eval += 1;
            n_ray += ray ? 1u : 0u;
            const bool kept_path = c == a;
            const float a0 = kept_path ? c0 : o0, a1 = kept_path ? c1 : o1, a2 = kept_path ? c2 : o2;
            const float b0 = kept_path ? o0 : c0, b1 = kept_path ? o1 : c1, b2 = kept_path ? o2 : c2;
            const float err = fmaxf(fmaxf(lights[6 * N + bb] * fabsf(b0 - a0), lights[7 * N + bb] * fabsf(b1 - a1)),
                                    lights[8 * N + bb] * fabsf(b2 - a2));
            if (err > 0.0f) {
                unsigned int *slot = reinterpret_cast<unsigned int *>(node_eps + kk);
                const unsigned int bits = __float_as_uint(err);
                if (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < bits) atomicMax(slot, bits);
            }
            c0 = a0;
            c1 = a1;
            c2 = a2;
        }
    }
    if (counts) {
        add_count(counts, n_eval);
        add_count(counts + 1, n_ray);
    }
}

// every entry of one slice, row-major: out[(i n + j) 3 + c]
template <int KIND>
__global__ __launch_bounds__(256) void k_full_matrix(Bvh bvh, vplmc_points pts, const float *__restrict__ lights,
                                                     int32_t n_lights, int32_t m, int32_t n,
                                                     const int32_t *__restrict__ pt_ids,
                                                     const int32_t *__restrict__ cl_ids, float r_min2, float eps,
                                                     float *__restrict__ out) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= (int64_t)m * n) return;
    const int i = (int)(g / n), j = (int)(g % n);
    const int c = clamp_index(cl_ids[j], n_lights);
    const size_t N = (size_t)n_lights;
    const Light L = {{lights[c], lights[N + c], lights[2 * N + c]},
                     {lights[3 * N + c], lights[4 * N + c], lights[5 * N + c]},
                     lights[6 * N + c], lights[7 * N + c], lights[8 * N + c]};
    const PointData q = load_point(pts, pt_ids[i]);
    float o0, o1, o2;
    shade<KIND>(bvh, q, L, r_min2, eps, o0, o1, o2);
    out[3 * g] = o0;
    out[3 * g + 1] = o1;
    out[3 * g + 2] = o2;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_eval_pairs(Bvh bvh, vplmc_points pts, vplmc_lights l, int64_t n,
                                                    const int32_t *__restrict__ pid,
                                                    const int32_t *__restrict__ lid, float r_min2, float eps,
                                                    float *__restrict__ out) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int c = clamp_index(lid[g], l.n);
    const Light L = {{l.x[c], l.y[c], l.z[c]}, {l.nx[c], l.ny[c], l.nz[c]}, l.ir[c], l.ig[c], l.ib[c]};
    const PointData q = load_point(pts, pid[g]);
    float o0, o1, o2;
    shade<KIND>(bvh, q, L, r_min2, eps, o0, o1, o2);
    out[3 * g] = o0;
    out[3 * g + 1] = o1;
    out[3 * g + 2] = o2;
}

// Brute-force column sum: one thread per point and light chunk (grid.y),
// lights staged through LDS; FP32 entries summed in FP64, chunk partial sums
// added to the zeroed output with FP64 atomics.
constexpr int BF_TILE = 256;
constexpr int BF_CHUNK = 2048;
template <int KIND>
__global__ __launch_bounds__(256) void k_brute_force(Bvh bvh, vplmc_points pts, vplmc_lights l, int32_t n_out,
                                                     const int32_t *__restrict__ pid, float r_min2, float eps,
                                                     double *__restrict__ out) {
    __shared__ float sl[9][BF_TILE];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = g < n_out;
    PointData q{};
    if (active) q = load_point(pts, pid ? pid[g] : g);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int c0 = blockIdx.y * BF_CHUNK;
    const int c1 = min(l.n, c0 + BF_CHUNK);
    for (int b = c0; b < c1; b += BF_TILE) {
        const int c = b + threadIdx.x;
        if (c < c1) {
            sl[0][threadIdx.x] = l.x[c];
            sl[1][threadIdx.x] = l.y[c];
            sl[2][threadIdx.x] = l.z[c];
            sl[3][threadIdx.x] = l.nx[c];
            sl[4][threadIdx.x] = l.ny[c];
            sl[5][threadIdx.x] = l.nz[c];
            sl[6][threadIdx.x] = l.ir[c];
            sl[7][threadIdx.x] = l.ig[c];
            sl[8][threadIdx.x] = l.ib[c];
        }
        __syncthreads();
        const int cnt = min(BF_TILE, c1 - b);
        if (active) {
            for (int k = 0; k < cnt; ++k) {
                const Light L = {{sl[0][k], sl[1][k], sl[2][k]}, {sl[3][k], sl[4][k], sl[5][k]}, sl[6][k], sl[7][k],
                                 sl[8][k]};
                float o0, o1, o2;
                shade<KIND>(bvh, q, L, r_min2, eps, o0, o1, o2);
                a0 += (double)o0;
                a1 += (double)o1;
                a2 += (double)o2;
            }
        }
        __syncthreads();
    }
    if (active) {
        atomicAdd(out + 3 * (size_t)g, a0);
        atomicAdd(out + 3 * (size_t)g + 1, a1);
        atomicAdd(out + 3 * (size_t)g + 2, a2);
    }
}

__global__ void k_zero_f64(double *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Training targets of the learned proposal from fully evaluated slices: per
// (slice, column) the mean and mean square of t = R + G + B over every row
// (one thread per column, FP64 sums in row order), then per slice
// p*_j ~ sigma_j + PROPOSAL_TARGET_MIX mean(sigma) (mix 3).
template <int KIND>
__global__ __launch_bounds__(256) void k_target_moments(Bvh bvh, vplmc_points pts, const float *__restrict__ lights,
                                                        int32_t n_lights, const SliceDesc *__restrict__ desc, int S,
                                                        int64_t total_cols, const int32_t *__restrict__ pt_ids,
                                                        const int32_t *__restrict__ cl_ids, float r_min2, float eps,
                                                        double *__restrict__ m1, double *__restrict__ m2) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= total_cols) return;
    int lo = 0, hi = S;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (desc[mid].off_colptr - mid <= g) lo = mid; else hi = mid;
    }
    const int s = lo;
    const SliceDesc d = desc[s];
    const int64_t j = g - (d.off_colptr - s);
    const int c = clamp_index(cl_ids[d.cl_off + j], n_lights);
    const size_t N = (size_t)n_lights;
    const Light L = {{lights[c], lights[N + c], lights[2 * N + c]},
                     {lights[3 * N + c], lights[4 * N + c], lights[5 * N + c]},
                     lights[6 * N + c], lights[7 * N + c], lights[8 * N + c]};
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < d.m; ++i) {
        const PointData q = load_point(pts, pt_ids[d.pt_off + i]);
        float o0, o1, o2;
        shade<KIND>(bvh, q, L, r_min2, eps, o0, o1, o2);
        const double tv = (double)((o0 + o1) + o2);
        s1 += tv;
        s2 += tv * tv;
    }
    m1[d.off_col + j] = s1 / d.m;
    m2[d.off_col + j] = s2 / d.m;
}

__global__ __launch_bounds__(256) void k_target_norm(const SliceDesc *__restrict__ desc, const double *__restrict__ m1,
                                                     const double *__restrict__ m2, float *__restrict__ pstar) {
    __shared__ double red[256];
    const int s = blockIdx.x, t = threadIdx.x;
    const SliceDesc d = desc[s];
    double a = 0.0;
    for (int j = t; j < d.n; j += 256) {
        const int64_t o = d.off_col + j;
        a += sqrt(fmax(0.0, m2[o] - m1[o] * m1[o]));
    }
    red[t] = a;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double mean = red[0] / d.n;
    const double add = PROPOSAL_TARGET_MIX * (mean > 0.0 ? mean : 1.0);
    const double total = red[0] + add * d.n;
    for (int j = t; j < d.n; j += 256) {
        const int64_t o = d.off_col + j;
        pstar[o] = (float)((sqrt(fmax(0.0, m2[o] - m1[o] * m1[o])) + add) / total);
    }
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

int launch_targets(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const Bvh &bvh,
                   const vplmc_points &pts, const float *lights, int32_t n_lights, const int32_t *pt_ids,
                   const int32_t *cl_ids, const vplmc_params &prm, double *moments, float *pstar) {
    if (plan.n_slices <= 0) return VPLMC_OK;
    const int64_t cols = plan.tot_col;
    if (bvh.kind == 1)
        hipLaunchKernelGGL((k_target_moments<1>), dim3(blocks_for(cols, 256)), dim3(256), 0, st, bvh, pts, lights, n_lights,
                           desc, plan.n_slices, cols, pt_ids, cl_ids, prm.r_min * prm.r_min, prm.ray_eps, moments,
                           moments + cols);
    else
        hipLaunchKernelGGL((k_target_moments<0>), dim3(blocks_for(cols, 256)), dim3(256), 0, st, bvh, pts, lights, n_lights,
                           desc, plan.n_slices, cols, pt_ids, cl_ids, prm.r_min * prm.r_min, prm.ray_eps, moments,
                           moments + cols);
    VPLMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_target_norm, dim3(plan.n_slices), dim3(256), 0, st, desc, moments, moments + cols, pstar);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_eval_omega(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const float *lights,
                      int32_t n_lights, const SliceDesc *desc, int32_t n_slices, const int32_t *pt_ids,
                      const int32_t *cl_ids, const uint32_t *keys, int64_t n_keys, int which,
                      const int32_t *stats, const vplmc_params &prm, float *vals, int threads, int n_cu,
                      unsigned long long *rays) {
    if (n_keys <= 0) return VPLMC_OK;
    if (threads != 64 && threads != 128 && threads != 256) threads = 256;   // __launch_bounds__(256)
    // enough workgroups to fill the chip several times over; each walks the
    // samples with a grid stride
    const int64_t blocks = std::min<int64_t>(blocks_for(n_keys, threads), (int64_t)EVAL_GRID_PER_CU * n_cu);
    const size_t staged = ((size_t)2 * bvh.n_nodes + bvh.n_spheres) * sizeof(float4);
    if (bvh.n_nodes > 0 && staged <= (size_t)EVAL_LDS_BYTES) {
        if (bvh.kind == 1)
            hipLaunchKernelGGL((k_eval_omega<true, 1>), dim3((unsigned)blocks), dim3(threads), staged, st, bvh, pts, lights,
                               n_lights, desc, n_slices, pt_ids, cl_ids, keys, n_keys, which, stats,
                               prm.r_min * prm.r_min, prm.ray_eps, vals, rays);
        else
            hipLaunchKernelGGL((k_eval_omega<true, 0>), dim3((unsigned)blocks), dim3(threads), staged, st, bvh, pts, lights,
                               n_lights, desc, n_slices, pt_ids, cl_ids, keys, n_keys, which, stats,
                               prm.r_min * prm.r_min, prm.ray_eps, vals, rays);
    } else {
        if (bvh.kind == 1)
            hipLaunchKernelGGL((k_eval_omega<false, 1>), dim3((unsigned)blocks), dim3(threads), 0, st, bvh, pts, lights,
                               n_lights, desc, n_slices, pt_ids, cl_ids, keys, n_keys, which, stats,
                               prm.r_min * prm.r_min, prm.ray_eps, vals, rays);
        else
            hipLaunchKernelGGL((k_eval_omega<false, 0>), dim3((unsigned)blocks), dim3(threads), 0, st, bvh, pts, lights,
                               n_lights, desc, n_slices, pt_ids, cl_ids, keys, n_keys, which, stats,
                               prm.r_min * prm.r_min, prm.ray_eps, vals, rays);
    }
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_coarsen_eps(hipStream_t st, const vplmc_plan &plan, const Bvh &bvh, const vplmc_points &pts,
                       const float *lights, const SliceDesc *desc, const int32_t *pt_ids, const CoarsenTree &tr,
                       const CoarsenSlices &cs, const vplmc_params &prm, int n_cu, unsigned long long *counts) {
    const int64_t total = (int64_t)plan.n_slices * plan.pixels;
    if (total <= 0) return VPLMC_OK;
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>(blocks_for(total, threads), (int64_t)EVAL_GRID_PER_CU * n_cu);
    const size_t staged = ((size_t)2 * bvh.n_nodes + bvh.n_spheres) * sizeof(float4);
    if (bvh.n_nodes > 0 && staged <= (size_t)EVAL_LDS_BYTES) {
        if (bvh.kind == 1)
            hipLaunchKernelGGL((k_coarsen_eps<true, 1>), dim3((unsigned)blocks), dim3(threads), staged, st, bvh, pts, lights,
                               desc, total, (int64_t)plan.pixels, pt_ids, tr, cs, prm.seed, prm.r_min * prm.r_min,
                               prm.ray_eps, counts);
        else
            hipLaunchKernelGGL((k_coarsen_eps<true, 0>), dim3((unsigned)blocks), dim3(threads), staged, st, bvh, pts, lights,
                               desc, total, (int64_t)plan.pixels, pt_ids, tr, cs, prm.seed, prm.r_min * prm.r_min,
                               prm.ray_eps, counts);
    } else {
        if (bvh.kind == 1)
            hipLaunchKernelGGL((k_coarsen_eps<false, 1>), dim3((unsigned)blocks), dim3(threads), 0, st, bvh, pts, lights,
                               desc, total, (int64_t)plan.pixels, pt_ids, tr, cs, prm.seed, prm.r_min * prm.r_min,
                               prm.ray_eps, counts);
        else
            hipLaunchKernelGGL((k_coarsen_eps<false, 0>), dim3((unsigned)blocks), dim3(threads), 0, st, bvh, pts, lights,
                               desc, total, (int64_t)plan.pixels, pt_ids, tr, cs, prm.seed, prm.r_min * prm.r_min,
                               prm.ray_eps, counts);
    }
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_full_matrix(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const float *lights,
                       int32_t n_lights, int32_t m, int32_t n, const int32_t *pt_ids, const int32_t *cl_ids,
                       const vplmc_params &prm, float *out) {
    const int64_t total = (int64_t)m * n;
    if (total <= 0) return VPLMC_OK;
    if (bvh.kind == 1)
        hipLaunchKernelGGL((k_full_matrix<1>), dim3(blocks_for(total, 256)), dim3(256), 0, st, bvh, pts, lights, n_lights, m, n,
                           pt_ids, cl_ids, prm.r_min * prm.r_min, prm.ray_eps, out);
    else
        hipLaunchKernelGGL((k_full_matrix<0>), dim3(blocks_for(total, 256)), dim3(256), 0, st, bvh, pts, lights, n_lights, m, n,
                           pt_ids, cl_ids, prm.r_min * prm.r_min, prm.ray_eps, out);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_eval_pairs(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const vplmc_lights &l, int64_t n,
                      const int32_t *pid, const int32_t *lid, const vplmc_params &prm, float *out) {
    if (n <= 0) return VPLMC_OK;
    if (bvh.kind == 1)
        hipLaunchKernelGGL((k_eval_pairs<1>), dim3(blocks_for(n, 256)), dim3(256), 0, st, bvh, pts, l, n, pid, lid,
                           prm.r_min * prm.r_min, prm.ray_eps, out);
    else
        hipLaunchKernelGGL((k_eval_pairs<0>), dim3(blocks_for(n, 256)), dim3(256), 0, st, bvh, pts, l, n, pid, lid,
                           prm.r_min * prm.r_min, prm.ray_eps, out);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

int launch_brute_force(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const vplmc_lights &l,
                       int32_t n_out, const int32_t *pid, const vplmc_params &prm, double *out) {
    if (n_out <= 0) return VPLMC_OK;
    const size_t nz = 3 * (size_t)n_out;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)std::min<size_t>((nz + 255) / 256, 65536)), dim3(256), 0, st, out, nz);
    VPLMC_HIP(hipGetLastError());
    if (l.n <= 0) return VPLMC_OK;
    const unsigned chunks = (unsigned)((l.n + BF_CHUNK - 1) / BF_CHUNK);
    if (bvh.kind == 1)
        hipLaunchKernelGGL((k_brute_force<1>), dim3(blocks_for(n_out, 256), chunks), dim3(256), 0, st, bvh, pts, l, n_out,
                           pid, prm.r_min * prm.r_min, prm.ray_eps, out);
    else
        hipLaunchKernelGGL((k_brute_force<0>), dim3(blocks_for(n_out, 256), chunks), dim3(256), 0, st, bvh, pts, l, n_out,
                           pid, prm.r_min * prm.r_min, prm.ray_eps, out);
    VPLMC_HIP(hipGetLastError());
    return VPLMC_OK;
}

}  // namespace vplmc
