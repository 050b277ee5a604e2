// Device-side pieces of a lighting-matrix entry (Sec. 3) shared by the
// kernels that evaluate entries: point and light records and their loads,
// and the entry without its visibility factor.
//
//   d = y - x, w = d / |d|, c_x = n_x . w, c_y = -n_y . w (0 if either <= 0)
//   G = c_x c_y / max(|d|^2, r_min^2)
//   f = kd / pi + ks (e + 2) / (2 pi) max(0, w_r . w_o)^e,  w_r = 2 c_x n_x - w
#ifndef VPLMC_SHADING_H
#define VPLMC_SHADING_H

#include "vplmc_internal.h"

namespace vplmc {
namespace {

constexpr float INV_PI = 0.318309886183790671538f;

struct P3 {
    float x, y, z;
};
__device__ __forceinline__ P3 sub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ float dot(P3 a, P3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

struct PointData {
    P3 x, n, wo;
    float kd0, kd1, kd2, ks, e;
};

__device__ __forceinline__ PointData load_point(const vplmc_points &p, int i) {
    i = clamp_index(i, p.m);
    PointData q;
    q.x = {p.px[i], p.py[i], p.pz[i]};
    q.n = {p.nx[i], p.ny[i], p.nz[i]};
    q.kd0 = p.kd_r[i];
    q.kd1 = p.kd_g[i];
    q.kd2 = p.kd_b[i];
    q.ks = p.ks ? p.ks[i] : 0.0f;
    q.e = p.phong_e ? p.phong_e[i] : 1.0f;
    q.wo = p.vx ? P3{p.vx[i], p.vy[i], p.vz[i]} : P3{0.0f, 0.0f, 1.0f};
    return q;
}

struct Light {
    P3 y, n;
    float i0, i1, i2;
};

__device__ __forceinline__ Light node_light(const float *__restrict__ lights, size_t N, int c, bool unit) {
    return Light{{lights[c], lights[N + c], lights[2 * N + c]},
                 {lights[3 * N + c], lights[4 * N + c], lights[5 * N + c]},
                 unit ? 1.0f : lights[6 * N + c], unit ? 1.0f : lights[7 * N + c], unit ? 1.0f : lights[8 * N + c]};
}

// f * I * G of one pair with the visibility taken as 1; false (and zeros)
// when the pair faces away
__device__ __forceinline__ bool entry_unoccluded(const PointData &q, const Light &L, float r_min2, float &o0,
                                                 float &o1, float &o2) {
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
    o0 = fmaf(q.kd0, INV_PI, spec) * L.i0 * G;
    o1 = fmaf(q.kd1, INV_PI, spec) * L.i1 * G;
    o2 = fmaf(q.kd2, INV_PI, spec) * L.i2 * G;
    return true;
}

}  // namespace
}  // namespace vplmc

#endif
