// Nodes of a light tree (Sec. 4: a merged light L_f is one child's light
// with the summed intensity), shared by the coarsening's tree above the
// global cut and the global light cut's tree over every VPL.
#ifndef VPLMC_TREE_NODES_H
#define VPLMC_TREE_NODES_H

#include "vplmc_internal.h"

namespace vplmc {

constexpr uint64_t TAG_LTREE = 8;  // kept child of a split node of the full light tree (global cut)

// total intensity t = (R + G) + B in FP64 of FP32 channels
__device__ __forceinline__ double total_t(float r, float g, float b) {
    return ((double)r + (double)g) + (double)b;
}

// max(1, floor(2^24 t / tmax)), or 1 when tmax is not positive
__device__ __forceinline__ uint64_t quantise(double t, double tmax) {
    if (!(tmax > 0.0)) return 1;
    const double f = floor((16777216.0 * t) / tmax);
    return f > 1.0 ? (uint64_t)f : 1ull;
}

// A split node f of a light tree from its children l, r (Sec. 4: L_f is the
// same light as one child L_a, I_f = I_a + I_b): the kept child a is drawn
// with probability Q_a / (Q_l + Q_r) by Philox(key = (seed, 0),
// ctr = (f, 0, tag, 0)); f takes a's representative and light, the FP32 sum
// (in FP64) of both intensities and the union of both boxes.  Planes of
// stride N: lights x y z nx ny nz ir ig ib, bbox lo xyz then hi xyz.
// Returns a.
__device__ __forceinline__ int combine_node(int32_t *rep, float *lights, float *bbox, size_t N, int f, int l, int r,
                                            uint64_t seed, uint64_t tag) {
    const float ir = (float)((double)lights[6 * N + l] + (double)lights[6 * N + r]);
    const float ig = (float)((double)lights[7 * N + l] + (double)lights[7 * N + r]);
    const float ib = (float)((double)lights[8 * N + l] + (double)lights[8 * N + r]);
    const double tl = total_t(lights[6 * N + l], lights[7 * N + l], lights[8 * N + l]);
    const double trr = total_t(lights[6 * N + r], lights[7 * N + r], lights[8 * N + r]);
    const double tmax = tl > trr ? tl : trr;
    const uint64_t ql = quantise(tl, tmax), qr = quantise(trr, tmax);
    const uint64_t u = mulhi64(philox(seed, 0, (uint64_t)f, 0, tag, 0).a, ql + qr);
    const int a = u < ql ? l : r;
    rep[f] = rep[a];
    for (int p = 0; p < 6; ++p) lights[p * N + f] = lights[p * N + a];
    lights[6 * N + f] = ir;
    lights[7 * N + f] = ig;
    lights[8 * N + f] = ib;
    for (int p = 0; p < 3; ++p) {
        bbox[p * N + f] = fminf(bbox[p * N + l], bbox[p * N + r]);
        bbox[(3 + p) * N + f] = fmaxf(bbox[(3 + p) * N + l], bbox[(3 + p) * N + r]);
    }
    return a;
}

}  // namespace vplmc

#endif
