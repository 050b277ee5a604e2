// Host-side bounding-volume hierarchy over occluder spheres, built once per
// scene and uploaded; shadow rays traverse it on the device (the paper
// casts its visibility rays through an SBVH over triangles, Sec. 6; the
// scenes here are made of spheres).
//
// Top-down build: node bounds are the union of the spheres' boxes, padded
// so that an FP32 slab test never rejects a segment that meets a sphere;
// inner nodes split their spheres at the median of the centroids along
// the longest centroid extent; leaves hold at most two spheres.  Nodes are
// stored in depth-first order, each with the index of the node after its
// subtree, so a traversal needs no stack: on a hit go to the next node
// (the left child), on a miss or after a leaf go to the skip index.

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "vplmc_internal.h"

namespace vplmc {
namespace {

struct Builder {
    const float *c[3];
    const float *r;
    std::vector<int32_t> idx;
    std::vector<BvhNode> nodes;
    int max_depth = 0;

    int build(int lo, int hi, int depth) {
        max_depth = std::max(max_depth, depth);
        const int id = (int)nodes.size();
        nodes.push_back(BvhNode{});
        float blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = lo; k < hi; ++k) {
            const int s = idx[k];
            for (int a = 0; a < 3; ++a) {
                blo[a] = std::min(blo[a], c[a][s] - r[s]);
                bhi[a] = std::max(bhi[a], c[a][s] + r[s]);
                clo[a] = std::min(clo[a], c[a][s]);
                chi[a] = std::max(chi[a], c[a][s]);
            }
        }
        for (int a = 0; a < 3; ++a) {
            const float pad_lo = 1e-5f + 1e-6f * std::fabs(blo[a]);
            const float pad_hi = 1e-5f + 1e-6f * std::fabs(bhi[a]);
            nodes[id].lo[a] = blo[a] - pad_lo;
            nodes[id].hi[a] = bhi[a] + pad_hi;
        }
        if (hi - lo <= 2) {
            nodes[id].leaf = (lo << 4) | (hi - lo);
            nodes[id].skip = (int)nodes.size();
            return id;
        }
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
        const int mid = (lo + hi) / 2;
        const float *ca = c[axis];
        std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [ca](int32_t a, int32_t b) {
            return ca[a] < ca[b] || (ca[a] == ca[b] && a < b);
        });
        build(lo, mid, depth + 1);           // left child: id + 1
        build(mid, hi, depth + 1);
        nodes[id].leaf = 0;
        nodes[id].skip = (int)nodes.size();
        return id;
    }
};

}  // namespace

void build_bvh(int32_t n, const float *cx, const float *cy, const float *cz, const float *r,
               std::vector<BvhNode> &nodes, std::vector<float> &sph4) {
    nodes.clear();
    sph4.clear();
    if (n <= 0) return;
    Builder b;
    b.c[0] = cx;
    b.c[1] = cy;
    b.c[2] = cz;
    b.r = r;
    b.idx.resize(n);
    std::iota(b.idx.begin(), b.idx.end(), 0);
    b.build(0, n, 0);
    nodes.swap(b.nodes);
    sph4.resize(4 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        const int s = b.idx[k];
        sph4[4 * k] = cx[s];
        sph4[4 * k + 1] = cy[s];
        sph4[4 * k + 2] = cz[s];
        sph4[4 * k + 3] = r[s];
    }
}

}  // namespace vplmc
