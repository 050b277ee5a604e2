// Host-side bounding-volume hierarchies, built once per scene and uploaded;
// shadow rays traverse them on the device: one over occluder spheres, and a
// spatial-split BVH over triangles (the paper casts its visibility rays
// through an SBVH over its scenes' triangles, Sec. 6), below.
//
// Top-down build: node bounds are the union of the spheres' boxes, padded
// so that an FP32 slab test never rejects a segment that meets a sphere;
// inner nodes split their spheres by the binned surface-area heuristic over
// the centroids (16 bins per axis, C = 1 + (A_L N_L + A_R N_R) / A, a sphere
// test costing as much as a node test), or at the median of the longest
// centroid extent when no bin boundary separates them; a node of at most two
// spheres is a leaf (leaves of up to four where no split is cheaper, or of
// up to eight, were measured slower).  The
// shape of the tree changes which boxes a shadow ray visits, never its
// answer: every sphere a segment could meet lies in a box the segment meets.  Nodes are
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
        const int N = hi - lo;
        if (N <= 2) {
            nodes[id].leaf = (lo << 4) | N;
            nodes[id].skip = (int)nodes.size();
            return id;
        }
        // binned surface-area heuristic over the centroids (16 bins per axis)
        auto area = [](const double *l, const double *h) {
            const double dx = h[0] - l[0], dy = h[1] - l[1], dz = h[2] - l[2];
            return dx < 0 ? 0.0 : 2.0 * (dx * dy + dy * dz + dz * dx);
        };
        double nl[3], nh[3];
        for (int a = 0; a < 3; ++a) {
            nl[a] = blo[a];
            nh[a] = bhi[a];
        }
        const double An = area(nl, nh);
        constexpr int NB = 16;
        double best = INFINITY;
        int b_axis = -1, b_bin = -1;
        for (int a = 0; a < 3; ++a) {
            const double ext = (double)chi[a] - (double)clo[a];
            if (!(ext > 0.0)) continue;
            double bl[NB][3], bh[NB][3];
            int cnt[NB] = {0};
            for (int k = 0; k < NB; ++k)
                for (int e = 0; e < 3; ++e) {
                    bl[k][e] = INFINITY;
                    bh[k][e] = -INFINITY;
                }
            for (int k = lo; k < hi; ++k) {
                const int s = idx[k];
                const int bi = std::min(NB - 1, (int)(((double)c[a][s] - clo[a]) / ext * NB));
                ++cnt[bi];
                for (int e = 0; e < 3; ++e) {
                    bl[bi][e] = std::min(bl[bi][e], (double)c[e][s] - r[s]);
                    bh[bi][e] = std::max(bh[bi][e], (double)c[e][s] + r[s]);
                }
            }
            double rA[NB];
            int rN[NB];
            double al[3] = {INFINITY, INFINITY, INFINITY}, ah[3] = {-INFINITY, -INFINITY, -INFINITY};
            int n_acc = 0;
            for (int k = NB - 1; k > 0; --k) {
                for (int e = 0; e < 3; ++e) {
                    al[e] = std::min(al[e], bl[k][e]);
                    ah[e] = std::max(ah[e], bh[k][e]);
                }
                n_acc += cnt[k];
                rA[k] = n_acc ? area(al, ah) : 0.0;
                rN[k] = n_acc;
            }
            double ll[3] = {INFINITY, INFINITY, INFINITY}, lh[3] = {-INFINITY, -INFINITY, -INFINITY};
            int ln = 0;
            for (int k = 0; k < NB - 1; ++k) {
                for (int e = 0; e < 3; ++e) {
                    ll[e] = std::min(ll[e], bl[k][e]);
                    lh[e] = std::max(lh[e], bh[k][e]);
                }
                ln += cnt[k];
                if (ln == 0 || rN[k + 1] == 0) continue;
                const double cost = 1.0 + (area(ll, lh) * ln + rA[k + 1] * rN[k + 1]) / An;
                if (cost < best) {
                    best = cost;
                    b_axis = a;
                    b_bin = k;
                }
            }
        }
        int mid = lo;
        if (b_axis >= 0) {
            const int a = b_axis;
            const double ext = (double)chi[a] - (double)clo[a];
            const float *ca = c[a];
            auto it = std::stable_partition(idx.begin() + lo, idx.begin() + hi, [&](int32_t s) {
                return std::min(NB - 1, (int)(((double)ca[s] - clo[a]) / ext * NB)) <= b_bin;
            });
            mid = (int)(it - idx.begin());
        }
        if (mid <= lo || mid >= hi) {                // no usable split: median of the longest extent
            int axis = 0;
            for (int a = 1; a < 3; ++a)
                if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
            mid = (lo + hi) / 2;
            const float *ca = c[axis];
            std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [ca](int32_t a, int32_t b) {
                return ca[a] < ca[b] || (ca[a] == ca[b] && a < b);
            });
        }
        build(lo, mid, depth + 1);           // left child: id + 1
        build(mid, hi, depth + 1);
        nodes[id].leaf = 0;
        nodes[id].skip = (int)nodes.size();
        return id;
    }
};

}  // namespace

void build_bvh(int32_t n, const float *cx, const float *cy, const float *cz, const float *r,
               std::vector<BvhNode> &nodes, std::vector<float> &sph4, std::vector<int32_t> *order) {
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
    if (order) *order = b.idx;
    sph4.resize(4 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        const int s = b.idx[k];
        sph4[4 * k] = cx[s];
        sph4[4 * k + 1] = cy[s];
        sph4[4 * k + 2] = cz[s];
        sph4[4 * k + 3] = r[s];
    }
}


// ---------------------------------------------------------------------------
// SBVH over triangles (the paper traces its visibility rays through a
// spatial-split BVH, Sec. 6; Stich, Friedrich and Dietrich 2009).
//
// Top-down over references (a triangle and the box of the part of it that a
// node holds).  At every node two candidates are costed by the surface-area
// heuristic, C = C_T + (A_L N_L + A_R N_R) / A C_I with C_T = 1, C_I = 1:
//   * an object split: references binned by box centroid (16 bins per axis);
//   * a spatial split, tried only when the object split's two children
//     overlap by more than 1e-5 of the root's area: 16 equal bins of the node
//     along each axis; a reference is chopped at every bin plane it spans (the
//     exact bounds of the triangle's part between the planes, intersected
//     with the reference's box) and counted as entering its first bin and
//     leaving its last.  Applying it sends a straddling reference to both
//     children, each with the box of its side.
// A node becomes a leaf when no split is cheaper than intersecting all its
// references (N C_I) and it holds at most 15 (the leaf code's 4 bits), or
// when it holds at most 2.  Spatial splits stop once the references number
// twice the triangles (so at most 2^25 references for the 2^24 triangles
// allowed, inside the leaf code's 2^27).  Nodes are laid out as in build_bvh (depth-first,
// skip indices, padded FP32 bounds); a leaf's references are contiguous, each
// as three float4 (v0, v1 - v0, v2 - v0).
namespace {

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const double *p) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    void grow(const Box &b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    bool empty() const { return !(lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2]); }
    double area() const {
        if (empty()) return 0.0;
        const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
    Box meet(const Box &b) const {
        Box r;
        for (int a = 0; a < 3; ++a) {
            r.lo[a] = std::max(lo[a], b.lo[a]);
            r.hi[a] = std::min(hi[a], b.hi[a]);
        }
        return r;
    }
};

struct Ref {
    int32_t tri;
    Box box;
};

constexpr int SB_BINS = 16;
constexpr int SB_LEAF_MAX = 15;

struct SBuilder {
    const float *v;          // 9 per triangle
    std::vector<BvhNode> nodes;
    std::vector<int32_t> leaf_refs;
    double root_area = 0.0;
    int max_depth = 0;
    size_t refs_live = 0;    // references in the tree being built
    size_t ref_budget = 0;   // spatial splits stop at this many (twice the triangles)

    void vert(int t, int k, double *p) const {
        for (int a = 0; a < 3; ++a) p[a] = (double)v[9 * (size_t)t + 3 * k + a];
    }
    // bounds of the part of triangle t with coordinate `axis` in [s0, s1], met with `clip`
    Box chop(int t, int axis, double s0, double s1, const Box &clip) const {
        double P[3][3];
        for (int k = 0; k < 3; ++k) vert(t, k, P[k]);
        Box b;
        for (int k = 0; k < 3; ++k) {
            const double *p = P[k], *q = P[(k + 1) % 3];
            if (p[axis] >= s0 && p[axis] <= s1) b.grow(p);
            for (const double s : {s0, s1}) {       // edge crossings of the two planes
                if ((p[axis] < s && q[axis] > s) || (p[axis] > s && q[axis] < s)) {
                    const double f = (s - p[axis]) / (q[axis] - p[axis]);
                    double x[3];
                    for (int a = 0; a < 3; ++a) x[a] = p[a] + f * (q[a] - p[a]);
                    x[axis] = s;
                    b.grow(x);
                }
            }
        }
        return b.meet(clip);
    }

    int emit_node(const Box &b) {
        BvhNode nd{};
        for (int a = 0; a < 3; ++a) {
            const float lo = (float)b.lo[a], hi = (float)b.hi[a];
            nd.lo[a] = lo - (1e-5f + 1e-6f * std::fabs(lo));
            nd.hi[a] = hi + (1e-5f + 1e-6f * std::fabs(hi));
        }
        nodes.push_back(nd);
        return (int)nodes.size() - 1;
    }

    void leaf(int id, std::vector<Ref> &refs) {
        nodes[id].leaf = ((int32_t)leaf_refs.size() << 4) | (int32_t)refs.size();
        for (const Ref &r : refs) leaf_refs.push_back(r.tri);
        nodes[id].skip = (int)nodes.size();
    }

    void build(std::vector<Ref> &refs, int depth) {
        max_depth = std::max(max_depth, depth);
        Box nb, cb;
        for (const Ref &r : refs) {
            nb.grow(r.box);
            double c[3];
            for (int a = 0; a < 3; ++a) c[a] = 0.5 * (r.box.lo[a] + r.box.hi[a]);
            cb.grow(c);
        }
        const int id = emit_node(nb);
        const size_t N = refs.size();
        if (N <= 2 || depth >= 60) {
            if (N <= (size_t)SB_LEAF_MAX) {
                leaf(id, refs);
                return;
            }
        }
        const double A = nb.area();
        // ---- object split: binned centroids
        double best_o = INFINITY, ov_area = 0.0;
        int bo_axis = -1, bo_bin = -1;
        for (int a = 0; a < 3; ++a) {
            const double ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0)) continue;
            Box bins[SB_BINS];
            int cnt[SB_BINS] = {0};
            for (const Ref &r : refs) {
                const double c = 0.5 * (r.box.lo[a] + r.box.hi[a]);
                const int k = std::min(SB_BINS - 1, (int)((c - cb.lo[a]) / ext * SB_BINS));
                bins[k].grow(r.box);
                ++cnt[k];
            }
            Box rb[SB_BINS];
            int rc[SB_BINS];
            Box acc;
            int n = 0;
            for (int k = SB_BINS - 1; k > 0; --k) {
                acc.grow(bins[k]);
                n += cnt[k];
                rb[k] = acc;
                rc[k] = n;
            }
            Box lb;
            int ln = 0;
            for (int k = 0; k < SB_BINS - 1; ++k) {
                lb.grow(bins[k]);
                ln += cnt[k];
                if (ln == 0 || rc[k + 1] == 0) continue;
                const double c = 1.0 + (lb.area() * ln + rb[k + 1].area() * rc[k + 1]) / A;
                if (c < best_o) {
                    best_o = c;
                    bo_axis = a;
                    bo_bin = k;
                    ov_area = lb.meet(rb[k + 1]).area();
                }
            }
        }
        // ---- spatial split: chopped references over equal bins
        double best_s = INFINITY;
        int bs_axis = -1, bs_bin = -1;
        if (depth < 48 && ov_area > 1e-5 * root_area && refs_live < ref_budget) {
            for (int a = 0; a < 3; ++a) {
                const double ext = nb.hi[a] - nb.lo[a];
                if (!(ext > 0.0)) continue;
                const double w = ext / SB_BINS;
                Box bins[SB_BINS];
                int enter[SB_BINS] = {0}, leave[SB_BINS] = {0};
                for (const Ref &r : refs) {
                    const int k0 = std::max(0, std::min(SB_BINS - 1, (int)((r.box.lo[a] - nb.lo[a]) / w)));
                    const int k1 = std::max(k0, std::min(SB_BINS - 1, (int)((r.box.hi[a] - nb.lo[a]) / w)));
                    for (int k = k0; k <= k1; ++k) {
                        const double s0 = k == k0 ? r.box.lo[a] : nb.lo[a] + k * w;
                        const double s1 = k == k1 ? r.box.hi[a] : nb.lo[a] + (k + 1) * w;
                        bins[k].grow(chop(r.tri, a, s0, s1, r.box));
                    }
                    ++enter[k0];
                    ++leave[k1];
                }
                Box rb[SB_BINS];
                int rc[SB_BINS];
                Box acc;
                int n = 0;
                for (int k = SB_BINS - 1; k > 0; --k) {
                    acc.grow(bins[k]);
                    n += leave[k];
                    rb[k] = acc;
                    rc[k] = n;
                }
                Box lb;
                int ln = 0;
                for (int k = 0; k < SB_BINS - 1; ++k) {
                    lb.grow(bins[k]);
                    ln += enter[k];
                    if (ln == 0 || rc[k + 1] == 0) continue;
                    const double c = 1.0 + (lb.area() * ln + rb[k + 1].area() * rc[k + 1]) / A;
                    if (c < best_s) {
                        best_s = c;
                        bs_axis = a;
                        bs_bin = k;
                    }
                }
            }
        }
        const double leaf_cost = (double)N;
        if (N <= (size_t)SB_LEAF_MAX && leaf_cost <= std::min(best_o, best_s)) {
            leaf(id, refs);
            return;
        }
        std::vector<Ref> L, R;
        if (best_s < best_o && bs_axis >= 0) {
            const int a = bs_axis;
            const double w = (nb.hi[a] - nb.lo[a]) / SB_BINS;
            const double s = nb.lo[a] + (bs_bin + 1) * w;
            for (const Ref &r : refs) {
                if (r.box.hi[a] <= s) {
                    L.push_back(r);
                } else if (r.box.lo[a] >= s) {
                    R.push_back(r);
                } else {
                    const Box bl = chop(r.tri, a, r.box.lo[a], s, r.box), br = chop(r.tri, a, s, r.box.hi[a], r.box);
                    if (!bl.empty()) L.push_back(Ref{r.tri, bl});
                    if (!br.empty()) R.push_back(Ref{r.tri, br});
                }
            }
        } else if (bo_axis >= 0) {
            const int a = bo_axis;
            const double ext = cb.hi[a] - cb.lo[a];
            for (const Ref &r : refs) {
                const double c = 0.5 * (r.box.lo[a] + r.box.hi[a]);
                const int k = std::min(SB_BINS - 1, (int)((c - cb.lo[a]) / ext * SB_BINS));
                (k <= bo_bin ? L : R).push_back(r);
            }
        }
        if (L.empty() || R.empty() || L.size() + R.size() > 2 * N || refs_live + L.size() + R.size() - N > ref_budget) {
            // no usable split (coincident centroids) or the duplication budget
            // is spent: halve the list
            L.assign(refs.begin(), refs.begin() + N / 2);
            R.assign(refs.begin() + N / 2, refs.end());
        }
        refs_live += L.size() + R.size() - N;
        std::vector<Ref>().swap(refs);
        build(L, depth + 1);      // left child: id + 1
        build(R, depth + 1);
        nodes[id].leaf = 0;
        nodes[id].skip = (int)nodes.size();
    }
};

}  // namespace

void build_sbvh(int32_t n, const float *v, std::vector<BvhNode> &nodes, std::vector<int32_t> &refs,
                std::vector<float> &prim4) {
    nodes.clear();
    refs.clear();
    prim4.clear();
    if (n <= 0) return;
    SBuilder b;
    b.v = v;
    std::vector<Ref> all((size_t)n);
    Box root;
    for (int t = 0; t < n; ++t) {
        all[t].tri = t;
        for (int k = 0; k < 3; ++k) {
            double p[3];
            b.vert(t, k, p);
            all[t].box.grow(p);
        }
        root.grow(all[t].box);
    }
    b.root_area = root.area();
    b.refs_live = (size_t)n;
    b.ref_budget = 2 * (size_t)n;
    b.build(all, 0);
    nodes.swap(b.nodes);
    refs.swap(b.leaf_refs);
    prim4.resize(12 * refs.size());
    for (size_t k = 0; k < refs.size(); ++k) {
        const float *p = v + 9 * (size_t)refs[k];
        float *o = prim4.data() + 12 * k;
        for (int a = 0; a < 3; ++a) {
            o[a] = p[a];
            o[4 + a] = p[3 + a] - p[a];
            o[8 + a] = p[6 + a] - p[a];
        }
        o[3] = o[7] = o[11] = 0.f;
    }
}

}  // namespace vplmc
