// C ABI of the library: argument validation (host only, before any launch),
// frame planning and workspace layout, and the launch sequence of a frame.

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>
#include <cmath>
#include <algorithm>

#include "vplmc_internal.h"
#include "lightcut.h"

namespace vplmc {

namespace {
thread_local char g_err[512] = "";
}

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_error(hipError_t e, const char *what) {
    return set_error(VPLMC_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

namespace {

// Workspace of vplmc_render_static: a file-scope device array, so the call
// needs no allocation.  Every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the device symbol): the
// device address comes from hipGetSymbolAddress, once per device, below.
__device__ __align__(256) unsigned char scratch[VPLMC_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device` (the current device): looked up on
// the first call for that device and kept.
int scratch_address(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return set_error(VPLMC_EUNSUPPORTED, "device %d >= %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return VPLMC_OK;
}

int64_t count_from_ppm(int64_t ppm, int64_t D) { return (ppm * D + 500000) / 1000000; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool bad_ptrs_points(const vplmc_points *p) {
    if (!p->px || !p->py || !p->pz || !p->nx || !p->ny || !p->nz || !p->kd_r || !p->kd_g || !p->kd_b) return true;
    if ((p->ks == nullptr) != (p->phong_e == nullptr)) return true;
    if (!((p->vx && p->vy && p->vz) || (!p->vx && !p->vy && !p->vz))) return true;
    return false;
}

bool bad_ptrs_lights(const vplmc_lights *l) {
    return !l->x || !l->y || !l->z || !l->nx || !l->ny || !l->nz || !l->ir || !l->ig || !l->ib;
}

int check_params(const vplmc_params *p) {
    if (!p) return set_error(VPLMC_EINVAL, "params is NULL");
    if (p->pass1_ppm < 0 || p->pass2_ppm < 0 || p->pass1_ppm > 1000000 || p->pass2_ppm > 1000000 ||
        (int64_t)p->pass1_ppm + p->pass2_ppm > 1000000)
        return set_error(VPLMC_EINVAL, "sampling rates must be in [0, 1e6] ppm and sum to at most 1e6 (got %d + %d)",
                         p->pass1_ppm, p->pass2_ppm);
    if (p->max_iter < 0) return set_error(VPLMC_EINVAL, "max_iter must be >= 0 (got %d)", p->max_iter);
    if (!(p->alpha0 > 0.f) || !(p->beta0 > 0.f))
        return set_error(VPLMC_EINVAL, "alpha0 and beta0 must be > 0");
    if (!(p->gamma > 0.f && p->gamma < 1.618034f))
        return set_error(VPLMC_EINVAL, "gamma must be in (0, 1.618) (got %g)", (double)p->gamma);
    if (!(p->tol >= 0.f)) return set_error(VPLMC_EINVAL, "tol must be >= 0");
    if (!(p->r_min > 0.f) || !(p->ray_eps >= 0.f)) return set_error(VPLMC_EINVAL, "r_min must be > 0, ray_eps >= 0");
    if (!(p->lam > 0.f)) return set_error(VPLMC_EINVAL, "lam must be > 0");
    if (!(p->pass2_mix >= 0.f)) return set_error(VPLMC_EINVAL, "pass2_mix must be >= 0 (got %g)", (double)p->pass2_mix);
    if (p->flags & ~(VPLMC_FIXED_ITERS | VPLMC_LEARNED | VPLMC_FEATURES | VPLMC_GIVEN_INIT | VPLMC_NO_NONNEG | VPLMC_ALS))
        return set_error(VPLMC_EINVAL, "unknown flags 0x%x", p->flags);
    return VPLMC_OK;
}

// rank group of a slice completed at rank q: the kernels run at the next of
// 4, 8, 16, 32 (extra components of the factors stay 0)
int rank_bucket(int q) { return q <= 4 ? 0 : (q <= 8 ? 1 : (q <= 16 ? 2 : 3)); }
int padded_rank(int q) { return 4 << rank_bucket(q); }

// records the boundary event `b` (0 .. VPLMC_N_PHASES) of the current frame
struct PhaseMarks {
    vplmc_ctx *ctx;
    hipEvent_t *ev = nullptr;
    explicit PhaseMarks(vplmc_ctx *c) : ctx(c) {
        if (c->prof_on && !c->capturing && c->prof_frames < c->prof_max_frames)
            ev = &c->prof_events[(size_t)c->prof_frames * (VPLMC_N_PHASES + 1)];
    }
    int mark(int b) {
        if (ev) VPLMC_HIP(hipEventRecord(ev[b], ctx->stream));
        return VPLMC_OK;
    }
    void done() {
        if (ev) ctx->prof_frames++;
    }
};

template <typename T>
T *region(void *ws, const vplmc_plan *plan, int r) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + plan->layout.off[r]);
}

}  // namespace
}  // namespace vplmc

using namespace vplmc;

extern "C" {

int vplmc_version(void) { return VPLMC_VERSION; }

const char *vplmc_last_error(void) { return g_err; }

int vplmc_default_params(vplmc_params *out) {
    if (!out) return set_error(VPLMC_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    out->seed = 1;
    out->pass1_ppm = 50000;
    out->pass2_ppm = 50000;
    out->max_iter = 100;
    out->flags = 0;
    out->tol = 1e-3f;
    out->alpha0 = 0.1f;
    out->beta0 = 0.1f;
    out->gamma = 1.6f;
    out->r_min = 0.05f;
    out->ray_eps = 1e-4f;
    out->lam = 0.01f;
    return VPLMC_OK;
}

int vplmc_create(int device, void *stream, vplmc_ctx **out) {
    if (!out) return set_error(VPLMC_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return set_error(VPLMC_EHIP, "no HIP device available");
    if (device < 0 || device >= count) return set_error(VPLMC_EINVAL, "device %d out of range [0, %d)", device, count);
    VPLMC_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    VPLMC_HIP(hipGetDeviceProperties(&prop, device));
    vplmc_ctx *ctx = new (std::nothrow) vplmc_ctx();
    if (!ctx) return set_error(VPLMC_ENOMEM, "context allocation failed");
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->n_cu = prop.multiProcessorCount;
    if (int rc = scratch_address(device, &ctx->scratch)) {
        delete ctx;
        return rc;
    }
    hipError_t he = hipEventCreateWithFlags(&ctx->adm.fork, hipEventDisableTiming);
    for (int k = 0; k < 3 && he == hipSuccess; ++k) {
        he = hipStreamCreateWithFlags(&ctx->adm.side[k], hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&ctx->adm.join[k], hipEventDisableTiming);
    }
    if (he != hipSuccess) {
        vplmc_destroy(ctx);
        return hip_error(he, "completion streams");
    }
    *out = ctx;
    return VPLMC_OK;
}

int vplmc_destroy(vplmc_ctx *ctx) {
    if (!ctx) return VPLMC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->bvh_mem) (void)hipFree(ctx->bvh_mem);
    for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
    for (int k = 0; k < 3; ++k) {
        if (ctx->adm.side[k]) {
            (void)hipStreamSynchronize(ctx->adm.side[k]);
            (void)hipStreamDestroy(ctx->adm.side[k]);
        }
        if (ctx->adm.join[k]) (void)hipEventDestroy(ctx->adm.join[k]);
    }
    if (ctx->adm.fork) (void)hipEventDestroy(ctx->adm.fork);
    delete ctx;
    return VPLMC_OK;
}

int vplmc_set_stream(vplmc_ctx *ctx, void *stream) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(stream);
    return VPLMC_OK;
}

static int check_spheres(int32_t n, const float *cx, const float *cy, const float *cz, const float *r) {
    if (n < 0 || n > BVH_MAX_SPHERES) return set_error(VPLMC_EINVAL, "n must be in [0, 2^27]");
    if (n > 0 && (!cx || !cy || !cz || !r)) return set_error(VPLMC_EINVAL, "sphere arrays must be non-NULL");
    for (int k = 0; k < n; ++k)
        if (!(r[k] > 0.f) || !std::isfinite(cx[k]) || !std::isfinite(cy[k]) || !std::isfinite(cz[k]))
            return set_error(VPLMC_EINVAL, "sphere %d: radius must be > 0 and centre finite", k);
    return VPLMC_OK;
}

int vplmc_bvh_build(int32_t n, const float *cx, const float *cy, const float *cz, const float *r, int32_t max_nodes,
                    float *box, int32_t *code, int32_t *order, int32_t *n_nodes) {
    if (!n_nodes) return set_error(VPLMC_EINVAL, "n_nodes is NULL");
    int rc = check_spheres(n, cx, cy, cz, r);
    if (rc) return rc;
    std::vector<BvhNode> nodes;
    std::vector<float> sph;
    std::vector<int32_t> ord;
    build_bvh(n, cx, cy, cz, r, nodes, sph, &ord);
    *n_nodes = (int32_t)nodes.size();
    if ((int64_t)nodes.size() > max_nodes)
        return set_error(VPLMC_EINVAL, "the BVH has %zu nodes (room for %d)", nodes.size(), max_nodes);
    if (n > 0 && (!box || !code || !order)) return set_error(VPLMC_EINVAL, "output arrays must be non-NULL");
    for (size_t k = 0; k < nodes.size(); ++k) {
        for (int a = 0; a < 3; ++a) {
            box[6 * k + a] = nodes[k].lo[a];
            box[6 * k + 3 + a] = nodes[k].hi[a];
        }
        code[2 * k] = nodes[k].leaf;
        code[2 * k + 1] = nodes[k].skip;
    }
    std::copy(ord.begin(), ord.end(), order);
    return VPLMC_OK;
}

int vplmc_set_occluders(vplmc_ctx *ctx, int32_t n, const float *cx, const float *cy, const float *cz,
                        const float *r) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    int rc0 = check_spheres(n, cx, cy, cz, r);
    if (rc0) return rc0;
    std::vector<BvhNode> nodes;
    std::vector<float> sph;
    build_bvh(n, cx, cy, cz, r, nodes, sph);
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (ctx->bvh_mem) {
        VPLMC_HIP(hipStreamSynchronize(ctx->stream));
        VPLMC_HIP(hipFree(ctx->bvh_mem));
        ctx->bvh_mem = nullptr;
    }
    ctx->bvh = Bvh{};
    if (n == 0) return VPLMC_OK;
    const size_t nb = align256(nodes.size() * sizeof(BvhNode));
    const size_t sb = sph.size() * sizeof(float);
    void *mem = nullptr;
    if (hipMalloc(&mem, nb + sb) != hipSuccess) return set_error(VPLMC_ENOMEM, "BVH allocation failed");
    ctx->bvh_mem = mem;
    VPLMC_HIP(hipMemcpy(mem, nodes.data(), nodes.size() * sizeof(BvhNode), hipMemcpyHostToDevice));
    VPLMC_HIP(hipMemcpy(static_cast<char *>(mem) + nb, sph.data(), sb, hipMemcpyHostToDevice));
    ctx->bvh.nodes = static_cast<const BvhNode *>(mem);
    ctx->bvh.spheres = reinterpret_cast<const float4 *>(static_cast<char *>(mem) + nb);
    ctx->bvh.n_nodes = (int32_t)nodes.size();
    ctx->bvh.n_spheres = n;
    return VPLMC_OK;
}

static int check_triangles(int32_t n, const float *v) {
    if (n < 0 || n > BVH_MAX_TRIANGLES) return set_error(VPLMC_EINVAL, "n must be in [0, 2^24]");
    if (n > 0 && !v) return set_error(VPLMC_EINVAL, "triangle array must be non-NULL");
    for (size_t k = 0; k < 9 * (size_t)n; ++k)
        if (!std::isfinite(v[k])) return set_error(VPLMC_EINVAL, "triangle %zu: vertex not finite", k / 9);
    return VPLMC_OK;
}

int vplmc_set_triangles(vplmc_ctx *ctx, int32_t n, const float *v) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    int rc = check_triangles(n, v);
    if (rc) return rc;
    std::vector<BvhNode> nodes;
    std::vector<int32_t> refs;
    std::vector<float> prim;
    build_sbvh(n, v, nodes, refs, prim);
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (ctx->bvh_mem) {
        VPLMC_HIP(hipStreamSynchronize(ctx->stream));
        VPLMC_HIP(hipFree(ctx->bvh_mem));
        ctx->bvh_mem = nullptr;
    }
    ctx->bvh = Bvh{};
    if (n == 0) return VPLMC_OK;
    if (3 * refs.size() > (size_t)INT32_MAX) return set_error(VPLMC_EINVAL, "too many SBVH references");
    const size_t nb = align256(nodes.size() * sizeof(BvhNode));
    const size_t pb = prim.size() * sizeof(float);
    void *mem = nullptr;
    if (hipMalloc(&mem, nb + pb) != hipSuccess) return set_error(VPLMC_ENOMEM, "SBVH allocation failed");
    ctx->bvh_mem = mem;
    VPLMC_HIP(hipMemcpy(mem, nodes.data(), nodes.size() * sizeof(BvhNode), hipMemcpyHostToDevice));
    VPLMC_HIP(hipMemcpy(static_cast<char *>(mem) + nb, prim.data(), pb, hipMemcpyHostToDevice));
    ctx->bvh.nodes = static_cast<const BvhNode *>(mem);
    ctx->bvh.spheres = reinterpret_cast<const float4 *>(static_cast<char *>(mem) + nb);
    ctx->bvh.n_nodes = (int32_t)nodes.size();
    ctx->bvh.n_spheres = (int32_t)(3 * refs.size());
    ctx->bvh.kind = 1;
    return VPLMC_OK;
}

int vplmc_sbvh_build(int32_t n, const float *v, int32_t max_nodes, float *box, int32_t *code, int32_t max_refs,
                     int32_t *refs, int32_t *n_nodes, int32_t *n_refs) {
    if (!n_nodes || !n_refs) return set_error(VPLMC_EINVAL, "count outputs must be non-NULL");
    int rc = check_triangles(n, v);
    if (rc) return rc;
    std::vector<BvhNode> nodes;
    std::vector<int32_t> rf;
    std::vector<float> prim;
    build_sbvh(n, v, nodes, rf, prim);
    *n_nodes = (int32_t)nodes.size();
    *n_refs = (int32_t)rf.size();
    if ((int64_t)nodes.size() > max_nodes || (int64_t)rf.size() > max_refs)
        return set_error(VPLMC_EINVAL, "the SBVH has %zu nodes and %zu references (room for %d and %d)", nodes.size(),
                         rf.size(), max_nodes, max_refs);
    if ((!nodes.empty() && (!box || !code)) || (!rf.empty() && !refs))
        return set_error(VPLMC_EINVAL, "output arrays must be non-NULL");
    for (size_t k = 0; k < nodes.size(); ++k) {
        for (int a = 0; a < 3; ++a) {
            box[6 * k + a] = nodes[k].lo[a];
            box[6 * k + 3 + a] = nodes[k].hi[a];
        }
        code[2 * k] = nodes[k].leaf;
        code[2 * k + 1] = nodes[k].skip;
    }
    std::copy(rf.begin(), rf.end(), refs);
    return VPLMC_OK;
}

// Topology of the tree above the cut (integer bookkeeping, no method
// arithmetic): validates that every node but the root is the child of
// exactly one later split node, and lays out left, right, parent, height,
// smallest leaf, the split nodes ordered by (height, id) and the level offsets.
static int build_tree(const vplmc_coarsen *co, std::vector<int32_t> &tree, int32_t &height_max) {
    const int ng = co->n_leaves, ns = ng - 1, NC = 2 * ng - 1;
    if (ns > 0 && (!co->left || !co->right)) return set_error(VPLMC_EINVAL, "tree arrays must be non-NULL");
    std::vector<int32_t> parent(NC, -1), height(NC, 0), min_leaf(NC);
    for (int x = 0; x < NC; ++x) min_leaf[x] = x;
    for (int k = 0; k < ns; ++k) {
        const int f = ng + k, l = co->left[k], r = co->right[k];
        if (l < 0 || r < 0 || l >= f || r >= f || l == r)
            return set_error(VPLMC_EINVAL, "tree: split node %d has children %d, %d (must be distinct and earlier)", f, l, r);
        if (parent[l] >= 0 || parent[r] >= 0)
            return set_error(VPLMC_EINVAL, "tree: node %d or %d already has a parent", l, r);
        parent[l] = parent[r] = f;
        height[f] = 1 + std::max(height[l], height[r]);
        min_leaf[f] = std::min(min_leaf[l], min_leaf[r]);
    }
    for (int x = 0; x < NC - 1; ++x)
        if (parent[x] < 0) return set_error(VPLMC_EINVAL, "tree: node %d has no parent (one root expected)", x);
    height_max = ns > 0 ? height[NC - 1] : 0;
    std::vector<int32_t> level_off(height_max + 1, 0), order(ns);
    for (int k = 0; k < ns; ++k) level_off[height[ng + k]]++;
    for (int h = 1; h <= height_max; ++h) level_off[h] += level_off[h - 1];
    std::vector<int32_t> fill(level_off.begin(), level_off.end());
    for (int k = 0; k < ns; ++k) order[fill[height[ng + k] - 1]++] = ng + k;
    tree.clear();
    tree.insert(tree.end(), co->left, co->left + ns);
    tree.insert(tree.end(), co->right, co->right + ns);
    tree.insert(tree.end(), parent.begin(), parent.end());
    tree.insert(tree.end(), height.begin(), height.end());
    tree.insert(tree.end(), min_leaf.begin(), min_leaf.end());
    tree.insert(tree.end(), order.begin(), order.end());
    tree.insert(tree.end(), level_off.begin(), level_off.end());
    return VPLMC_OK;
}

static CoarsenTree tree_view(const vplmc_plan *plan, const int32_t *dev) {
    CoarsenTree t;
    const int ng = plan->n_leaves, ns = ng - 1, NC = 2 * ng - 1;
    t.n_leaves = ng;
    t.height_max = plan->height_max;
    t.left = dev;
    t.right = dev + ns;
    t.parent = dev + 2 * ns;
    t.height = dev + 2 * ns + NC;
    t.min_leaf = dev + 2 * ns + 2 * NC;
    t.order = dev + 2 * ns + 3 * NC;
    t.level_off = dev + 3 * ns + 3 * NC;
    return t;
}

// The plan of a frame: the columns of slice s are the cut clusters
// cl_offsets[s] .. cl_offsets[s+1], or (co given) the slice's own coarsening
// of the tree above the cut, at most min(n_leaves, max(q, n_max[s])) nodes.
static int plan_build(int32_t n_slices, const int32_t *pt_offsets, const int32_t *cl_offsets, const int32_t *rank,
                      int32_t n_clusters, const vplmc_params *params, const vplmc_coarsen *co, vplmc_plan **out) {
    if (!out) return set_error(VPLMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_slices < 0) return set_error(VPLMC_EINVAL, "n_slices must be >= 0");
    if (n_slices > 0 && (!pt_offsets || (!co && !cl_offsets) || !rank || (co && !co->n_max)))
        return set_error(VPLMC_EINVAL, "slice layout arrays must be non-NULL");
    if (n_clusters < 0) return set_error(VPLMC_EINVAL, "n_clusters must be >= 0");
    int rc = check_params(params);
    if (rc) return rc;
    if (n_slices > 0 && (pt_offsets[0] != 0 || (!co && cl_offsets[0] != 0)))
        return set_error(VPLMC_EINVAL, "pt_offsets[0] and cl_offsets[0] must be 0");
    vplmc_plan *plan = new (std::nothrow) vplmc_plan();
    if (!plan) return set_error(VPLMC_ENOMEM, "plan allocation failed");
    plan->n_slices = n_slices;
    plan->n_clusters = n_clusters;
    plan->n_lights = n_clusters;
    plan->pass1_ppm = params->pass1_ppm;
    plan->pass2_ppm = params->pass2_ppm;
    plan->als = (params->flags & VPLMC_ALS) != 0;
    if (co) {
        plan->coarse = true;
        plan->n_leaves = co->n_leaves;
        plan->n_lights = 2 * co->n_leaves - 1;
        plan->pixels = co->pixels;
        plan->bound = co->bound;
        if ((rc = build_tree(co, plan->tree, plan->height_max))) {
            delete plan;
            return rc;
        }
    }
    plan->desc.resize(n_slices);
    int64_t o1 = 0, o2 = 0, oo = 0, oc = 0, orow = 0, ocp = 0, ox = 0, oy = 0, obm = 0, obmt = 0, summ = 0;
    int64_t ogrp = 0, oell = 0, nell = 0, opart = 0;
    for (int s = 0; s < n_slices; ++s) {
        const int64_t m = (int64_t)pt_offsets[s + 1] - pt_offsets[s];
        const int q = rank[s];
        if (co && co->n_max[s] < 1) {
            delete plan;
            return set_error(VPLMC_EINVAL, "slice %d: n_max must be >= 1", s);
        }
        const int64_t n = co ? std::min<int64_t>(co->n_leaves, std::max<int64_t>(q, co->n_max[s]))
                             : (int64_t)cl_offsets[s + 1] - cl_offsets[s];
        if (m < 1 || m > VPLMC_MAX_ROWS || n < 1 || n > VPLMC_MAX_COLS) {
            delete plan;
            return set_error(VPLMC_EINVAL, "slice %d: %lld rows x %lld columns outside [1, 65535]", s, (long long)m,
                             (long long)n);
        }
        if (q < 1 || q > VPLMC_MAX_RANK || q > m || q > n) {
            delete plan;
            return set_error(VPLMC_EINVAL, "slice %d: rank %d must be in [1, min(32, %lld, %lld)]", s, q,
                             (long long)m, (long long)n);
        }
        const int bucket = rank_bucket(q);
        const int qp = padded_rank(q);
        const int64_t D = m * n;
        // coarsened slices: capacities (the first pass is the coarsening's
        // row draws, at most `pixels` distinct entries)
        const int64_t N1 = co ? std::min<int64_t>(co->pixels, D) : count_from_ppm(params->pass1_ppm, D);
        int64_t N2 = count_from_ppm(params->pass2_ppm, D);
        if (N2 > D - (co ? 0 : N1)) N2 = D - (co ? 0 : N1);
        if (N1 + N2 > INT32_MAX) {
            delete plan;
            return set_error(VPLMC_EINVAL, "slice %d: %lld samples exceed 2^31 - 1", s, (long long)(N1 + N2));
        }
        SliceDesc &d = plan->desc[s];
        memset(&d, 0, sizeof(d));
        d.m = (int32_t)m;
        d.n = (int32_t)n;
        d.q = qp;
        d.qr = q;
        d.N1 = (int32_t)N1;
        d.N2 = (int32_t)N2;
        d.pt_off = pt_offsets[s];
        d.cl_off = co ? (int32_t)oc : cl_offsets[s];
        d.nmax = co ? co->n_max[s] : 0;
        d.words_row = (int32_t)((n + 31) / 32);
        d.words_col = (int32_t)((m + 31) / 32);
        d.off1 = o1;
        d.off2 = o2;
        d.off_omega = oo;
        d.off_col = oc;
        d.off_row = orow;
        d.off_colptr = ocp;
        d.off_x = ox;
        d.off_y = oy;
        d.off_bm = obm;
        d.off_bmt = obmt;
        // the LDS-resident ADM kernel takes the slices that fit; masked ALS
        // reads every slice's CSR and CSC copies
        const bool in_lds = !plan->als && adm_fits_lds(qp, (int)m);
        d.ell = in_lds ? 1 : 0;
        d.off_grp = (int32_t)ogrp;
        d.off_ell = oell;
        d.off_red = (int64_t)s * ADM_RED_FLOATS;
        d.off_part = opart;
        if (in_lds) {
            // parts: sum_j max(1, ceil(c_j / LMAX)) <= n + |Omega| / LMAX; the padded
            // lengths sum to at most |Omega| + 64 LMAX (lengths sorted descending)
            const int64_t parts = n + (N1 + N2) / ELL_LMAX + 1;
            opart += parts;
            ogrp += (parts + 63) / 64 + 1;
            oell += N1 + N2 + 64 * ELL_LMAX;
            ++nell;
        }
        o1 += N1;
        o2 += N2;
        oo += N1 + N2;
        oc += n;
        orow += m + 1;
        ocp += n + 1;
        ox += m * qp;
        oy += 3 * n * qp;
        obm += m * d.words_row;
        obmt += n * d.words_col;
        summ += m;
        const int grp = 2 * bucket + (in_lds ? 0 : 1);
        plan->groups[grp].push_back(s);
        plan->group_max_m[grp] = std::max<int32_t>(plan->group_max_m[grp], (int32_t)m);
        plan->max_m = std::max<int64_t>(plan->max_m, m);
    }
    // largest slices first in every launch group (longest-processing-time order for
    // the hardware dispatcher and for the work queue); cost as in the multi-GPU split
    for (int g = 0; g < 8; ++g) {
        auto cost = [&](int32_t s) {
            const SliceDesc &d = plan->desc[s];
            const double q = d.q;
            return (double)(d.N1 + d.N2) * (18.0 * q + 40.0) + 2.0 * q * q * (4.0 * d.m + 9.0 * d.n);
        };
        std::stable_sort(plan->groups[g].begin(), plan->groups[g].end(),
                         [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    }
    // global-memory completion: row and column blocks of every slice, as prefixes
    // per group (the launch grids), and the squared-residual slot of each row block
    plan->gblk.clear();
    int64_t e2b = 0;
    for (int g = 1; g < 8; g += 2) {
        plan->gblk_off[g] = (int64_t)plan->gblk.size();
        int64_t r = 0, c = 0;
        plan->gblk.push_back(0);
        for (int32_t sl : plan->groups[g]) {
            r += ((int64_t)plan->desc[sl].m + GADM_RB - 1) / GADM_RB;
            plan->gblk.push_back((int32_t)r);
        }
        plan->gblk.push_back(0);
        for (int32_t sl : plan->groups[g]) {
            c += ((int64_t)plan->desc[sl].n + GADM_CB - 1) / GADM_CB;
            plan->gblk.push_back((int32_t)c);
        }
        plan->g_rows[g] = r;
        plan->g_cols[g] = c;
        plan->ge2_base[g] = e2b;
        e2b += r;
    }
    plan->tot1 = o1;
    plan->tot2 = o2;
    plan->tot_omega = oo;
    plan->tot_col = oc;
    plan->tot_row = orow;
    plan->tot_x = ox;
    plan->tot_y = oy;
    plan->tot_bm = obm;
    plan->tot_bmt = obmt;
    plan->tot_grp = ogrp;
    plan->tot_part = opart;
    plan->tot_ell = oell;
    plan->n_ell = nell;
    if (co && oc > INT32_MAX) {
        delete plan;
        return set_error(VPLMC_EINVAL, "too many columns (%lld)", (long long)oc);
    }
    if (ogrp > INT32_MAX) {
        delete plan;
        return set_error(VPLMC_EINVAL, "too many column groups (%lld)", (long long)ogrp);
    }
    plan->sum_m = summ;
    plan->ids.clear();
    for (int g = 0; g < 8; ++g) plan->ids.insert(plan->ids.end(), plan->groups[g].begin(), plan->groups[g].end());

    Layout &L = plan->layout;
    memset(&L, 0, sizeof(L));
    const int64_t S = n_slices, NC = plan->n_lights;
    size_t bytes[R_INTERNAL_END] = {};
    if (co) {
        const int64_t ng = co->n_leaves, ns = ng - 1;
        bytes[VPLMC_R_COLUMNS] = oc * 4;
        bytes[VPLMC_R_NODE_EPS] = S * ns * 4;
        bytes[VPLMC_R_LEAF_DRAWS] = ng * 4;
        bytes[VPLMC_R_NODE_MEMBERS] = NC * 4;
        bytes[R_TREE] = plan->tree.size() * 4;
        bytes[R_NODE_KD] = 2 * ns * 4;
        bytes[R_LEAF_KPRE] = (ng + 1) * 8;
        bytes[R_NODE_COST] = S * ns * 4;
        bytes[R_NODE_EFF] = S * ns * 4;
        bytes[R_NODE_MERGED] = S * ns;
        bytes[R_NODE_TOP] = S * NC * 4;
        bytes[R_LEAF_COL] = S * ng * 4;
        bytes[R_ZETA] = S * (int64_t)co->pixels * 2;
    }
    bytes[VPLMC_R_LIGHTS] = 9 * NC * 4;
    bytes[VPLMC_R_REP] = NC * 4;
    bytes[VPLMC_R_BBOX] = 6 * NC * 4;
    bytes[VPLMC_R_OMEGA1] = o1 * 4;
    bytes[VPLMC_R_VAL1] = 3 * o1 * 4;
    bytes[VPLMC_R_OMEGA2] = o2 * 4;
    bytes[VPLMC_R_VAL2] = 3 * o2 * 4;
    bytes[VPLMC_R_WEIGHTS] = oc * 4;
    bytes[VPLMC_R_COLMIN] = oc * 4;
    bytes[VPLMC_R_COLMAX] = oc * 4;
    bytes[VPLMC_R_COLCNT] = oc * 4;
    bytes[VPLMC_R_ROW_PTR] = orow * 4;
    bytes[VPLMC_R_CSR_COL] = oo * 4;
    bytes[VPLMC_R_CSR_VAL] = 3 * oo * 4;
    bytes[VPLMC_R_COL_PTR] = ocp * 4;
    bytes[VPLMC_R_CSC_ROW] = oo * 4;
    bytes[VPLMC_R_CSC_VAL] = 3 * oo * 4;
    bytes[VPLMC_R_X] = ox * 4;
    bytes[VPLMC_R_Y] = oy * 4;
    bytes[VPLMC_R_SLICE_SCALE] = S * 4;
    bytes[R_DESC] = S * sizeof(SliceDesc) + S * 4 + plan->gblk.size() * 4;
    bool any_global = false;
    for (int g = 1; g < 8; g += 2) any_global = any_global || !plan->groups[g].empty();
    bytes[R_GSYS] = any_global ? (size_t)S * GADM_SYS_BYTES : 0;
    bytes[R_GE2] = (size_t)e2b * 8;
    bytes[R_COLW_PREFIX] = oc * 8;
    bytes[R_BITMAP] = obm * 4;
    bytes[R_BITMAPT] = obmt * 4;
    bytes[R_WPRE] = obm * 2;
    bytes[R_WPRET] = obmt * 2;
    bytes[R_XNEXT] = ox * 4;
    bytes[R_XP] = ox * 4;
    bytes[R_LAMBDA] = ox * 4;
    bytes[R_YP] = oy * 4;
    bytes[R_PI] = oy * 4;
    bytes[R_SLICE_STATS] = S * 16;
    bytes[R_COLSUM] = oc * 8;
    bytes[R_COLSUMSQ] = oc * 8;
    bytes[R_COLZERO] = oc * 4;
    bytes[R_SLICE_GEO] = S * 8 * 4;
    bytes[R_ELL_PART] = plan->tot_part * 8;
    bytes[R_ELL_PPOS] = plan->tot_part * 4;
    bytes[R_ELL_PBASE] = ocp * 4;
    bytes[R_ELL_PARTIAL] = plan->tot_part * 48 * 4;
    bytes[R_ELL_GRP] = plan->tot_grp * 4;
    bytes[R_ELL_SPLIT] = oc * 4;
    bytes[R_ELL_NSPLIT] = S * 4;
    bytes[R_ELL_ROW] = plan->tot_ell * 2;
    bytes[R_ELL_VAL] = 3 * plan->tot_ell * 4;
    bytes[R_ELL_RES] = 3 * plan->tot_ell * 4;
    bytes[R_YT] = oy * 4;
    bytes[R_ADM_RED] = S * ADM_RED_FLOATS * 4;
    bytes[R_E2PART] = plan->tot_part * 16;   // two halves per part
    bytes[R_QUEUE] = 8 * 4;
    bytes[R_COUNTS] = 4 * 8;
    bytes[VPLMC_R_FEATURES] = oc * MLP_IN * 4;
    bytes[VPLMC_R_LOGITS] = oc * 4;
    size_t off = 0;
    for (int r = 0; r < R_INTERNAL_END; ++r) {
        L.off[r] = off;
        L.bytes[r] = bytes[r];
        off = align256(off + bytes[r]);
    }
    L.total = off;
    // host staging copy of the descriptor table followed by the bucketed slice ids
    plan->upload.resize(bytes[R_DESC]);
    if (n_slices > 0) {
        memcpy(plan->upload.data(), plan->desc.data(), S * sizeof(SliceDesc));
        memcpy(plan->upload.data() + S * sizeof(SliceDesc), plan->ids.data(), S * 4);
        if (!plan->gblk.empty())
            memcpy(plan->upload.data() + S * sizeof(SliceDesc) + S * 4, plan->gblk.data(), plan->gblk.size() * 4);
    }
    *out = plan;
    return VPLMC_OK;
}

int vplmc_plan_create(int32_t n_slices, const int32_t *pt_offsets, const int32_t *cl_offsets, const int32_t *rank,
                      int32_t n_clusters, const vplmc_params *params, vplmc_plan **out) {
    return plan_build(n_slices, pt_offsets, cl_offsets, rank, n_clusters, params, nullptr, out);
}

int vplmc_plan_create_coarse(int32_t n_slices, const int32_t *pt_offsets, const int32_t *rank,
                             const vplmc_coarsen *coarsen, const vplmc_params *params, vplmc_plan **out) {
    if (out) *out = nullptr;
    if (!coarsen) return set_error(VPLMC_EINVAL, "coarsen is NULL");
    if (coarsen->n_leaves < 1 || coarsen->n_leaves > VPLMC_MAX_LEAVES)
        return set_error(VPLMC_EINVAL, "n_leaves must be in [1, %d] (got %d)", VPLMC_MAX_LEAVES, coarsen->n_leaves);
    if (coarsen->pixels < 0 || coarsen->pixels > (1 << 30))
        return set_error(VPLMC_EINVAL, "pixels must be in [0, 2^30] (got %d)", coarsen->pixels);
    if (!(coarsen->bound >= 0.0)) return set_error(VPLMC_EINVAL, "bound must be >= 0");
    if (coarsen->reserved != 0) return set_error(VPLMC_EINVAL, "reserved must be 0");
    return plan_build(n_slices, pt_offsets, nullptr, rank, coarsen->n_leaves, params, coarsen, out);
}

int vplmc_plan_destroy(vplmc_plan *plan) {
    delete plan;
    return VPLMC_OK;
}

int vplmc_workspace_size(const vplmc_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(VPLMC_EINVAL, "plan and bytes must be non-NULL");
    *bytes = plan->layout.total;
    return VPLMC_OK;
}

int vplmc_plan_slice(const vplmc_plan *plan, int32_t s, vplmc_slice_info *out) {
    if (!plan || !out) return set_error(VPLMC_EINVAL, "plan and out must be non-NULL");
    if (s < 0 || s >= plan->n_slices) return set_error(VPLMC_EINVAL, "slice %d out of range", s);
    const SliceDesc &d = plan->desc[s];
    out->m = d.m;
    out->n = d.n;
    out->q = d.qr;
    out->q_pad = d.q;
    out->N1 = d.N1;
    out->N2 = d.N2;
    out->adm_in_lds = d.ell;
    out->off1 = d.off1;
    out->off2 = d.off2;
    out->off_omega = d.off_omega;
    out->off_col = d.off_col;
    out->off_row = d.off_row;
    out->off_colptr = d.off_colptr;
    out->off_x = d.off_x;
    out->off_y = d.off_y;
    return VPLMC_OK;
}

int vplmc_plan_region(const vplmc_plan *plan, int32_t region, size_t *offset, size_t *bytes) {
    if (!plan || !offset || !bytes) return set_error(VPLMC_EINVAL, "plan, offset and bytes must be non-NULL");
    if (region < 0 || region >= VPLMC_R_COUNT) return set_error(VPLMC_EINVAL, "unknown region %d", region);
    *offset = plan->layout.off[region];
    *bytes = plan->layout.bytes[region];
    return VPLMC_OK;
}

int vplmc_render(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points, const vplmc_lights *vpls,
                 const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params,
                 void *workspace, size_t workspace_bytes, float *radiance) {
    if (!ctx || !plan || !points || !vpls || !cut || !params)
        return set_error(VPLMC_EINVAL, "ctx, plan, points, vpls, cut and params must be non-NULL");
    int rc = check_params(params);
    if (rc) return rc;
    if (params->pass1_ppm != plan->pass1_ppm || params->pass2_ppm != plan->pass2_ppm)
        return set_error(VPLMC_EINVAL, "params rates differ from the plan's");
    if (((params->flags & VPLMC_ALS) != 0) != plan->als)
        return set_error(VPLMC_EINVAL, "the completion method (VPLMC_ALS) differs from the plan's");
    if (points->m < 0 || bad_ptrs_points(points)) return set_error(VPLMC_EINVAL, "incomplete points arrays");
    if (vpls->n < 1 || bad_ptrs_lights(vpls)) return set_error(VPLMC_EINVAL, "incomplete VPL arrays");
    if (cut->n_clusters != plan->n_clusters || !cut->offsets || !cut->members)
        return set_error(VPLMC_EINVAL, "cut does not match the plan (%d clusters planned)", plan->n_clusters);
    if (plan->n_slices > 0 && (!pt_ids || (!cl_ids && !plan->coarse)))
        return set_error(VPLMC_EINVAL, "pt_ids and cl_ids must be non-NULL");
    if (!radiance) return set_error(VPLMC_EINVAL, "radiance is NULL");
    if (!workspace || workspace_bytes < plan->layout.total)
        return set_error(VPLMC_EINVAL, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes,
                         plan->layout.total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return set_error(VPLMC_EINVAL, "workspace must be 256-byte aligned");
    if (plan->sum_m > points->m) return set_error(VPLMC_EINVAL, "slices hold more rows than there are points");
    VPLMC_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    void *ws = workspace;
    const int S = plan->n_slices;
    PhaseMarks ph(ctx);
    if ((rc = ph.mark(VPLMC_PH_SETUP))) return rc;

    SliceDesc *desc = region<SliceDesc>(ws, plan, R_DESC);
    const int32_t *ids = reinterpret_cast<const int32_t *>(desc + S);
    // (a captured frame reuses the tables uploaded by the eager frame before the capture)
    if (S > 0 && !ctx->capturing)
        VPLMC_HIP(hipMemcpyAsync(desc, plan->upload.data(), plan->upload.size(), hipMemcpyHostToDevice, st));
    if (plan->coarse && !plan->tree.empty() && !ctx->capturing)
        VPLMC_HIP(hipMemcpyAsync(region<int32_t>(ws, plan, R_TREE), plan->tree.data(), plan->tree.size() * 4,
                                 hipMemcpyHostToDevice, st));

    uint32_t *bm = region<uint32_t>(ws, plan, R_BITMAP);
    uint32_t *bmt = region<uint32_t>(ws, plan, R_BITMAPT);
    int32_t *cnt = region<int32_t>(ws, plan, VPLMC_R_COLCNT);
    float *mn = region<float>(ws, plan, VPLMC_R_COLMIN);
    float *mx = region<float>(ws, plan, VPLMC_R_COLMAX);
    int32_t *stats = region<int32_t>(ws, plan, R_SLICE_STATS);
    if ((rc = launch_fill_u32(st, bm, plan->tot_bm, 0u))) return rc;
    if ((rc = launch_fill_u32(st, bmt, plan->tot_bmt, 0u))) return rc;
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(stats), 4 * (size_t)S, 0u))) return rc;
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(radiance), 3 * (size_t)points->m, 0u))) return rc;
    unsigned long long *counts = region<unsigned long long>(ws, plan, R_COUNTS);
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(counts), 8, 0u))) return rc;

    if ((rc = ph.mark(VPLMC_PH_CLUSTER))) return rc;
    float *lights = region<float>(ws, plan, VPLMC_R_LIGHTS);
    int32_t *rep = region<int32_t>(ws, plan, VPLMC_R_REP);
    float *bbox = region<float>(ws, plan, VPLMC_R_BBOX);
    if ((rc = launch_cluster_table(st, *vpls, *cut, params->seed, rep, lights, bbox, plan->n_lights))) return rc;
    uint32_t *omega1 = region<uint32_t>(ws, plan, VPLMC_R_OMEGA1);
    float *val1 = region<float>(ws, plan, VPLMC_R_VAL1);
    uint32_t *omega2 = region<uint32_t>(ws, plan, VPLMC_R_OMEGA2);
    float *val2 = region<float>(ws, plan, VPLMC_R_VAL2);
    const int32_t *node_members = nullptr;
    if (plan->coarse) {
        // light coarsening (Sec. 4): node table, row draws and merge errors,
        // merge decisions and columns, then the first pass from the draws
        const CoarsenTree tr = tree_view(plan, region<int32_t>(ws, plan, R_TREE));
        const int ng = plan->n_leaves, ns = ng - 1;
        int32_t *kd = region<int32_t>(ws, plan, R_NODE_KD);
        int32_t *members = region<int32_t>(ws, plan, VPLMC_R_NODE_MEMBERS);
        node_members = members;
        if ((rc = launch_node_table(st, tr, cut->offsets, params->seed, rep, lights, bbox, members, kd, kd + ns)))
            return rc;
        CoarsenSlices cs;
        cs.eps = region<float>(ws, plan, VPLMC_R_NODE_EPS);
        cs.cost = region<float>(ws, plan, R_NODE_COST);
        cs.eff = region<float>(ws, plan, R_NODE_EFF);
        cs.merged = region<uint8_t>(ws, plan, R_NODE_MERGED);
        cs.top = region<int32_t>(ws, plan, R_NODE_TOP);
        cs.leaf_col = region<int32_t>(ws, plan, R_LEAF_COL);
        cs.kept = kd;
        cs.dropped = kd + ns;
        int64_t *kpre = region<int64_t>(ws, plan, R_LEAF_KPRE);
        cs.kpre = kpre;
        cs.zeta = region<uint16_t>(ws, plan, R_ZETA);
        if ((rc = launch_leaf_draws(st, ng, lights, plan->pixels, region<int32_t>(ws, plan, VPLMC_R_LEAF_DRAWS),
                                    kpre)))
            return rc;
        if ((rc = ph.mark(VPLMC_PH_COARSEN))) return rc;
        if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(cs.eps), (size_t)S * ns, 0u))) return rc;
        if ((rc = launch_coarsen_eps(st, *plan, ctx->bvh, *points, lights, desc, pt_ids, tr, cs, *params, ctx->n_cu,
                                     counts + 1)))
            return rc;
        int32_t *columns = region<int32_t>(ws, plan, VPLMC_R_COLUMNS);
        if ((rc = launch_coarsen_merge(st, *plan, desc, tr, cs, columns))) return rc;
        cl_ids = columns;
        if ((rc = ph.mark(VPLMC_PH_PASS1))) return rc;
        if ((rc = launch_coarsen_pass1(st, *plan, desc, cs, bm, bmt, region<int32_t>(ws, plan, VPLMC_R_ROW_PTR),
                                       omega1)))
            return rc;
    } else {
        if ((rc = ph.mark(VPLMC_PH_COARSEN))) return rc;
        if ((rc = ph.mark(VPLMC_PH_PASS1))) return rc;
        if ((rc = launch_pass1(st, *plan, desc, params->seed, omega1, bm, bmt))) return rc;
    }
    if ((rc = ph.mark(VPLMC_PH_EVAL1))) return rc;
    if ((rc = launch_eval_omega(st, ctx->bvh, *points, lights, plan->n_lights, desc, S, pt_ids, cl_ids, omega1,
                                plan->tot1, 0, stats, *params, val1, plan->tune.eval_threads, ctx->n_cu, counts)))
        return rc;
    if ((rc = ph.mark(VPLMC_PH_WEIGHTS))) return rc;
    int32_t *col_ptr = region<int32_t>(ws, plan, VPLMC_R_COL_PTR);
    int32_t *csc_row = region<int32_t>(ws, plan, VPLMC_R_CSC_ROW);
    float *csc_val = region<float>(ws, plan, VPLMC_R_CSC_VAL);
    double *csum = region<double>(ws, plan, R_COLSUM);
    double *csumsq = region<double>(ws, plan, R_COLSUMSQ);
    int32_t *czero = region<int32_t>(ws, plan, R_COLZERO);
    if ((rc = launch_colstats(st, *plan, desc, omega1, val1, bmt, region<uint16_t>(ws, plan, R_WPRET), col_ptr, csc_row,
                              csc_val, cnt, mn, mx, csum, csumsq, czero)))
        return rc;
    const bool learned = (params->flags & VPLMC_LEARNED) != 0;
    const float *logits = nullptr;
    if (learned || (params->flags & VPLMC_FEATURES)) {
        float *feat = region<float>(ws, plan, VPLMC_R_FEATURES);
        if ((rc = launch_features(st, *plan, desc, *points, pt_ids, cl_ids, lights, bbox, *cut, node_members, cnt, mn,
                                  mx, csum, csumsq, czero, region<float>(ws, plan, R_SLICE_GEO), feat)))
            return rc;
        if (learned) {
            float *lg = region<float>(ws, plan, VPLMC_R_LOGITS);
            if (ctx->mlp) {
                if ((rc = launch_mlp_forward(st, ctx->mlp, plan->tot_col, feat, lg))) return rc;
            } else {
                // no model: every logit non-finite, every slice falls back to the g weights
                if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(lg), plan->tot_col, 0x7FC00000u))) return rc;
            }
            logits = lg;
        }
    }
    uint64_t *prefix = region<uint64_t>(ws, plan, R_COLW_PREFIX);
    if ((rc = launch_weights(st, *plan, desc, cnt, mn, mx, logits, params->pass2_mix,
                             region<uint32_t>(ws, plan, VPLMC_R_WEIGHTS), prefix, stats)))
        return rc;
    if ((rc = ph.mark(VPLMC_PH_PASS2))) return rc;
    if ((rc = launch_pass2(st, *plan, desc, params->seed, prefix, bm, bmt, omega2, stats))) return rc;
    if ((rc = ph.mark(VPLMC_PH_EVAL2))) return rc;
    if ((rc = launch_eval_omega(st, ctx->bvh, *points, lights, plan->n_lights, desc, S, pt_ids, cl_ids, omega2,
                                plan->tot2, 1, stats, *params, val2, plan->tune.eval_threads, ctx->n_cu, counts)))
        return rc;
    if ((rc = ph.mark(VPLMC_PH_SORT))) return rc;
    int32_t *row_ptr = region<int32_t>(ws, plan, VPLMC_R_ROW_PTR);
    int32_t *csr_col = region<int32_t>(ws, plan, VPLMC_R_CSR_COL);
    float *csr_val = region<float>(ws, plan, VPLMC_R_CSR_VAL);
    EllView ell;
    ell.part = region<int2>(ws, plan, R_ELL_PART);
    ell.ppos = region<int32_t>(ws, plan, R_ELL_PPOS);
    ell.pbase = region<int32_t>(ws, plan, R_ELL_PBASE);
    ell.partial = region<float>(ws, plan, R_ELL_PARTIAL);
    ell.grp = region<int32_t>(ws, plan, R_ELL_GRP);
    ell.split = region<int32_t>(ws, plan, R_ELL_SPLIT);
    ell.nsplit = region<int32_t>(ws, plan, R_ELL_NSPLIT);
    ell.row = plan->tot_ell > 0 ? region<uint16_t>(ws, plan, R_ELL_ROW) : nullptr;
    ell.val = region<float>(ws, plan, R_ELL_VAL);
    ell.res = region<float>(ws, plan, R_ELL_RES);
    if ((rc = launch_sort(st, *plan, desc, bm, bmt, region<uint16_t>(ws, plan, R_WPRE), region<uint16_t>(ws, plan, R_WPRET),
                          row_ptr, col_ptr, omega1, val1, omega2, val2, stats, csr_col, csr_val, csc_row, csc_val,
                          ell)))
        return rc;
    float *X = region<float>(ws, plan, VPLMC_R_X);
    float *Y = region<float>(ws, plan, VPLMC_R_Y);
    float *scale = region<float>(ws, plan, VPLMC_R_SLICE_SCALE);
    if ((rc = ph.mark(VPLMC_PH_ADM))) return rc;
    if (plan->als)
        rc = launch_als(st, *plan, desc, ids, *params, row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, X, Y,
                        scale, stats);
    else
        rc = launch_adm(st, &ctx->adm, *plan, ctx->n_cu, desc, ids, ids + S, region<char>(ws, plan, R_GSYS),
                        region<double>(ws, plan, R_GE2), region<int32_t>(ws, plan, R_QUEUE), *params,
                        row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, ell, X, region<float>(ws, plan, R_XNEXT),
                        region<float>(ws, plan, R_XP), region<float>(ws, plan, R_LAMBDA), Y,
                        region<float>(ws, plan, R_YP), region<float>(ws, plan, R_PI), region<float>(ws, plan, R_YT),
                        region<float>(ws, plan, R_ADM_RED), region<double>(ws, plan, R_E2PART), scale, stats);
    if (rc) return rc;
    if ((rc = ph.mark(VPLMC_PH_REDUCE))) return rc;
    if ((rc = launch_reduce(st, *plan, desc, pt_ids, X, Y, scale, points->m, radiance))) return rc;
    if ((rc = ph.mark(VPLMC_N_PHASES))) return rc;
    ph.done();
    return VPLMC_OK;
}

int vplmc_render_static(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points,
                        const vplmc_lights *vpls, const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids,
                        const vplmc_params *params, float *radiance) {
    if (!ctx || !plan) return set_error(VPLMC_EINVAL, "ctx and plan must be non-NULL");
    if (plan->layout.total > VPLMC_STATIC_WORKSPACE_BYTES)
        return set_error(VPLMC_EINVAL, "frame needs a %zu-byte workspace, above the %zu-byte static workspace "
                         "(use vplmc_render with a caller workspace)", plan->layout.total,
                         (size_t)VPLMC_STATIC_WORKSPACE_BYTES);
    if (!ctx->scratch) return set_error(VPLMC_EHIP, "static workspace address unknown");
    // the same frame as vplmc_render, on the device array: every buffer the
    // frame reads before writing is cleared by its fill kernels, so the
    // previous call's contents do not matter
    return vplmc_render(ctx, plan, points, vpls, cut, pt_ids, cl_ids, params, ctx->scratch,
                        (size_t)VPLMC_STATIC_WORKSPACE_BYTES, radiance);
}

static int check_tune(const vplmc_tune *t) {
    if (!t) return set_error(VPLMC_EINVAL, "tune is NULL");
    if (t->adm_queue != 0 && t->adm_queue != 1) return set_error(VPLMC_EINVAL, "adm_queue must be 0 or 1");
    if (t->adm_threads != 512 && t->adm_threads != 1024) return set_error(VPLMC_EINVAL, "adm_threads must be 512 or 1024");
    if (t->eval_threads != 64 && t->eval_threads != 128 && t->eval_threads != 256)
        return set_error(VPLMC_EINVAL, "eval_threads must be 64, 128 or 256");
    if (t->reserved != 0) return set_error(VPLMC_EINVAL, "reserved must be 0");
    return VPLMC_OK;
}

int vplmc_plan_get_tune(const vplmc_plan *plan, vplmc_tune *out) {
    if (!plan || !out) return set_error(VPLMC_EINVAL, "plan and out must be non-NULL");
    *out = plan->tune;
    return VPLMC_OK;
}

int vplmc_plan_set_tune(vplmc_plan *plan, const vplmc_tune *tune) {
    if (!plan) return set_error(VPLMC_EINVAL, "plan is NULL");
    int rc = check_tune(tune);
    if (rc) return rc;
    plan->tune = *tune;
    return VPLMC_OK;
}

int vplmc_autotune(vplmc_ctx *ctx, vplmc_plan *plan, const vplmc_points *points, const vplmc_lights *vpls,
                   const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params,
                   void *workspace, size_t workspace_bytes, float *radiance, int32_t reps, vplmc_tune *best) {
    if (!ctx || !plan) return set_error(VPLMC_EINVAL, "ctx and plan must be non-NULL");
    if (reps < 1 || reps > 100) return set_error(VPLMC_EINVAL, "reps must be in [1, 100]");
    if (ctx->prof_on) return set_error(VPLMC_EINVAL, "profiling is on");
    VPLMC_HIP(hipSetDevice(ctx->device));
    hipEvent_t e0, e1;
    VPLMC_HIP(hipEventCreate(&e0));
    VPLMC_HIP(hipEventCreate(&e1));
    auto time_of = [&](const vplmc_tune &t, float &ms) -> int {
        plan->tune = t;
        int rc = vplmc_render(ctx, plan, points, vpls, cut, pt_ids, cl_ids, params, workspace, workspace_bytes,
                              radiance);
        if (rc) return rc;
        VPLMC_HIP(hipEventRecord(e0, ctx->stream));
        for (int k = 0; k < reps && !rc; ++k)
            rc = vplmc_render(ctx, plan, points, vpls, cut, pt_ids, cl_ids, params, workspace, workspace_bytes,
                              radiance);
        if (rc) return rc;
        VPLMC_HIP(hipEventRecord(e1, ctx->stream));
        VPLMC_HIP(hipEventSynchronize(e1));
        VPLMC_HIP(hipEventElapsedTime(&ms, e0, e1));
        return VPLMC_OK;
    };
    const vplmc_tune start = plan->tune;
    vplmc_tune cur = start;
    float cur_ms = 0.f;
    int rc = time_of(cur, cur_ms);
    // coordinate descent: completion launch (queue x threads), then entry block size
    const vplmc_tune adm_cands[4] = {{0, 1024, 0, 0}, {1, 1024, 0, 0}, {0, 512, 0, 0}, {1, 512, 0, 0}};
    for (int k = 0; k < 4 && !rc; ++k) {
        vplmc_tune t = cur;
        t.adm_queue = adm_cands[k].adm_queue;
        t.adm_threads = adm_cands[k].adm_threads;
        if (t.adm_queue == cur.adm_queue && t.adm_threads == cur.adm_threads) continue;
        float ms;
        if ((rc = time_of(t, ms))) break;
        if (ms < cur_ms) {
            cur = t;
            cur_ms = ms;
        }
    }
    const int eval_cands[3] = {64, 128, 256};
    for (int k = 0; k < 3 && !rc; ++k) {
        if (eval_cands[k] == cur.eval_threads) continue;
        vplmc_tune t = cur;
        t.eval_threads = eval_cands[k];
        float ms;
        if ((rc = time_of(t, ms))) break;
        if (ms < cur_ms) {
            cur = t;
            cur_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->tune = rc ? start : cur;
    if (rc) return rc;
    if (best) *best = cur;
    return VPLMC_OK;
}

struct vplmc_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int vplmc_graph_create(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points, const vplmc_lights *vpls,
                       const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params,
                       void *workspace, size_t workspace_bytes, float *radiance, vplmc_graph **out) {
    if (!out) return set_error(VPLMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    if (ctx->prof_on) return set_error(VPLMC_EINVAL, "profiling is on");
    // one eager frame: validates everything and uploads the slice table
    int rc = vplmc_render(ctx, plan, points, vpls, cut, pt_ids, cl_ids, params, workspace, workspace_bytes, radiance);
    if (rc) return rc;
    VPLMC_HIP(hipStreamSynchronize(ctx->stream));
    hipStream_t cs;
    VPLMC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = cs;
    ctx->capturing = true;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        rc = vplmc_render(ctx, plan, points, vpls, cut, pt_ids, cl_ids, params, workspace, workspace_bytes, radiance);
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e2 != hipSuccess && !rc) e = e2;
    }
    ctx->stream = saved;
    ctx->capturing = false;
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : hip_error(e, "stream capture");
    }
    vplmc_graph *gr = new (std::nothrow) vplmc_graph();
    if (!gr) {
        (void)hipGraphDestroy(g);
        return set_error(VPLMC_ENOMEM, "graph allocation failed");
    }
    gr->device = ctx->device;
    gr->graph = g;
    e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete gr;
        return hip_error(e, "graph instantiate");
    }
    *out = gr;
    return VPLMC_OK;
}

int vplmc_graph_launch(vplmc_ctx *ctx, vplmc_graph *graph) {
    if (!ctx || !graph) return set_error(VPLMC_EINVAL, "ctx and graph must be non-NULL");
    if (graph->device != ctx->device) return set_error(VPLMC_EINVAL, "graph was captured on another device");
    VPLMC_HIP(hipSetDevice(ctx->device));
    VPLMC_HIP(hipGraphLaunch(graph->exec, ctx->stream));
    return VPLMC_OK;
}

int vplmc_graph_destroy(vplmc_graph *graph) {
    if (!graph) return VPLMC_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return VPLMC_OK;
}

int vplmc_profile_begin(vplmc_ctx *ctx, int32_t max_frames) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    if (max_frames < 1 || max_frames > 4096) return set_error(VPLMC_EINVAL, "max_frames must be in [1, 4096]");
    VPLMC_HIP(hipSetDevice(ctx->device));
    const size_t need = (size_t)max_frames * (VPLMC_N_PHASES + 1);
    while (ctx->prof_events.size() < need) {
        hipEvent_t e;
        VPLMC_HIP(hipEventCreate(&e));
        ctx->prof_events.push_back(e);
    }
    ctx->prof_max_frames = max_frames;
    ctx->prof_frames = 0;
    ctx->prof_on = true;
    return VPLMC_OK;
}

int vplmc_profile_end(vplmc_ctx *ctx, double *ms, int32_t *frames) {
    if (!ctx || !ms || !frames) return set_error(VPLMC_EINVAL, "ctx, ms and frames must be non-NULL");
    VPLMC_HIP(hipSetDevice(ctx->device));
    VPLMC_HIP(hipStreamSynchronize(ctx->stream));
    for (int p = 0; p < VPLMC_N_PHASES; ++p) ms[p] = 0.0;
    for (int f = 0; f < ctx->prof_frames; ++f) {
        hipEvent_t *ev = &ctx->prof_events[(size_t)f * (VPLMC_N_PHASES + 1)];
        for (int p = 0; p < VPLMC_N_PHASES; ++p) {
            float t = 0.f;
            VPLMC_HIP(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
            ms[p] += t;
        }
    }
    *frames = ctx->prof_frames;
    ctx->prof_on = false;
    ctx->prof_frames = 0;
    return VPLMC_OK;
}

int vplmc_read_stats(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace, int32_t *iters, int32_t *flags,
                     float *resid, int32_t *n2_accepted) {
    if (!ctx || !plan || !workspace) return set_error(VPLMC_EINVAL, "ctx, plan and workspace must be non-NULL");
    const int S = plan->n_slices;
    std::vector<int32_t> h(4 * (size_t)S);
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (S > 0) {
        VPLMC_HIP(hipMemcpyAsync(h.data(), static_cast<const char *>(workspace) + plan->layout.off[R_SLICE_STATS],
                                 h.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    }
    VPLMC_HIP(hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < S; ++s) {
        if (iters) iters[s] = h[4 * s];
        if (flags) flags[s] = h[4 * s + 1];
        if (resid) memcpy(&resid[s], &h[4 * s + 2], 4);
        if (n2_accepted) n2_accepted[s] = h[4 * s + 3];
    }
    return VPLMC_OK;
}

int vplmc_read_counts(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace, int32_t *n, int32_t *N1,
                      int32_t *N2) {
    if (!ctx || !plan || !workspace) return set_error(VPLMC_EINVAL, "ctx, plan and workspace must be non-NULL");
    const int S = plan->n_slices;
    std::vector<SliceDesc> h(S);
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (S > 0)
        VPLMC_HIP(hipMemcpyAsync(h.data(), static_cast<const char *>(workspace) + plan->layout.off[R_DESC],
                                 S * sizeof(SliceDesc), hipMemcpyDeviceToHost, ctx->stream));
    VPLMC_HIP(hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < S; ++s) {
        if (n) n[s] = h[s].n;
        if (N1) N1[s] = h[s].N1;
        if (N2) N2[s] = h[s].N2;
    }
    return VPLMC_OK;
}

// ---- stage calls: the frame's kernels on inputs placed in the workspace ----

namespace {

// validates a stage call's common arguments and uploads the slice table
int stage_setup(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_params *params, void *ws, size_t bytes) {
    if (!ctx || !plan || !params || !ws) return set_error(VPLMC_EINVAL, "ctx, plan, params and workspace must be non-NULL");
    if (plan->coarse) return set_error(VPLMC_EUNSUPPORTED, "stage calls take plans without coarsening");
    int rc = check_params(params);
    if (rc) return rc;
    if (bytes < plan->layout.total) return set_error(VPLMC_EINVAL, "workspace smaller than vplmc_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(VPLMC_EINVAL, "workspace must be 256-byte aligned");
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (plan->n_slices > 0)
        VPLMC_HIP(hipMemcpyAsync(region<char>(ws, plan, R_DESC), plan->upload.data(), plan->upload.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    return VPLMC_OK;
}

// occupancy bitmaps from the first-pass keys in OMEGA1; EINVAL if a key lies
// outside its slice or repeats (synchronises)
int stage_bitmaps(vplmc_ctx *ctx, const vplmc_plan *plan, void *ws) {
    hipStream_t st = ctx->stream;
    uint32_t *bm = region<uint32_t>(ws, plan, R_BITMAP);
    uint32_t *bmt = region<uint32_t>(ws, plan, R_BITMAPT);
    unsigned long long *bad = region<unsigned long long>(ws, plan, R_COUNTS);
    int rc;
    if ((rc = launch_fill_u32(st, bm, plan->tot_bm, 0u))) return rc;
    if ((rc = launch_fill_u32(st, bmt, plan->tot_bmt, 0u))) return rc;
    if ((rc = launch_fill_u32(st, region<uint32_t>(ws, plan, R_SLICE_STATS), 4 * (size_t)plan->n_slices, 0u))) return rc;
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(bad), 8, 0u))) return rc;
    if ((rc = launch_keys_bitmap(st, *plan, region<SliceDesc>(ws, plan, R_DESC),
                                 region<uint32_t>(ws, plan, VPLMC_R_OMEGA1), bm, bmt, bad)))
        return rc;
    unsigned long long h = 0;
    VPLMC_HIP(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, st));
    VPLMC_HIP(hipStreamSynchronize(st));
    if (h) return set_error(VPLMC_EINVAL, "%llu first-pass entries lie outside their slice or repeat", h);
    return VPLMC_OK;
}

}  // namespace

int vplmc_stage_pass2(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_params *params, void *workspace,
                      size_t workspace_bytes) {
    int rc = stage_setup(ctx, plan, params, workspace, workspace_bytes);
    if (rc) return rc;
    if (params->pass2_ppm != plan->pass2_ppm) return set_error(VPLMC_EINVAL, "params rates differ from the plan's");
    if ((rc = stage_bitmaps(ctx, plan, workspace))) return rc;
    hipStream_t st = ctx->stream;
    SliceDesc *desc = region<SliceDesc>(workspace, plan, R_DESC);
    uint64_t *prefix = region<uint64_t>(workspace, plan, R_COLW_PREFIX);
    if ((rc = launch_prefix_given(st, *plan, desc, region<uint32_t>(workspace, plan, VPLMC_R_WEIGHTS), prefix)))
        return rc;
    if ((rc = launch_pass2(st, *plan, desc, params->seed, prefix, region<uint32_t>(workspace, plan, R_BITMAP),
                           region<uint32_t>(workspace, plan, R_BITMAPT), region<uint32_t>(workspace, plan, VPLMC_R_OMEGA2),
                           region<int32_t>(workspace, plan, R_SLICE_STATS))))
        return rc;
    VPLMC_HIP(hipStreamSynchronize(st));
    return VPLMC_OK;
}

int vplmc_stage_adm(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_params *params, const int32_t *pt_ids,
                    int32_t n_points, void *workspace, size_t workspace_bytes, float *radiance) {
    int rc = stage_setup(ctx, plan, params, workspace, workspace_bytes);
    if (rc) return rc;
    if (!radiance || (plan->n_slices > 0 && !pt_ids)) return set_error(VPLMC_EINVAL, "radiance and pt_ids must be non-NULL");
    if (n_points < plan->sum_m) return set_error(VPLMC_EINVAL, "slices hold more rows than there are points");
    if ((rc = stage_bitmaps(ctx, plan, workspace))) return rc;
    hipStream_t st = ctx->stream;
    void *ws = workspace;
    SliceDesc *desc = region<SliceDesc>(ws, plan, R_DESC);
    const int32_t *ids = reinterpret_cast<const int32_t *>(desc + plan->n_slices);
    EllView ell;
    ell.part = region<int2>(ws, plan, R_ELL_PART);
    ell.ppos = region<int32_t>(ws, plan, R_ELL_PPOS);
    ell.pbase = region<int32_t>(ws, plan, R_ELL_PBASE);
    ell.partial = region<float>(ws, plan, R_ELL_PARTIAL);
    ell.grp = region<int32_t>(ws, plan, R_ELL_GRP);
    ell.split = region<int32_t>(ws, plan, R_ELL_SPLIT);
    ell.nsplit = region<int32_t>(ws, plan, R_ELL_NSPLIT);
    ell.row = plan->tot_ell > 0 ? region<uint16_t>(ws, plan, R_ELL_ROW) : nullptr;
    ell.val = region<float>(ws, plan, R_ELL_VAL);
    ell.res = region<float>(ws, plan, R_ELL_RES);
    int32_t *stats = region<int32_t>(ws, plan, R_SLICE_STATS);
    int32_t *row_ptr = region<int32_t>(ws, plan, VPLMC_R_ROW_PTR);
    int32_t *col_ptr = region<int32_t>(ws, plan, VPLMC_R_COL_PTR);
    int32_t *csr_col = region<int32_t>(ws, plan, VPLMC_R_CSR_COL);
    float *csr_val = region<float>(ws, plan, VPLMC_R_CSR_VAL);
    int32_t *csc_row = region<int32_t>(ws, plan, VPLMC_R_CSC_ROW);
    float *csc_val = region<float>(ws, plan, VPLMC_R_CSC_VAL);
    // the second pass is empty (accepted count 0 from the cleared stats)
    if ((rc = launch_sort(st, *plan, desc, region<uint32_t>(ws, plan, R_BITMAP), region<uint32_t>(ws, plan, R_BITMAPT),
                          region<uint16_t>(ws, plan, R_WPRE), region<uint16_t>(ws, plan, R_WPRET), row_ptr, col_ptr,
                          region<uint32_t>(ws, plan, VPLMC_R_OMEGA1), region<float>(ws, plan, VPLMC_R_VAL1),
                          region<uint32_t>(ws, plan, VPLMC_R_OMEGA2), region<float>(ws, plan, VPLMC_R_VAL2), stats,
                          csr_col, csr_val, csc_row, csc_val, ell)))
        return rc;
    float *X = region<float>(ws, plan, VPLMC_R_X);
    float *Y = region<float>(ws, plan, VPLMC_R_Y);
    float *scale = region<float>(ws, plan, VPLMC_R_SLICE_SCALE);
    if (plan->als)
        rc = launch_als(st, *plan, desc, ids, *params, row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, X, Y,
                        scale, stats);
    else
        rc = launch_adm(st, &ctx->adm, *plan, ctx->n_cu, desc, ids, ids + plan->n_slices, region<char>(ws, plan, R_GSYS),
                        region<double>(ws, plan, R_GE2), region<int32_t>(ws, plan, R_QUEUE), *params,
                        row_ptr, csr_col, csr_val, col_ptr, csc_row, csc_val, ell, X, region<float>(ws, plan, R_XNEXT),
                        region<float>(ws, plan, R_XP), region<float>(ws, plan, R_LAMBDA), Y,
                        region<float>(ws, plan, R_YP), region<float>(ws, plan, R_PI), region<float>(ws, plan, R_YT),
                        region<float>(ws, plan, R_ADM_RED), region<double>(ws, plan, R_E2PART), scale, stats);
    if (rc) return rc;
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(radiance), 3 * (size_t)n_points, 0u))) return rc;
    if ((rc = launch_reduce(st, *plan, desc, pt_ids, X, Y, scale, n_points, radiance))) return rc;
    VPLMC_HIP(hipStreamSynchronize(st));
    return VPLMC_OK;
}

int vplmc_stage_reduce(vplmc_ctx *ctx, const vplmc_plan *plan, const int32_t *pt_ids, int32_t n_points,
                       void *workspace, size_t workspace_bytes, float *radiance) {
    vplmc_params p;
    vplmc_default_params(&p);
    p.pass1_ppm = plan ? plan->pass1_ppm : 0;
    p.pass2_ppm = plan ? plan->pass2_ppm : 0;
    int rc = stage_setup(ctx, plan, &p, workspace, workspace_bytes);
    if (rc) return rc;
    if (!radiance || (plan->n_slices > 0 && !pt_ids)) return set_error(VPLMC_EINVAL, "radiance and pt_ids must be non-NULL");
    if (n_points < plan->sum_m) return set_error(VPLMC_EINVAL, "slices hold more rows than there are points");
    hipStream_t st = ctx->stream;
    if ((rc = launch_fill_u32(st, reinterpret_cast<uint32_t *>(radiance), 3 * (size_t)n_points, 0u))) return rc;
    return launch_reduce(st, *plan, region<SliceDesc>(workspace, plan, R_DESC), pt_ids,
                         region<float>(workspace, plan, VPLMC_R_X), region<float>(workspace, plan, VPLMC_R_Y),
                         region<float>(workspace, plan, VPLMC_R_SLICE_SCALE), n_points, radiance);
}

int vplmc_full_matrix(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points, const float *lights,
                      int32_t n_lights, const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params,
                      int32_t slice_begin, int32_t slice_end, float *out) {
    if (!ctx || !plan || !points || !lights || !params || !out) return set_error(VPLMC_EINVAL, "NULL argument");
    if (plan->coarse) return set_error(VPLMC_EUNSUPPORTED, "full matrices need a plan with fixed cluster columns");
    if (bad_ptrs_points(points)) return set_error(VPLMC_EINVAL, "incomplete points arrays");
    if (n_lights < 1) return set_error(VPLMC_EINVAL, "n_lights must be >= 1");
    if (slice_begin < 0 || slice_end > plan->n_slices || slice_begin > slice_end)
        return set_error(VPLMC_EINVAL, "slice range [%d, %d) outside [0, %d]", slice_begin, slice_end, plan->n_slices);
    if (slice_end > slice_begin && (!pt_ids || !cl_ids)) return set_error(VPLMC_EINVAL, "pt_ids and cl_ids must be non-NULL");
    int rc = check_params(params);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    int64_t o = 0;
    for (int s = slice_begin; s < slice_end; ++s) {
        const SliceDesc &d = plan->desc[s];
        if ((rc = launch_full_matrix(ctx->stream, ctx->bvh, *points, lights, n_lights, d.m, d.n, pt_ids + d.pt_off,
                                     cl_ids + d.cl_off, *params, out + 3 * o)))
            return rc;
        o += (int64_t)d.m * d.n;
    }
    return VPLMC_OK;
}

int vplmc_read_totals(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace, int64_t *out) {
    if (!ctx || !plan || !workspace || !out) return set_error(VPLMC_EINVAL, "ctx, plan, workspace and out must be non-NULL");
    const int S = plan->n_slices;
    std::vector<SliceDesc> d(S);
    std::vector<int32_t> st(4 * (size_t)S);
    unsigned long long c[4] = {0, 0, 0, 0};
    const char *ws = static_cast<const char *>(workspace);
    VPLMC_HIP(hipSetDevice(ctx->device));
    if (S > 0) {
        VPLMC_HIP(hipMemcpyAsync(d.data(), ws + plan->layout.off[R_DESC], S * sizeof(SliceDesc), hipMemcpyDeviceToHost,
                                 ctx->stream));
        VPLMC_HIP(hipMemcpyAsync(st.data(), ws + plan->layout.off[R_SLICE_STATS], st.size() * 4, hipMemcpyDeviceToHost,
                                 ctx->stream));
    }
    VPLMC_HIP(hipMemcpyAsync(c, ws + plan->layout.off[R_COUNTS], sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    VPLMC_HIP(hipStreamSynchronize(ctx->stream));
    int64_t entries = 0;
    for (int s = 0; s < S; ++s) entries += (int64_t)d[s].N1 + st[4 * s + 3];
    out[0] = entries;
    out[1] = (int64_t)c[0];
    out[2] = (int64_t)c[1];
    out[3] = (int64_t)c[2];
    return VPLMC_OK;
}

int vplmc_cluster_table(vplmc_ctx *ctx, const vplmc_lights *vpls, const vplmc_cut *cut, uint64_t seed, int32_t *rep,
                        float *lights, float *bbox) {
    if (!ctx || !vpls || !cut || !rep || !lights || !bbox) return set_error(VPLMC_EINVAL, "NULL argument");
    if (vpls->n < 1 || bad_ptrs_lights(vpls)) return set_error(VPLMC_EINVAL, "incomplete VPL arrays");
    if (cut->n_clusters < 0 || (cut->n_clusters > 0 && (!cut->offsets || !cut->members)))
        return set_error(VPLMC_EINVAL, "invalid cut");
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_cluster_table(ctx->stream, *vpls, *cut, seed, rep, lights, bbox, cut->n_clusters);
}

int vplmc_eval_pairs(vplmc_ctx *ctx, const vplmc_points *points, const vplmc_lights *lights, int64_t n_pairs,
                     const int32_t *point_ids, const int32_t *light_ids, const vplmc_params *params, float *out) {
    if (!ctx || !points || !lights || !params) return set_error(VPLMC_EINVAL, "NULL argument");
    if (n_pairs < 0) return set_error(VPLMC_EINVAL, "n_pairs must be >= 0");
    if (n_pairs > 0 && (!point_ids || !light_ids || !out)) return set_error(VPLMC_EINVAL, "NULL pair arrays");
    if (n_pairs > 0 && (points->m < 1 || lights->n < 1)) return set_error(VPLMC_EINVAL, "no points or no lights");
    if (bad_ptrs_points(points) || bad_ptrs_lights(lights)) return set_error(VPLMC_EINVAL, "incomplete arrays");
    int rc = check_params(params);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_eval_pairs(ctx->stream, ctx->bvh, *points, *lights, n_pairs, point_ids, light_ids, *params, out);
}

int vplmc_brute_force(vplmc_ctx *ctx, const vplmc_points *points, const vplmc_lights *lights, int32_t n_out,
                      const int32_t *point_ids, const vplmc_params *params, double *out) {
    if (!ctx || !points || !lights || !params) return set_error(VPLMC_EINVAL, "NULL argument");
    if (n_out < 0 || (n_out > 0 && !out)) return set_error(VPLMC_EINVAL, "invalid output");
    if (!point_ids && n_out > points->m) return set_error(VPLMC_EINVAL, "n_out exceeds the number of points");
    if (n_out > 0 && (points->m < 1 || lights->n < 1)) return set_error(VPLMC_EINVAL, "no points or no lights");
    if (bad_ptrs_points(points) || bad_ptrs_lights(lights)) return set_error(VPLMC_EINVAL, "incomplete arrays");
    int rc = check_params(params);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_brute_force(ctx->stream, ctx->bvh, *points, *lights, n_out, point_ids, *params, out);
}

int vplmc_set_proposal(vplmc_ctx *ctx, const float *params) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    ctx->mlp = params;
    return VPLMC_OK;
}

int vplmc_mlp_param_count(void) { return MLP_PARAMS; }

int vplmc_mlp_scratch_size(int64_t rows, size_t *bytes) {
    if (rows < 0 || !bytes) return set_error(VPLMC_EINVAL, "rows must be >= 0 and bytes non-NULL");
    *bytes = (size_t)rows * 4 * (2 + 4 * MLP_HID) + (size_t)MLP_PARAMS * 4 + 256;
    return VPLMC_OK;
}

static int mlp_scratch(int64_t rows, void *scratch, size_t scratch_bytes, float **y, float **dy, float **cache,
                       float **grad) {
    size_t need = 0;
    vplmc_mlp_scratch_size(rows, &need);
    if (!scratch || scratch_bytes < need)
        return set_error(VPLMC_EINVAL, "scratch of %zu bytes is smaller than the %zu required", scratch_bytes, need);
    float *p = static_cast<float *>(scratch);
    *grad = p;
    p += MLP_PARAMS;
    *y = p;
    p += rows;
    *dy = p;
    p += rows;
    *cache = p;
    return VPLMC_OK;
}

int vplmc_mlp_forward(vplmc_ctx *ctx, const float *params, int64_t rows, const float *features, float *y) {
    if (!ctx || !params || rows < 0 || (rows > 0 && (!features || !y))) return set_error(VPLMC_EINVAL, "invalid arguments");
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_mlp_forward(ctx->stream, params, rows, features, y);
}

int vplmc_mlp_grad(vplmc_ctx *ctx, const float *params, int64_t rows, const float *features, const float *dy_in,
                   void *scratch, size_t scratch_bytes, float *grad) {
    if (!ctx || !params || !grad || rows < 0 || (rows > 0 && (!features || !dy_in)))
        return set_error(VPLMC_EINVAL, "invalid arguments");
    float *y, *dy, *cache, *g;
    int rc = mlp_scratch(rows, scratch, scratch_bytes, &y, &dy, &cache, &g);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_mlp_grad(ctx->stream, params, rows, features, dy_in, grad, y, cache);
}

int vplmc_mlp_adam(vplmc_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr) {
    if (!ctx || !params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return set_error(VPLMC_EINVAL, "invalid arguments");
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_mlp_adam(ctx->stream, params, grad, m, v, step, lr);
}

int vplmc_mlp_train_step(vplmc_ctx *ctx, float *params, float *m, float *v, int32_t step, float lr, int64_t rows,
                         const float *features, const float *pstar, int32_t n_groups, const int32_t *group_offsets,
                         void *scratch, size_t scratch_bytes, float *loss) {
    if (!ctx || !params || !m || !v || step < 1 || !(lr > 0.f) || rows < 0 || n_groups < 0 || !loss ||
        (rows > 0 && (!features || !pstar || !group_offsets)))
        return set_error(VPLMC_EINVAL, "invalid arguments");
    float *y, *dy, *cache, *g;
    int rc = mlp_scratch(rows, scratch, scratch_bytes, &y, &dy, &cache, &g);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_mlp_train_step(ctx->stream, params, m, v, step, lr, rows, features, pstar, n_groups, group_offsets, y,
                                 dy, g, loss, cache);
}

int vplmc_proposal_targets(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points, const float *lights,
                           const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params, void *workspace,
                           size_t workspace_bytes, float *pstar) {
    if (!ctx || !plan || !points || !lights || !params || !pstar) return set_error(VPLMC_EINVAL, "NULL argument");
    if (plan->coarse) return set_error(VPLMC_EUNSUPPORTED, "training targets need a plan with fixed cluster columns");
    if (bad_ptrs_points(points)) return set_error(VPLMC_EINVAL, "incomplete points arrays");
    if (plan->n_slices > 0 && (!pt_ids || !cl_ids)) return set_error(VPLMC_EINVAL, "pt_ids and cl_ids must be non-NULL");
    if (!workspace || workspace_bytes < plan->layout.total)
        return set_error(VPLMC_EINVAL, "workspace smaller than vplmc_workspace_size");
    int rc = check_params(params);
    if (rc) return rc;
    VPLMC_HIP(hipSetDevice(ctx->device));
    SliceDesc *desc = region<SliceDesc>(workspace, plan, R_DESC);
    if (plan->n_slices > 0)
        VPLMC_HIP(hipMemcpyAsync(desc, plan->upload.data(), plan->upload.size(), hipMemcpyHostToDevice, ctx->stream));
    // the first-pass moment regions serve as FP64 scratch (2 x columns doubles)
    double *moments = region<double>(workspace, plan, R_COLSUM);
    return launch_targets(ctx->stream, *plan, desc, ctx->bvh, *points, lights, plan->n_clusters, pt_ids, cl_ids,
                          *params, moments, pstar);
}

int vplmc_check_inputs(vplmc_ctx *ctx, const vplmc_plan *plan, int32_t n_points, int32_t n_vpls,
                       const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids, int64_t *n_bad) {
    if (!ctx || !plan || !cut || !n_bad) return set_error(VPLMC_EINVAL, "ctx, plan, cut and n_bad must be non-NULL");
    *n_bad = 0;
    if (n_points < 0 || n_vpls < 0) return set_error(VPLMC_EINVAL, "n_points and n_vpls must be >= 0");
    if (cut->n_clusters != plan->n_clusters) return set_error(VPLMC_EINVAL, "cut does not match the plan");
    if (cut->n_clusters > 0 && (!cut->offsets || !cut->members)) return set_error(VPLMC_EINVAL, "invalid cut");
    if (plan->n_slices > 0 && (!pt_ids || (!cl_ids && !plan->coarse)))
        return set_error(VPLMC_EINVAL, "pt_ids and cl_ids must be non-NULL");
    VPLMC_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    unsigned long long *bad = nullptr;
    if (hipMalloc(&bad, 2 * sizeof(unsigned long long)) != hipSuccess)
        return set_error(VPLMC_ENOMEM, "counter allocation failed");
    unsigned long long h[2] = {0, 0};
    int32_t n_members = 0;
    int rc = VPLMC_OK;
    auto run = [&]() -> int {
        VPLMC_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(unsigned long long), st));
        int r;
        if ((r = launch_count_out_of_range(st, pt_ids, plan->sum_m, n_points, bad))) return r;
        if (!plan->coarse && (r = launch_count_out_of_range(st, cl_ids, plan->tot_col, plan->n_clusters, bad)))
            return r;
        if (cut->n_clusters > 0) {
            if ((r = launch_count_unordered(st, cut->offsets, cut->n_clusters, bad + 1))) return r;
            VPLMC_HIP(hipMemcpyAsync(&n_members, cut->offsets + cut->n_clusters, 4, hipMemcpyDeviceToHost, st));
        }
        VPLMC_HIP(hipMemcpyAsync(h, bad, sizeof(h), hipMemcpyDeviceToHost, st));
        VPLMC_HIP(hipStreamSynchronize(st));
        // members are read only when the offsets are ordered (their count is then offsets[n_clusters])
        if (h[1] == 0 && n_members > 0) {
            if ((r = launch_count_out_of_range(st, cut->members, n_members, n_vpls, bad))) return r;
            VPLMC_HIP(hipMemcpyAsync(h, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            VPLMC_HIP(hipStreamSynchronize(st));
        }
        return VPLMC_OK;
    };
    rc = run();
    (void)hipFree(bad);
    if (rc) return rc;
    *n_bad = (int64_t)(h[0] + h[1]);
    return VPLMC_OK;
}

int vplmc_philox4x64(vplmc_ctx *ctx, uint64_t key0, uint64_t key1, const uint64_t *ctr, int64_t n, uint64_t *out) {
    if (!ctx) return set_error(VPLMC_EINVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && (!ctr || !out))) return set_error(VPLMC_EINVAL, "invalid counter/output arrays");
    VPLMC_HIP(hipSetDevice(ctx->device));
    return launch_philox(ctx->stream, key0, key1, ctr, n, out);
}

// ---- global light cut ------------------------------------------------------

}  // extern "C"

struct vplmc_lightcut_plan {
    int32_t n = 0, S = 0, cap = 0, F = 0, height_max = 0, depth = 0;
    std::vector<int32_t> upload;      // perm | left | right | order | min_leaf
    std::vector<int32_t> level_off;   // height_max + 1
    enum { L_TREE, L_REP, L_LIGHTS, L_BBOX, L_SAMP, L_EST, L_INV, L_PART, L_STATE, L_FRONT, L_RHO, L_SPLIT, L_CTL,
           L_LEAF, L_REN, L_BLK, L_END };
    size_t off[L_END + 1] = {};
};

namespace {

LightcutView lightcut_view(const vplmc_lightcut_plan *p, void *ws, const int32_t *sample_ids) {
    char *b = static_cast<char *>(ws);
    const size_t n = p->n;
    LightcutView v;
    v.n = p->n;
    v.S = p->S;
    v.cap = p->cap;
    v.F = p->F;
    const int32_t *t = reinterpret_cast<const int32_t *>(b + p->off[vplmc_lightcut_plan::L_TREE]);
    v.perm = t;
    v.left = t + n;
    v.right = t + n + (n - 1);
    v.order = t + n + 2 * (n - 1);
    v.min_leaf = t + n + 3 * (n - 1);
    v.sample_ids = sample_ids;
    v.rep = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_REP]);
    v.lights = reinterpret_cast<float *>(b + p->off[vplmc_lightcut_plan::L_LIGHTS]);
    v.bbox = reinterpret_cast<float *>(b + p->off[vplmc_lightcut_plan::L_BBOX]);
    v.samp = reinterpret_cast<float *>(b + p->off[vplmc_lightcut_plan::L_SAMP]);
    v.est = reinterpret_cast<double *>(b + p->off[vplmc_lightcut_plan::L_EST]);
    v.inv_est = reinterpret_cast<float *>(b + p->off[vplmc_lightcut_plan::L_INV]);
    v.part = reinterpret_cast<double *>(b + p->off[vplmc_lightcut_plan::L_PART]);
    v.state = reinterpret_cast<uint32_t *>(b + p->off[vplmc_lightcut_plan::L_STATE]);
    v.front = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_FRONT]);
    v.rho_f = reinterpret_cast<uint32_t *>(b + p->off[vplmc_lightcut_plan::L_RHO]);
    v.split = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_SPLIT]);
    v.ctl = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_CTL]);
    v.leafmark = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_LEAF]);
    v.ren = reinterpret_cast<int32_t *>(b + p->off[vplmc_lightcut_plan::L_REN]);
    v.blk = reinterpret_cast<uint32_t *>(b + p->off[vplmc_lightcut_plan::L_BLK]);
    return v;
}

}  // namespace

extern "C" {

int vplmc_lightcut_plan_create(const vplmc_light_tree *tree, int32_t n_samples, int32_t max_cut,
                               vplmc_lightcut_plan **out) {
    if (!out) return set_error(VPLMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tree) return set_error(VPLMC_EINVAL, "tree is NULL");
    const int64_t n = tree->n_leaves;
    if (n < 1 || n > VPLMC_MAX_TREE_LEAVES)
        return set_error(VPLMC_EINVAL, "n_leaves %lld outside [1, %d]", (long long)n, VPLMC_MAX_TREE_LEAVES);
    if (!tree->perm || (n > 1 && (!tree->left || !tree->right))) return set_error(VPLMC_EINVAL, "tree arrays must be non-NULL");
    if (n_samples < 0) return set_error(VPLMC_EINVAL, "n_samples must be >= 0");
    if (max_cut < 1) return set_error(VPLMC_EINVAL, "max_cut must be >= 1");
    const int64_t N = 2 * n - 1;
    std::vector<int32_t> seen(n, 0);
    for (int64_t x = 0; x < n; ++x) {
        const int32_t j = tree->perm[x];
        if (j < 0 || j >= n || seen[j]) return set_error(VPLMC_EINVAL, "perm is not a permutation of 0 .. %lld", (long long)(n - 1));
        seen[j] = 1;
    }
    std::vector<int32_t> parent(N, -1), height(N, 0), min_leaf(N), max_leaf(N), depth(N, 0);
    for (int64_t x = 0; x < N; ++x) min_leaf[x] = max_leaf[x] = (int32_t)x;
    for (int64_t k = 0; k + 1 < n; ++k) {
        const int64_t f = n + k;
        const int32_t l = tree->left[k], r = tree->right[k];
        if (l < 0 || r < 0 || l >= f || r >= f || l == r)
            return set_error(VPLMC_EINVAL, "tree: split node %lld has children %d, %d (must be distinct and earlier)", (long long)f, l, r);
        if (parent[l] >= 0 || parent[r] >= 0) return set_error(VPLMC_EINVAL, "tree: node %d or %d already has a parent", l, r);
        if (max_leaf[l] + 1 != min_leaf[r])
            return set_error(VPLMC_EINVAL, "tree: the leaves of node %lld are not contiguous (left before right)", (long long)f);
        parent[l] = parent[r] = (int32_t)f;
        height[f] = 1 + std::max(height[l], height[r]);
        min_leaf[f] = min_leaf[l];
        max_leaf[f] = max_leaf[r];
    }
    auto plan = new (std::nothrow) vplmc_lightcut_plan;
    if (!plan) return set_error(VPLMC_ENOMEM, "host allocation failed");
    plan->n = (int32_t)n;
    plan->S = n_samples;
    plan->cap = max_cut;
    plan->F = (int32_t)(2 * std::min<int64_t>(max_cut, n));
    plan->height_max = n > 1 ? height[N - 1] : 0;
    int32_t dmax = 0;
    for (int64_t f = N - 1; f >= n; --f) {
        const int64_t k = f - n;
        depth[tree->left[k]] = depth[tree->right[k]] = depth[f] + 1;
        dmax = std::max(dmax, depth[f] + 1);
    }
    plan->depth = dmax;
    const int H = plan->height_max;
    plan->level_off.assign(H + 1, 0);
    for (int64_t k = 0; k + 1 < n; ++k) plan->level_off[height[n + k]]++;
    for (int h = 1; h <= H; ++h) plan->level_off[h] += plan->level_off[h - 1];
    std::vector<int32_t> order(n - 1), fill(plan->level_off.begin(), plan->level_off.end());
    for (int64_t k = 0; k + 1 < n; ++k) order[fill[height[n + k] - 1]++] = (int32_t)(n + k);
    plan->upload.reserve(n + 3 * (n - 1) + N);
    plan->upload.insert(plan->upload.end(), tree->perm, tree->perm + n);
    if (n > 1) {
        plan->upload.insert(plan->upload.end(), tree->left, tree->left + (n - 1));
        plan->upload.insert(plan->upload.end(), tree->right, tree->right + (n - 1));
    }
    plan->upload.insert(plan->upload.end(), order.begin(), order.end());
    plan->upload.insert(plan->upload.end(), min_leaf.begin(), min_leaf.end());
    const size_t S = n_samples, F = plan->F, cap = max_cut;
    const size_t chunks = (std::min<size_t>(cap, n) + LC_UPDATE_CHUNK - 1) / LC_UPDATE_CHUNK;
    const size_t bytes[vplmc_lightcut_plan::L_END] = {
        plan->upload.size() * 4, (size_t)N * 4, (size_t)N * 36, (size_t)N * 24, S * 36, S * 8, S * 4,
        chunks * S * 8, (size_t)N * 4, 2 * F * 4, 2 * F * 4, cap * 4, 8 * 4, (size_t)n * 4, (size_t)N * 4,
        2 * (size_t)((n + LC_ORDER_BLOCK - 1) / LC_ORDER_BLOCK) * 4};
    size_t o = 0;
    for (int r = 0; r < vplmc_lightcut_plan::L_END; ++r) {
        plan->off[r] = o;
        o += align256(bytes[r]);
    }
    plan->off[vplmc_lightcut_plan::L_END] = o;
    *out = plan;
    return VPLMC_OK;
}

int vplmc_lightcut_plan_destroy(vplmc_lightcut_plan *plan) {
    delete plan;
    return VPLMC_OK;
}

int vplmc_lightcut_workspace_size(const vplmc_lightcut_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(VPLMC_EINVAL, "plan and bytes must be non-NULL");
    *bytes = plan->off[vplmc_lightcut_plan::L_END];
    return VPLMC_OK;
}

int vplmc_lightcut(vplmc_ctx *ctx, const vplmc_lightcut_plan *plan, const vplmc_points *points,
                   const vplmc_lights *vpls, const int32_t *sample_ids, double eps, float r_min, uint64_t seed,
                   void *workspace, size_t workspace_bytes, int32_t *n_cut, int32_t *cut_nodes, int32_t *cut_offsets,
                   int32_t *above_left, int32_t *above_right, float *rho) {
    if (!ctx || !plan || !points || !vpls) return set_error(VPLMC_EINVAL, "NULL argument");
    if (vpls->n != plan->n) return set_error(VPLMC_EINVAL, "vpls->n = %d, the tree has %d leaves", vpls->n, plan->n);
    if (bad_ptrs_lights(vpls)) return set_error(VPLMC_EINVAL, "incomplete VPL arrays");
    if (plan->S > 0 && (points->m < 1 || bad_ptrs_points(points) || !sample_ids))
        return set_error(VPLMC_EINVAL, "samples need points and sample_ids");
    if (!(eps >= 0.0)) return set_error(VPLMC_EINVAL, "eps must be >= 0");
    if (!(r_min > 0.0f) || !std::isfinite(r_min)) return set_error(VPLMC_EINVAL, "r_min must be finite and > 0");
    if (!n_cut || !cut_nodes || !cut_offsets) return set_error(VPLMC_EINVAL, "n_cut, cut_nodes and cut_offsets must be non-NULL");
    const size_t need = plan->off[vplmc_lightcut_plan::L_END];
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return set_error(VPLMC_EINVAL, "workspace must be 256-byte aligned and hold %zu bytes", need);
    VPLMC_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    VPLMC_HIP(hipMemcpyAsync(static_cast<char *>(workspace) + plan->off[vplmc_lightcut_plan::L_TREE],
                             plan->upload.data(), plan->upload.size() * 4, hipMemcpyHostToDevice, st));
    const LightcutView v = lightcut_view(plan, workspace, sample_ids);
    return launch_lightcut(st, v, plan->level_off.data(), plan->height_max, plan->depth, *points, *vpls, eps, r_min,
                           seed, n_cut, cut_nodes, cut_offsets, above_left, above_right, rho);
}

}  // extern "C"
