// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "vplmc.h"

namespace vplmc {

// ---------------------------------------------------------------- errors
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);

#define VPLMC_HIP(call)                                      \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::vplmc::hip_error(e_, #call); \
    } while (0)

// ------------------------------------------------------- random numbers
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round maps
// (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)); the key is bumped by (W0, W1) between rounds.
constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

// Counter tags: the third counter word separates the method's streams.
constexpr uint64_t TAG_PASS1 = 1;
constexpr uint64_t TAG_PASS2 = 2;
constexpr uint64_t TAG_INITX = 3;
constexpr uint64_t TAG_INITY = 4;
constexpr uint64_t TAG_REP = 5;
constexpr uint64_t TAG_TREE = 6;   // kept child of a split node (light coarsening)
constexpr uint64_t TAG_ZETA = 7;   // row draws of the light coarsening

struct U64x4 {
    uint64_t a, b, c, d;
};

__device__ __forceinline__ U64x4 philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t c3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t lo0 = PHILOX_M0 * c0, hi0 = __umul64hi(PHILOX_M0, c0);
        const uint64_t lo1 = PHILOX_M1 * c2, hi1 = __umul64hi(PHILOX_M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return U64x4{c0, c1, c2, c3};
}

// An index read from a caller's array, clamped into [0, n): out-of-range ids
// never reach memory (vplmc_check_inputs reports them).
__device__ __forceinline__ int clamp_index(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// floor(r * n / 2^64): a uniform 64-bit word mapped onto [0, n).
__device__ __forceinline__ uint64_t mulhi64(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// ------------------------------------------------------------ geometry
struct BvhNode {            // 32 bytes, depth-first order: an inner node's left child follows it
    float lo[3];
    int32_t leaf;           // leaf: first sphere << 4 | sphere count (1..15); inner: 0
    float hi[3];
    int32_t skip;           // the node after this node's subtree (n_nodes past the last)
};
constexpr int32_t BVH_MAX_SPHERES = 1 << 27;

struct Bvh {
    const BvhNode *nodes = nullptr;
    // kind 0: spheres (cx, cy, cz, r) in node order, one float4 each; kind 1:
    // triangle references in node order, three float4 each (v0, v1 - v0, v2 - v0)
    const float4 *spheres = nullptr;
    int32_t n_nodes = 0;
    int32_t n_spheres = 0;             // float4 records after the nodes
    int32_t kind = 0;
};
constexpr int32_t BVH_MAX_TRIANGLES = 1 << 24;

// host build: spheres -> nodes + reordered spheres
void build_bvh(int32_t n, const float *cx, const float *cy, const float *cz, const float *r,
               std::vector<BvhNode> &nodes, std::vector<float> &sph4, std::vector<int32_t> *order = nullptr);
// host build: triangles (9 floats each) -> SBVH nodes, the triangle of every
// leaf reference, and the references as 12 floats each (kernels' layout)
void build_sbvh(int32_t n, const float *v, std::vector<BvhNode> &nodes, std::vector<int32_t> &refs,
                std::vector<float> &prim4);

// --------------------------------------------------------- frame layout
// Device copy of one slice's layout (offsets in elements).  With light
// coarsening the host plan holds capacities (n, N1, N2 at most these) and
// the frame's coarsening kernels write the slice's own n, N1 and N2 here
// before anything reads them; every region is laid out for the capacities.
struct SliceDesc {
    int32_t m, n, q, N1;
    int32_t N2, pt_off, cl_off, words_row;     // words_row = ceil(n / 32) (of the capacity)
    int32_t words_col, off_grp, ell, nmax;     // words_col = ceil(m / 32); ell: completed from the ELL copy;
                                               // nmax: column cap of the coarsening
    int64_t off1, off2, off_omega, off_col;
    int64_t off_row, off_colptr, off_x, off_y;
    int64_t off_bm, off_bmt;                   // bitmap word offsets (row- and column-major)
    int64_t off_ell, off_red;                  // ELL entry offset; cross-wave reduction scratch (floats)
    int64_t off_part;                          // first part slot of the slice
    int32_t qr, pad1;                          // qr: the slice's rank; q: the kernels' rank (4, 8, 16 or 32
                                               // >= qr), the row length of X and Y (components past qr are 0)
};

// Column-major ELL copy of a slice's samples for the LDS-resident completion.
// Column j with c_j samples is cut into p_j = max(1, ceil(c_j / ELL_LMAX))
// parts of ceil(c_j / p_j) consecutive samples (CSC order; the last part may
// be shorter).  The parts, sorted by length (descending), are cut into groups
// of 64; sample k of the part at sorted position 64 g + l is entry
// grp[g] + 64 k + l, so that one load instruction of a wavefront whose lane l
// walks that part reads 64 consecutive entries and every lane of a group has
// nearly the same number of samples.  Entries past a part's length are
// padding and never read.  Parts are numbered in column order by
// pbase[j] + t.
struct EllView {
    int2 *part;        // per (slice, sorted position): {j | len << 16 | (column of several parts) << 23,
                       //  part number in column order}
    int32_t *ppos;     // per (slice, part in column order): sorted position
    int32_t *pbase;    // per (slice, column + 1): first part of the column (like col_ptr)
    int32_t *grp;      // per slice: groups + 1 offsets, relative to off_ell
    uint16_t *row;     // per entry: row of the sample (rows < ELL_MAX_M)
    float *val;        // 3 per entry: sampled values
    float *res;        // 3 per entry: residual of the current iterate
    float *partial;    // 48 per part slot: X+^T R of the part (columns cut into several parts)
    int32_t *split;    // per (slice, column): the columns of more than one part, first nsplit entries
    int32_t *nsplit;   // per slice
};
constexpr int ELL_LMAX = 64;      // longest part
// uniform mass of the proposal's training target, in units of the slice's mean
// column standard deviation: p*_j ~ sigma_j + PROPOSAL_TARGET_MIX mean(sigma)
constexpr double PROPOSAL_TARGET_MIX = 3.0;
constexpr int ELL_MAX_M = 8192;   // rows of a slice that may use the ELL copy
constexpr int ADM_RED_FLOATS = 16 * 2 * 256;   // per slice: 16 wavefronts x two 16 x 16 partial Grams

// extra (internal) regions, after the public ones
enum {
    R_DESC = VPLMC_R_COUNT,
    R_COLW_PREFIX,   // uint64 per (slice, column): inclusive prefix of the weights
    R_BITMAP,        // uint32 words, row-major per slice
    R_BITMAPT,       // uint32 words, column-major per slice
    R_WPRE,          // uint16 per row-major word: popcount prefix within the row
    R_WPRET,         // uint16 per column-major word
    R_XNEXT,         // float[m][q]: second X buffer
    R_XP,            // float[m][q]
    R_LAMBDA,        // float[m][q]
    R_YP,            // float[n][3][q]
    R_PI,            // float[n][3][q]
    R_SLICE_STATS,   // int32 iters, int32 flags, float resid, int32 n2 per slice
    R_COLSUM,        // double per (slice, column): sum of t over the first pass
    R_COLSUMSQ,      // double per (slice, column): sum of t^2
    R_COLZERO,       // int32 per (slice, column): observations with t = 0
    R_SLICE_GEO,     // float[8] per slice: centroid xyz, bbox diagonal, mean normal xyz, -
    R_ELL_PART,      // int2 per part slot
    R_ELL_PPOS,      // int32 per part slot
    R_ELL_PBASE,     // int32 per (slice, column + 1)
    R_ELL_PARTIAL,   // float[48] per part slot
    R_ELL_GRP,       // int32 per group slot
    R_ELL_SPLIT,     // int32 per (slice, column)
    R_ELL_NSPLIT,    // int32 per slice
    R_ELL_ROW,       // uint16 per ELL entry
    R_ELL_VAL,       // float[3] per ELL entry
    R_ELL_RES,       // float[3] per ELL entry
    R_YT,            // float[n][3][q]: staging of the right-hand sides of the Y update
    R_ADM_RED,       // float per slice: ADM_RED_FLOATS
    R_E2PART,        // double per part slot: squared residual over the part's samples
    R_QUEUE,         // int32[8]: work-queue counters of the completion launches
    R_TREE,          // int32: the coarsening tree (uploaded with the plan)
    R_NODE_KD,       // int32 per split node: kept child, then dropped child
    R_LEAF_KPRE,     // int64 per leaf + 1: prefix of the draw counts
    R_NODE_COST,     // float per (slice, split node)
    R_NODE_EFF,      // float per (slice, split node)
    R_NODE_MERGED,   // uint8 per (slice, split node)
    R_NODE_TOP,      // int32 per (slice, node)
    R_LEAF_COL,      // int32 per (slice, leaf)
    R_ZETA,          // uint16 per (slice, draw slot)
    R_COUNTS,        // uint64[4]: shadow rays of the entries, coarsening evaluations and rays, -
    R_GSYS,          // GADM_SYS_BYTES per slice: q x q systems and state of the global-memory completion
    R_GE2,           // double per row block of the global-memory slices: squared residual sums
    R_INTERNAL_END
};

// Light tree above the global cut, as uploaded by the plan: leaves 0 .. n_g - 1,
// split node n_g + k with children left[k], right[k] (children first); the
// root is node 2 n_g - 2.
struct CoarsenTree {
    int32_t n_leaves = 0, height_max = 0;
    const int32_t *left = nullptr, *right = nullptr;      // per split node
    const int32_t *parent = nullptr;                      // per node (-1 at the root)
    const int32_t *height = nullptr, *min_leaf = nullptr; // per node (leaves: 0, itself)
    const int32_t *order = nullptr;                       // split nodes by (height, id)
    const int32_t *level_off = nullptr;                   // height_max + 1: order[level_off[h-1] .. level_off[h]) have height h
};

// Per-frame and per-slice state of the coarsening.
struct CoarsenSlices {
    float *eps = nullptr, *cost = nullptr, *eff = nullptr;   // per (slice, split node)
    uint8_t *merged = nullptr;                               // per (slice, split node)
    int32_t *top = nullptr;                                  // per (slice, node): column node above it
    int32_t *leaf_col = nullptr;                             // per (slice, leaf): its column
    const int32_t *kept = nullptr, *dropped = nullptr;       // per split node
    const int64_t *kpre = nullptr;                           // n_leaves + 1: prefix of the draw counts
    uint16_t *zeta = nullptr;                                // per (slice, draw slot): row of the draw
};

// Regions of the workspace: byte offsets.
struct Layout {
    size_t off[R_INTERNAL_END];
    size_t bytes[R_INTERNAL_END];
    size_t total;
};

}  // namespace vplmc

// Streams forked from the caller's stream for the completion's rank groups,
// which touch disjoint slices and so may run side by side (default priority;
// joined back by events, which stream capture records as graph edges).
struct AdmStreams {
    hipStream_t side[3] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[3] = {};
};

struct vplmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    AdmStreams adm;
    vplmc::Bvh bvh;
    void *bvh_mem = nullptr;   // owned device allocation holding nodes + spheres
    int n_cu = 256;
    const float *mlp = nullptr;   // learned-proposal parameters (device), or none
    // phase timing: events[frame][phase boundary]
    std::vector<hipEvent_t> prof_events;
    int prof_max_frames = 0;
    int prof_frames = 0;
    bool prof_on = false;
    bool capturing = false;                     // a frame is being recorded into a graph
    void *scratch = nullptr;                    // device address of the static workspace on this device
};

struct vplmc_plan {
    int32_t n_slices = 0;
    int32_t n_clusters = 0;
    int32_t n_lights = 0;          // lights of the table: n_clusters, or 2 n_leaves - 1 tree nodes
    // light coarsening (Sec. 4): on when the plan was made with a tree
    bool coarse = false;
    bool als = false;              // completion by per-row masked ALS (VPLMC_ALS)
    int32_t n_leaves = 0, height_max = 0, pixels = 0;
    double bound = 0.0;
    std::vector<int32_t> tree;     // left, right, parent, height, min_leaf, order, level_off
    int32_t pass1_ppm = 0, pass2_ppm = 0;
    int64_t sum_m = 0, max_m = 0;
    std::vector<vplmc::SliceDesc> desc;
    // slice ids by ADM kernel group: 2 * bucket + variant, bucket = rank 4, 8, 16, 32,
    // variant 0 = X resident in LDS, 1 = X in global memory
    std::vector<int32_t> groups[8];
    int32_t group_max_m[8] = {};
    vplmc::Layout layout;
    int64_t tot1 = 0, tot2 = 0, tot_omega = 0, tot_col = 0, tot_row = 0, tot_x = 0, tot_y = 0;
    int64_t tot_bm = 0, tot_bmt = 0;
    int64_t tot_grp = 0, tot_ell = 0, n_ell = 0;   // ELL group table entries, ELL entries, ELL slices
    int64_t tot_part = 0;                           // part slots
    vplmc_tune tune = {0, 1024, 256, 0};             // launch shapes
    std::vector<int32_t> ids;                  // slice ids grouped by rank bucket
    // global-memory completion: per group (odd g) the prefix over its slices of
    // the row blocks and of the column blocks (count + 1 each), at gblk_off[g]
    // ints into gblk; the first row block's squared-residual slot at ge2_base[g]
    std::vector<int32_t> gblk;
    int64_t gblk_off[8] = {}, ge2_base[8] = {}, g_rows[8] = {}, g_cols[8] = {};
    std::vector<char> upload;                  // descriptor table + ids + gblk, as copied to the workspace
};

namespace vplmc {
// global-memory completion: rows per row block, columns per column block,
// bytes of a slice's system state (F and Inv in FP64, their FP32 copies, flags)
constexpr int GADM_RB = 64;
constexpr int GADM_CB = 256;
constexpr size_t GADM_SYS_BYTES = 2 * 32 * 32 * 8 + 2 * 32 * 32 * 4 + 256;
// LDS budget of the LDS-resident ADM kernel (gfx950: 160 KiB per workgroup)
constexpr size_t LDS_BYTES = 160 * 1024;
constexpr int adm_lds_threads(int q) { return q == 32 ? 0 : 1024; }
constexpr size_t adm_lds_static_bytes(int q) {
    return (size_t)(4 * q * q * 8 + 2 * q * q * 4 + 32 * 8) + 2 * 256 * 4 + 1024;
}
// two LDS buffers of m (q + 1) words (X_k and R Y^T / X+)
constexpr size_t adm_lds_dynamic_bytes(int q, int m) { return (size_t)2 * m * (q + 1) * 4; }
inline bool adm_fits_lds(int q, int m) {
    return q <= 16 && m <= ELL_MAX_M && (int64_t)m * q <= 18 * 1024 &&
           adm_lds_static_bytes(q) + adm_lds_dynamic_bytes(q, m) <= LDS_BYTES;
}

// kernel launchers (kernels_*.hip)
int launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v);
int launch_cluster_table(hipStream_t st, const vplmc_lights &v, const vplmc_cut &cut, uint64_t seed,
                         int32_t *rep, float *lights, float *bbox, int32_t stride);
// light coarsening (kernels_coarsen.hip, kernels_eval.hip)
int launch_node_table(hipStream_t st, const CoarsenTree &tr, const int32_t *cut_offsets, uint64_t seed, int32_t *rep,
                      float *lights, float *bbox, int32_t *members, int32_t *kept, int32_t *dropped);
int launch_leaf_draws(hipStream_t st, int32_t ng, const float *lights, int64_t K, int32_t *quota, int64_t *kpre);
int launch_coarsen_eps(hipStream_t st, const vplmc_plan &plan, const Bvh &bvh, const vplmc_points &pts,
                       const float *lights, const SliceDesc *desc, const int32_t *pt_ids, const CoarsenTree &tr,
                       const CoarsenSlices &cs, const vplmc_params &prm, int n_cu, unsigned long long *counts);
int launch_coarsen_merge(hipStream_t st, const vplmc_plan &plan, SliceDesc *desc, const CoarsenTree &tr,
                         const CoarsenSlices &cs, int32_t *columns);
int launch_coarsen_pass1(hipStream_t st, const vplmc_plan &plan, SliceDesc *desc, const CoarsenSlices &cs,
                         uint32_t *bm, uint32_t *bmt, int32_t *row_ptr, uint32_t *omega1);
int launch_count_out_of_range(hipStream_t st, const int32_t *ids, int64_t n, int32_t hi, unsigned long long *bad);
int launch_count_unordered(hipStream_t st, const int32_t *offsets, int64_t n, unsigned long long *bad);
int launch_philox(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t *ctr, int64_t n,
                  uint64_t *out);
int launch_pass1(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, uint64_t seed,
                 uint32_t *omega1, uint32_t *bm, uint32_t *bmt);
int launch_eval_omega(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const float *lights,
                      int32_t n_lights, const SliceDesc *desc, int32_t n_slices, const int32_t *pt_ids,
                      const int32_t *cl_ids, const uint32_t *keys, int64_t n_keys, int which_pass,
                      const int32_t *stats, const vplmc_params &prm, float *vals, int threads, int n_cu,
                      unsigned long long *rays);
int launch_colstats(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *omega1,
                    const float *val1, const uint32_t *bmt, uint16_t *wpret, int32_t *col_ptr, int32_t *csc_row,
                    float *csc_val, int32_t *cnt, float *mn, float *mx, double *sum, double *sumsq, int32_t *zeros);
int launch_weights(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *cnt,
                   const float *mn, const float *mx, const float *logits, float mix, uint32_t *w, uint64_t *prefix,
                   int32_t *stats);
// learned proposal (kernels_mlp.hip)
constexpr int MLP_IN = 12, MLP_HID = 128;
constexpr int MLP_PARAMS = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_HID + 1;
int launch_features(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const vplmc_points &pts,
                    const int32_t *pt_ids, const int32_t *cl_ids, const float *lights, const float *bbox,
                    const vplmc_cut &cut, const int32_t *node_members, const int32_t *cnt, const float *mn,
                    const float *mx, const double *sum, const double *sumsq, const int32_t *zeros, float *slice_geo,
                    float *features);
int launch_mlp_forward(hipStream_t st, const float *params, int64_t rows, const float *features, float *y);
int launch_mlp_train_step(hipStream_t st, float *params, float *m, float *v, int32_t step, float lr, int64_t rows,
                          const float *features, const float *pstar, int32_t n_groups, const int32_t *group_off,
                          float *y, float *dy, float *grad, float *loss, float *cache);
int launch_mlp_grad(hipStream_t st, const float *params, int64_t rows, const float *features, const float *dy,
                    float *grad, float *y, float *cache);
int launch_mlp_adam(hipStream_t st, float *params, const float *grad, float *m, float *v, int32_t step, float lr);
int launch_targets(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const Bvh &bvh,
                   const vplmc_points &pts, const float *lights, int32_t n_lights, const int32_t *pt_ids,
                   const int32_t *cl_ids, const vplmc_params &prm, double *moments, float *pstar);
int launch_pass2(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, uint64_t seed,
                 const uint64_t *prefix, uint32_t *bm, uint32_t *bmt, uint32_t *omega2, int32_t *stats);
int launch_sort(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *bm,
                const uint32_t *bmt, uint16_t *wpre, uint16_t *wpret, int32_t *row_ptr, int32_t *col_ptr,
                const uint32_t *omega1, const float *val1, const uint32_t *omega2, const float *val2,
                const int32_t *stats, int32_t *csr_col, float *csr_val, int32_t *csc_row, float *csc_val,
                const EllView &ell);
int launch_adm(hipStream_t st, const AdmStreams *ss, const vplmc_plan &plan, int n_cu, const SliceDesc *desc,
               const int32_t *ids_dev, const int32_t *gblk_dev, char *gsys, double *ge2,
               int32_t *queues, const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col,
               const float *csr_val, const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val,
               const EllView &ell, float *X, float *Xn, float *Xp, float *Lam, float *Y, float *Yp, float *Pi,
               float *Yt, float *red, double *e2part, float *scale, int32_t *stats);
// the global-memory completion of plan group grp (rank q = 4, 8, 16 or 32; kernels_gadm.hip)
int launch_gadm_group(hipStream_t st, int q, const vplmc_plan &plan, int grp, const int32_t *ids,
                      const int32_t *gblk_dev, char *gsys, double *ge2, const SliceDesc *desc,
                      const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
                      const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Xn,
                      float *Xp, float *Lam, float *Y, float *Yp, float *Pi, float *scale, int32_t *stats);
int launch_als(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *ids_dev,
               const vplmc_params &prm, const int32_t *row_ptr, const int32_t *csr_col, const float *csr_val,
               const int32_t *col_ptr, const int32_t *csc_row, const float *csc_val, float *X, float *Y, float *scale,
               int32_t *stats);
int launch_reduce(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const int32_t *pt_ids,
                  const float *X, const float *Y, const float *scale, int32_t n_points, float *radiance);
int launch_keys_bitmap(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *keys,
                       uint32_t *bm, uint32_t *bmt, unsigned long long *bad);
int launch_prefix_given(hipStream_t st, const vplmc_plan &plan, const SliceDesc *desc, const uint32_t *w,
                        uint64_t *prefix);
int launch_full_matrix(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const float *lights,
                       int32_t n_lights, int32_t m, int32_t n, const int32_t *pt_ids, const int32_t *cl_ids,
                       const vplmc_params &prm, float *out);
int launch_eval_pairs(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const vplmc_lights &l,
                      int64_t n, const int32_t *pid, const int32_t *lid, const vplmc_params &prm, float *out);
int launch_brute_force(hipStream_t st, const Bvh &bvh, const vplmc_points &pts, const vplmc_lights &l,
                       int32_t n_out, const int32_t *pid, const vplmc_params &prm, double *out);
}  // namespace vplmc
