/*
 * vplmc -- sparse sampling and completion of VPL lighting matrices on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Huo, Wang, Liu, Bao, "Sparse Sampling and Completion for Light
 * Transport in VPL-based Rendering", arXiv 2202.12567.
 *
 * The lighting matrix A has one row per surface point (pixel) and one
 * column per light; the image is the sum of its columns (Sec. 3).  The
 * rows are partitioned into slices and the columns of each slice are the
 * nodes of a light cut (Sec. 3, steps 1-3).  For every slice the library
 * samples entries in two passes (Sec. 5), evaluates them with shadow rays,
 * completes the slice matrix by non-negative ADM factorisation M = X Y
 * (Appendix A) and renders I(s) = X (Y e) (Sec. 3, step 5).
 *
 * Conventions for every call:
 *  - Return 0 on success or a negative VPLMC_E* code; no exception crosses
 *    this boundary and nothing aborts.  The message of the last failure on
 *    the calling thread is returned by vplmc_last_error().
 *  - Pointers are DEVICE pointers on the context's device unless a comment
 *    says HOST.  Arrays are contiguous structure-of-arrays, float32 / int32.
 *  - The caller owns every buffer it passes (inputs, outputs, workspace).
 *    The library owns only what its create calls return (context, plan)
 *    and the occluder BVH it uploads in vplmc_set_occluders or
 *    vplmc_set_triangles.
 *  - All device work is ordered on the context's stream: the completion's
 *    rank groups run on three streams of the context forked from it and
 *    joined back into it by events, so work enqueued on the stream after a
 *    call sees all of that call's results.  Only calls that fill HOST
 *    outputs synchronise that stream.
 *  - Arguments are validated on the host before anything is launched.
 */
#ifndef VPLMC_H
#define VPLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 110: vplmc_params.pass2_mix (was a reserved zero field, so 0 keeps the
 * old behaviour), triangle occluders and the host BVH builders. */
#define VPLMC_VERSION 110

#define VPLMC_OK 0
#define VPLMC_EINVAL (-1)       /* invalid argument or shape                  */
#define VPLMC_ENOMEM (-2)       /* host or device allocation failed           */
#define VPLMC_EHIP (-3)         /* a HIP runtime call failed                  */
#define VPLMC_EUNSUPPORTED (-4) /* valid request this build cannot serve      */

/* Limits of one slice (packed entry index (i << 16) | j, Appendix A ranks). */
#define VPLMC_MAX_ROWS 65535
#define VPLMC_MAX_COLS 65535
#define VPLMC_MAX_RANK 32
#define VPLMC_MAX_LEAVES 32768  /* leaves of a coarsening tree (node ids and heights fit in 16 bits) */
#define VPLMC_MAX_TREE_LEAVES (1 << 27) /* VPLs under the light tree of vplmc_lightcut */

/* vplmc_params.flags */
#define VPLMC_FIXED_ITERS 1     /* ignore tol: run exactly max_iter ADM iterations */
#define VPLMC_LEARNED 2         /* second pass by the learned proposal (vplmc_set_proposal) */
#define VPLMC_FEATURES 4        /* compute the proposal features even with the plain proposal */
#define VPLMC_GIVEN_INIT 8      /* ADM starts from the X and Y regions' contents (components past q
                                   are taken as 0) instead of the seeded draw X0, Y0 (Appendix A) */
#define VPLMC_NO_NONNEG 16      /* ADM without its non-negativity: U = X+ + L / alpha, V = Y+ + P / beta
                                   (no projection; the multipliers then stay 0) */
#define VPLMC_ALS 32            /* complete by per-row masked ALS instead of ADM (a plan property:
                                   the plan must be made with the same flag) */

/* per-slice result flags (vplmc_read_stats) -- outcomes, not errors */
#define VPLMC_SLICE_ALL_ZERO 1      /* every sampled entry is 0: radiance 0      */
#define VPLMC_SLICE_NOT_CONVERGED 2 /* ADM stopped at max_iter above tol         */
#define VPLMC_SLICE_SHORTFALL 4     /* second pass hit its attempt cap           */
#define VPLMC_SLICE_FALLBACK 8      /* learned proposal gave a non-finite logit: plain weights used */

/* Surface points: rows of the lighting matrix (Sec. 3).  Position, unit
 * normal, diffuse albedo; ks / phong_e (normalised Phong specular albedo and
 * exponent) may both be NULL for Lambertian points; vx/vy/vz (unit direction
 * to the viewer) may all be NULL for +z. */
typedef struct {
    int32_t m;
    const float *px, *py, *pz;
    const float *nx, *ny, *nz;
    const float *kd_r, *kd_g, *kd_b;
    const float *ks, *phong_e;
    const float *vx, *vy, *vz;
} vplmc_points;

/* Point lights: VPLs, or the representatives of light-cut clusters.
 * Position, unit emission normal, RGB intensity. */
typedef struct {
    int32_t n;
    const float *x, *y, *z;
    const float *nx, *ny, *nz;
    const float *ir, *ig, *ib;
} vplmc_lights;

/* Light cut: cluster c holds VPLs members[offsets[c] .. offsets[c+1]). */
typedef struct {
    int32_t n_clusters;
    const int32_t *offsets; /* n_clusters + 1 */
    const int32_t *members; /* offsets[n_clusters] VPL ids */
} vplmc_cut;

/* Method parameters (Sec. 5 rates, Appendix A constants). */
typedef struct {
    uint64_t seed;        /* key of every random draw                          */
    int32_t pass1_ppm;    /* first-pass rate, parts per million of m' n'       */
    int32_t pass2_ppm;    /* second-pass rate, parts per million of m' n'      */
    int32_t max_iter;     /* ADM iteration cap (paper: 100)                    */
    int32_t flags;        /* VPLMC_FIXED_ITERS                                 */
    float tol;            /* ADM stop: relative residual on the samples        */
    float alpha0, beta0;  /* penalties alpha = alpha0 3n'/q, beta = beta0 m'/q */
    float gamma;          /* multiplier step, in (0, 1.618)                    */
    float r_min;          /* distance clamp of the geometry term               */
    float ray_eps;        /* shadow-ray origin offset along the normal         */
    float lam;            /* masked-ALS regulariser: lam max(1, n) I per row / column (> 0) */
    float pass2_mix;      /* second-pass column density g(j) + pass2_mix mean g:
                           * 0 is Sec. 5's g (the default), +inf the uniform
                           * density; a comparison baseline for the learned
                           * proposal.  Integer weights: q_j = the g weights,
                           * c = floor(pass2_mix sum q / n'), w_j = q_j if c = 0,
                           * else max(1, floor(2^24 (q_j + c) / (2^24 + c))).
                           * Must be >= 0 (VPLMC_EINVAL otherwise); ignored for
                           * slices sampled by the learned proposal.          */
} vplmc_params;

typedef struct vplmc_ctx vplmc_ctx;
typedef struct vplmc_plan vplmc_plan;

/* Per-slice layout of one frame's intermediate data inside the workspace
 * (byte offsets are relative to the start of each region). */
typedef struct {
    int32_t m, n, q;         /* rows, cut columns, rank                           */
    int32_t N1, N2;          /* first-pass count and second-pass target           */
    int32_t adm_in_lds;      /* 1: the ADM kernel keeps X in LDS; 0: in global memory */
    int32_t q_pad;           /* row length of X and Y: the next of 4, 8, 16, 32 >= q;
                                components q .. q_pad-1 stay 0                     */
    int32_t reserved;
    int64_t off1, off2;      /* element offsets into OMEGA1/VAL1, OMEGA2/VAL2     */
    int64_t off_omega;       /* element offset into CSR_* / CSC_* (N1 + N2 each)  */
    int64_t off_col;         /* element offset into per-column regions            */
    int64_t off_row;         /* element offset into ROW_PTR (m + 1 each)          */
    int64_t off_colptr;      /* element offset into COL_PTR (n + 1 each)          */
    int64_t off_x;           /* element offset into X / XP / LAMBDA (m q each)    */
    int64_t off_y;           /* element offset into Y / YP / PI (n 3 q each)      */
} vplmc_slice_info;

/* Workspace regions readable after vplmc_render (for inspection and tests). */
enum {
    VPLMC_R_LIGHTS = 0,   /* float[9][n_clusters]: x y z nx ny nz ir ig ib of the cluster lights */
    VPLMC_R_REP,          /* int32[n_clusters]: representative VPL                         */
    VPLMC_R_BBOX,         /* float[6][n_clusters]: member bbox lo xyz, hi xyz              */
    VPLMC_R_OMEGA1,       /* uint32 (i << 16 | j): first-pass entries, draw order          */
    VPLMC_R_VAL1,         /* float[3] per first-pass entry                                 */
    VPLMC_R_OMEGA2,       /* uint32: second-pass entries, acceptance order                 */
    VPLMC_R_VAL2,         /* float[3] per second-pass entry                                */
    VPLMC_R_WEIGHTS,      /* uint32 per (slice, column): quantised importance g            */
    VPLMC_R_COLMIN,       /* float per (slice, column): min of R+G+B over the first pass   */
    VPLMC_R_COLMAX,       /* float per (slice, column): max                                */
    VPLMC_R_COLCNT,       /* int32 per (slice, column): first-pass observations            */
    /* ROW_PTR, CSR_* and CSC_* describe Omega only for slices completed in
     * global memory (vplmc_slice_info.adm_in_lds = 0); a slice completed in
     * LDS is completed from an internal ELL copy, and its CSC_* regions keep
     * the first pass alone (the column statistics' ordering). */
    VPLMC_R_ROW_PTR,      /* int32[m + 1] per slice: CSR row pointers                      */
    VPLMC_R_CSR_COL,      /* int32 per entry: column, CSR order (row-major)                */
    VPLMC_R_CSR_VAL,      /* float[3] per entry, CSR order                                 */
    VPLMC_R_COL_PTR,      /* int32[n + 1] per slice: CSC column pointers (every slice)     */
    VPLMC_R_CSC_ROW,      /* int32 per entry: row, CSC order (column-major)                */
    VPLMC_R_CSC_VAL,      /* float[3] per entry, CSC order                                 */
    VPLMC_R_X,            /* float[m][q_pad] per slice: final X (initial X when max_iter = 0) */
    VPLMC_R_Y,            /* float[n][3][q_pad] per slice: final Y (row c n + j of the paper's Y^T) */
    VPLMC_R_SLICE_SCALE,  /* float per slice: s0, the mean sampled value M is divided by   */
    VPLMC_R_FEATURES,     /* float[12] per (slice, column): proposal features (learned mode) */
    VPLMC_R_LOGITS,       /* float per (slice, column): proposal log-density (learned mode) */
    /* plans with light coarsening only (0 bytes otherwise); LIGHTS, REP and
     * BBOX then hold the 2 n_leaves - 1 nodes of the tree (leaves first) */
    VPLMC_R_COLUMNS,      /* int32 per (slice, column): tree node of the column             */
    VPLMC_R_NODE_EPS,     /* float per (slice, split node): merge error eps (Sec. 4)        */
    VPLMC_R_LEAF_DRAWS,   /* int32 per leaf: row draws per slice before the cap at m'       */
    VPLMC_R_NODE_MEMBERS, /* int32 per node: VPLs below it                                  */
    VPLMC_R_COUNT
};

/* ---- library ---------------------------------------------------------- */
int vplmc_version(void);
const char *vplmc_last_error(void);
/* Paper defaults: 5% + 5%, max_iter 100, tol 1e-3, alpha0 = beta0 = 0.1,
 * gamma 1.6, r_min 0.05, ray_eps 1e-4, seed 1; lam 0.01 (masked ALS). */
int vplmc_default_params(vplmc_params *out /* HOST */);

/* ---- context: device + stream ---------------------------------------- */
/* stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream), or
 * NULL for the null stream.  The context also creates three non-blocking
 * streams of default priority and four events for the completion's rank
 * groups; vplmc_destroy releases them. */
int vplmc_create(int device, void *stream, vplmc_ctx **out /* HOST */);
int vplmc_destroy(vplmc_ctx *ctx);
int vplmc_set_stream(vplmc_ctx *ctx, void *stream);

/* Occluder spheres (centre, radius; HOST arrays).  Builds a BVH on the host
 * and uploads it; shadow rays of every later call test against it
 * (Sec. 6 ray casting; vplmc_set_triangles takes triangle meshes instead).
 * n = 0 removes all occluders. */
int vplmc_set_occluders(vplmc_ctx *ctx, int32_t n, const float *cx, const float *cy,
                        const float *cz, const float *r);

/* Occluder triangles (HOST, 9 floats each: v0, v1, v2), replacing any
 * spheres: builds a spatial-split BVH (SBVH, Sec. 6's ray-casting structure;
 * binned surface-area heuristic with object and spatial splits, references
 * chopped at the split planes) on the host and uploads it; shadow rays of
 * every later call test the open segment against the triangles.  n = 0
 * removes all occluders.  Errors: VPLMC_EINVAL for n outside [0, 2^24], a
 * NULL array with n > 0 or a non-finite vertex; VPLMC_ENOMEM. */
int vplmc_set_triangles(vplmc_ctx *ctx, int32_t n, const float *v /* HOST */);

/* The sphere BVH vplmc_set_occluders builds, for inspection (host only, no
 * device): node boxes (6 floats per node), node codes (2 per node: leaf code
 * first << 4 | count, 0 for an inner node; skip index) in depth-first order,
 * and the sphere at every leaf position.  Counts in *n_nodes (and n spheres);
 * VPLMC_EINVAL if they exceed max_nodes (outputs untouched) or the input is
 * invalid (as for vplmc_set_occluders). */
int vplmc_bvh_build(int32_t n, const float *cx /* HOST */, const float *cy /* HOST */, const float *cz /* HOST */,
                    const float *r /* HOST */, int32_t max_nodes, float *box /* HOST */, int32_t *code /* HOST */,
                    int32_t *order /* HOST, n */, int32_t *n_nodes /* HOST */);

/* The SBVH vplmc_set_triangles builds, for inspection (host only, no
 * device): node boxes (6 floats per node: lo xyz, hi xyz, padded as used),
 * node codes (2 per node: leaf code first_reference << 4 | count, 0 for an
 * inner node; skip index, the node after the subtree) in depth-first order,
 * and the triangle of every leaf reference.  The counts are written to
 * *n_nodes and *n_refs; VPLMC_EINVAL if they exceed max_nodes / max_refs
 * (the outputs are then left untouched) or the input is invalid. */
int vplmc_sbvh_build(int32_t n, const float *v /* HOST */, int32_t max_nodes, float *box /* HOST */,
                     int32_t *code /* HOST */, int32_t max_refs, int32_t *refs /* HOST */, int32_t *n_nodes /* HOST */,
                     int32_t *n_refs /* HOST */);

/* ---- frame plan (host only: no device work) ---------------------------- */
/* Slice s owns points pt_ids[pt_offsets[s] .. pt_offsets[s+1]) and cut
 * clusters cl_ids[cl_offsets[s] .. cl_offsets[s+1]) and completes at rank
 * rank[s].  All three arrays are HOST (n_slices + 1, n_slices + 1, n_slices).
 * Rejects m' > VPLMC_MAX_ROWS, n' > VPLMC_MAX_COLS, q < 1,
 * q > min(VPLMC_MAX_RANK, m', n'), rates outside [0, 10^6] or summing above it.
 * Any rank 1..32 is served: the completion runs at the next of 4, 8, 16, 32
 * with the extra components of X and Y held at exactly 0, which leaves the
 * rank-q iteration unchanged. */
int vplmc_plan_create(int32_t n_slices, const int32_t *pt_offsets, const int32_t *cl_offsets,
                      const int32_t *rank, int32_t n_clusters, const vplmc_params *params,
                      vplmc_plan **out /* HOST */);

/* Per-slice light coarsening (Sec. 4).  The global cut's clusters are the
 * leaves of a binary tree, the light tree above the cut: split node
 * n_leaves + k has children left[k] and right[k], each a leaf or an earlier
 * split node, and every node but the root (node 2 n_leaves - 2) is the child
 * of exactly one split node.  A split node keeps the position and normal of
 * one child a, drawn with probability proportional to the children's
 * quantised intensities (Philox, seed), and the summed intensity.  For each
 * slice, `pixels` row draws are shared out over the leaves in proportion to
 * their intensity (each leaf's rows distinct, from its own keyed
 * permutation of the slice's rows, at most m' per leaf); the error of
 * merging split node f is eps(f) = max over the rows drawn below f and the
 * channels of |V_b - V_a I_b / I_a|, its cost eps(f) + cost(dropped child)
 * (leaves cost 0).  Sibling pairs are merged from the least cost on until
 * the slice has n_max[s] columns, and further while the cost stays below
 * `bound`, never below the slice's rank q; the remaining nodes, ordered by
 * their smallest leaf, are the slice's columns.  The first pass of the
 * coarsened slice is the set of (row, column) entries the draws hit (Sec. 5);
 * the second pass, completion and sum follow as in vplmc_render. */
typedef struct {
    int32_t n_leaves;        /* clusters of the global cut, [1, VPLMC_MAX_LEAVES]                */
    int32_t pixels;          /* row draws per slice, [0, 2^30]                                    */
    const int32_t *left;     /* HOST, n_leaves - 1                                                */
    const int32_t *right;    /* HOST, n_leaves - 1                                                */
    const int32_t *n_max;    /* HOST, n_slices: column cap of each slice (>= 1)                   */
    double bound;            /* merge further while the least cost is below it (>= 0; 0: caps only) */
    int32_t reserved;        /* 0 */
} vplmc_coarsen;
/* A frame plan whose slices coarsen the cut (HOST arrays as in
 * vplmc_plan_create; no column layout: slice s gets at most
 * n'_s = min(n_leaves, max(rank[s], n_max[s])) columns, exactly that many
 * when bound = 0).  vplmc_plan_slice then reports n', N1 (at most pixels)
 * and N2 as capacities; a frame's own counts are read with
 * vplmc_read_counts.  params.pass1_ppm is not used by such a plan.  Its
 * frames take the global cut (n_leaves clusters) as `cut` and ignore
 * `cl_ids` (which may be NULL). */
int vplmc_plan_create_coarse(int32_t n_slices, const int32_t *pt_offsets, const int32_t *rank,
                             const vplmc_coarsen *coarsen, const vplmc_params *params,
                             vplmc_plan **out /* HOST */);
int vplmc_plan_destroy(vplmc_plan *plan);
int vplmc_workspace_size(const vplmc_plan *plan, size_t *bytes /* HOST */);
int vplmc_plan_slice(const vplmc_plan *plan, int32_t s, vplmc_slice_info *out /* HOST */);
int vplmc_plan_region(const vplmc_plan *plan, int32_t region, size_t *offset /* HOST */,
                      size_t *bytes /* HOST */);

/* ---- the method ---------------------------------------------------------
 * One frame (Sec. 3 steps 4-5, Sec. 5, Appendix A):
 *   cluster table of the cut (Sec. 4: I_f = sum of member intensities,
 *   position/normal of one member) -> first pass (uniform distinct entries)
 *   -> entries with shadow rays -> g(j) = max - min of the first pass ->
 *   second pass by g -> CSR/CSC of all samples -> ADM completion of the
 *   stacked m' x 3n' slice matrix [M_R | M_G | M_B] -> I(s) = X (Y e).
 * pt_ids / cl_ids: DEVICE int32 arrays of the layout given to the plan.
 * workspace: DEVICE, at least vplmc_workspace_size bytes, 256-byte aligned.
 * radiance: DEVICE float[m][3]; points outside every slice are set to 0.
 * params must equal, in its rates, the params given to the plan.
 * Index arrays are not range-checked on the host (they live on the device):
 * an out-of-range point, cluster or member id is clamped into range by the
 * kernels, so it never reads or writes outside the caller's arrays, and the
 * frame's result is then meaningless; vplmc_check_inputs finds such ids.
 * The cut's offsets must be non-decreasing from 0 (also checked there). */
int vplmc_render(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points,
                 const vplmc_lights *vpls, const vplmc_cut *cut, const int32_t *pt_ids,
                 const int32_t *cl_ids, const vplmc_params *params, void *workspace,
                 size_t workspace_bytes, float *radiance);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * frame as vplmc_render, with the workspace replaced by a static device array
 * of VPLMC_STATIC_WORKSPACE_BYTES that the library holds on every GPU it runs
 * on until the process ends.  Calls no allocating routine.  Returns
 * VPLMC_EINVAL if the plan's workspace (vplmc_workspace_size) exceeds that
 * size; small frames only (the tiny 64 x 64 configuration needs 46 MiB).
 * All calls on one GPU share the array, which keeps the last frame's
 * contents (every buffer a frame reads is cleared or written by that frame
 * first): calls that overlap on one GPU, from any context or stream, race
 * and must be ordered by the caller.  The per-slice stats of such a frame
 * are not readable (vplmc_read_stats needs the workspace pointer). */
#define VPLMC_STATIC_WORKSPACE_BYTES (64u << 20)
int vplmc_render_static(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points,
                        const vplmc_lights *vpls, const vplmc_cut *cut, const int32_t *pt_ids,
                        const int32_t *cl_ids, const vplmc_params *params, float *radiance);

/* Per-slice outcome of the last vplmc_render on this workspace (synchronises).
 * HOST arrays of n_slices each; any may be NULL. */
int vplmc_read_stats(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace,
                     int32_t *iters, int32_t *flags, float *resid, int32_t *n2_accepted);

/* Per-slice column count n', first-pass count N1 and second-pass target N2
 * of the last frame rendered on this workspace (synchronises).  HOST arrays
 * of n_slices each; any may be NULL.  Without coarsening these equal the
 * plan's values. */
int vplmc_read_counts(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace, int32_t *n,
                      int32_t *N1, int32_t *N2);

/* Totals of the last frame rendered on this workspace (synchronises), HOST
 * int64[4]: sampled entries (both passes), shadow rays cast for them (entries
 * whose point and light face each other), entries the light coarsening
 * evaluated (unit-intensity lighting of a drawn row by a node's light), and
 * the shadow rays among those. */
int vplmc_read_totals(vplmc_ctx *ctx, const vplmc_plan *plan, const void *workspace, int64_t *out);

/* Counts, on the device, the ids that break the contract of vplmc_render:
 * pt_ids outside [0, n_points), cl_ids outside [0, n_clusters), cut offsets
 * not non-decreasing from 0, and (when the offsets are ordered) members
 * outside [0, n_vpls).  *n_bad (HOST) = 0 means every id is valid.
 * Synchronises the context's stream; allocates a 16-byte counter. */
int vplmc_check_inputs(vplmc_ctx *ctx, const vplmc_plan *plan, int32_t n_points, int32_t n_vpls,
                       const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids, int64_t *n_bad);

/* ---- phase timing ---------------------------------------------------------
 * Between begin and end, every vplmc_render on this context records HIP
 * events on its stream around each phase (at most max_frames frames; later
 * frames are not recorded).  end synchronises the stream and returns the
 * summed milliseconds per phase (HOST double[VPLMC_N_PHASES]) and the
 * number of frames recorded. */
#define VPLMC_N_PHASES 11
enum {
    VPLMC_PH_SETUP = 0,   /* descriptor upload and buffer clears     */
    VPLMC_PH_CLUSTER,     /* cluster table (and tree node table)     */
    VPLMC_PH_COARSEN,     /* light coarsening: merge errors, columns */
    VPLMC_PH_PASS1,       /* first-pass sampling                     */
    VPLMC_PH_EVAL1,       /* entries of the first pass               */
    VPLMC_PH_WEIGHTS,     /* column statistics and importance        */
    VPLMC_PH_PASS2,       /* second-pass sampling                    */
    VPLMC_PH_EVAL2,       /* entries of the second pass              */
    VPLMC_PH_SORT,        /* ordering of Omega (ELL copy, CSR / CSC) */
    VPLMC_PH_ADM,         /* ADM completion                          */
    VPLMC_PH_REDUCE       /* factorised column sum                   */
};
int vplmc_profile_begin(vplmc_ctx *ctx, int32_t max_frames);
int vplmc_profile_end(vplmc_ctx *ctx, double *ms /* HOST */, int32_t *frames /* HOST */);

/* ---- batching: launch shapes, autotuning, captured frames ----------------
 * All slices of a frame, whatever their m', n' and q, run in one launch per
 * phase (per rank bucket for the completion).  The plan carries the launch
 * shapes; integer results never depend on them, floating-point results only
 * through summation order within the completion's tolerance. */
typedef struct {
    int32_t adm_queue;     /* 0: one workgroup per slice; 1: as many workgroups as fit on the
                              device take slices (largest first) from a device work queue   */
    int32_t adm_threads;   /* threads of the LDS-resident completion workgroup: 512 or 1024 */
    int32_t eval_threads;  /* threads per block of the entry kernel: 64, 128 or 256         */
    int32_t reserved;      /* 0 */
} vplmc_tune;
/* Defaults: queue 0, 1024 completion threads, 256 entry threads. */
int vplmc_plan_get_tune(const vplmc_plan *plan, vplmc_tune *out /* HOST */);
int vplmc_plan_set_tune(vplmc_plan *plan, const vplmc_tune *tune /* HOST */);
/* Times `reps` frames (after one warm-up frame) of vplmc_render for each
 * candidate launch shape on these inputs, by coordinate descent over the
 * fields above, and leaves the fastest in the plan (also returned in *best,
 * which may be NULL).  Same arguments as vplmc_render; synchronises; the
 * radiance and workspace hold the last frame rendered.  reps in [1, 100]. */
int vplmc_autotune(vplmc_ctx *ctx, vplmc_plan *plan, const vplmc_points *points, const vplmc_lights *vpls,
                   const vplmc_cut *cut, const int32_t *pt_ids, const int32_t *cl_ids,
                   const vplmc_params *params, void *workspace, size_t workspace_bytes, float *radiance,
                   int32_t reps, vplmc_tune *best /* HOST, may be NULL */);

/* A whole vplmc_render recorded once as a HIP graph, replayed by one call.
 * create renders one frame eagerly (which validates the arguments and
 * uploads the slice table), then captures the frame on a private stream.
 * The inputs, workspace and radiance must stay at the same addresses; their
 * contents may change between launches.  The plan (and its launch shapes)
 * must outlive the graph; changing the plan's tune needs a new graph.
 * Profiling must be off during create.  launch enqueues on the context's
 * stream and does not synchronise. */
typedef struct vplmc_graph vplmc_graph;
int vplmc_graph_create(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points,
                       const vplmc_lights *vpls, const vplmc_cut *cut, const int32_t *pt_ids,
                       const int32_t *cl_ids, const vplmc_params *params, void *workspace,
                       size_t workspace_bytes, float *radiance, vplmc_graph **out /* HOST */);
int vplmc_graph_launch(vplmc_ctx *ctx, vplmc_graph *graph);
int vplmc_graph_destroy(vplmc_graph *graph);

/* ---- building blocks used by the frame, exposed for tests and tools ---- */
/* Cluster table (Sec. 4): rep[c], lights float[9][n_clusters] (x y z nx ny nz
 * ir ig ib), bbox float[6][n_clusters].  All DEVICE outputs. */
int vplmc_cluster_table(vplmc_ctx *ctx, const vplmc_lights *vpls, const vplmc_cut *cut,
                        uint64_t seed, int32_t *rep, float *lights, float *bbox);

/* Entries A(point_ids[k], light_ids[k]) (Sec. 3) for n_pairs pairs, with
 * shadow rays against the occluders: out float[n_pairs][3]. */
int vplmc_eval_pairs(vplmc_ctx *ctx, const vplmc_points *points, const vplmc_lights *lights,
                     int64_t n_pairs, const int32_t *point_ids, const int32_t *light_ids,
                     const vplmc_params *params, float *out);

/* Brute-force column sum over every light (the paper's reference images,
 * Sec. 6): out double[n_out][3] for points point_ids[0 .. n_out) (or points
 * 0 .. n_out-1 if point_ids is NULL).  FP32 entries, FP64 sums; partial sums
 * over chunks of 2048 lights are combined with FP64 atomics, so the last
 * bits may vary between runs. */
int vplmc_brute_force(vplmc_ctx *ctx, const vplmc_points *points, const vplmc_lights *lights,
                      int32_t n_out, const int32_t *point_ids, const vplmc_params *params,
                      double *out);

/* ---- global light cut (Sec. 3, step 1; Sec. 6) -------------------------------
 * Step 1 of the method: the cut of a light tree over every VPL that the
 * lightcut method (Walter et al. 2005) picks for the whole image, with the
 * visibility bounded by 1 (conservative) and the split test run for all
 * nodes of one tree level at a time.
 *
 * Tree (HOST arrays, read by vplmc_lightcut_plan_create only): leaves
 * 0 .. n_leaves-1 are the VPLs perm[0 .. n_leaves) (a permutation); split
 * node n_leaves + k has children left[k], right[k], both below
 * n_leaves + k, every node but the root 2 n_leaves - 2 the child of one split
 * node, and the leaves under every node contiguous, the left child's first.
 *
 * Node lights: a leaf is its VPL; split node f keeps the position and normal
 * of child a drawn with probability Q_a / (Q_l + Q_r),
 * Q = max(1, floor(2^24 t / max(t_l, t_r))), t = (R + G) + B in FP64, by
 * Philox4x64-10 with key (seed, 0) and counter (f, 0, 8, 0) (a = left iff
 * mulhi64(word 0, Q_l + Q_r) < Q_l); I_f = fp32(fp64(I_l) + fp64(I_r)); the
 * box is the union of the children's boxes.
 *
 * Split test at sample pixel x (position p, normal n, kd, ks, e):
 *   est(x)    = the current cut's entries with V = 1, summed over nodes and channels
 *   bound(x,f) = c / max(d^2, r_min^2) * sum_c (kd_c / pi + ks (e + 2) / (2 pi)) I_f,c
 *   d = distance from p to f's box, h = max over the box of n . (y - p),
 *   c = 0 if h <= 0, else min(1, h / d) (1 if d = 0)
 *   rho(f) = max over the samples of bound / est (b / 0 = inf, 0 / 0 = 0; no samples: 0)
 * The root is level 0; the nodes of a level that are not single VPLs are
 * tested against the estimate of the current cut and all with rho > eps
 * split at once, their children forming the next level.  When the failing
 * nodes would take the cut past max_cut, only the max_cut - |cut| with the
 * largest rho split (ties: lower node id) and the cut is final.
 *
 * Outputs, DEVICE: n_cut[1]; cut_nodes[max_cut] and cut_offsets[max_cut + 1]:
 * the cut by smallest leaf, cluster k holding the VPLs
 * perm[cut_offsets[k] .. cut_offsets[k+1]) (so {n_cut, cut_offsets, perm} is
 * a vplmc_cut); above_left / above_right [max_cut - 1] (each may be NULL): the
 * tree above the cut in the layout of vplmc_coarsen (the cut's nodes are
 * leaves 0 .. n_cut-1 in cut order, the split nodes follow by increasing tree
 * id); rho[2 n_leaves - 1] (may be NULL): rho of every tested node, -1
 * elsewhere.  Only the first n_cut (+1) entries of the cut arrays are
 * written.  sample_ids: DEVICE [n_samples] point ids in [0, points->m)
 * (others read a clamped point).  The bound is FP32, est FP64 over FP32
 * entries.  Errors: VPLMC_EINVAL for a malformed tree, eps < 0 or NaN,
 * r_min <= 0, vpls->n != n_leaves, a short or misaligned workspace. */
typedef struct {
    int32_t n_leaves;
    const int32_t *perm;  /* n_leaves     */
    const int32_t *left;  /* n_leaves - 1 */
    const int32_t *right; /* n_leaves - 1 */
} vplmc_light_tree;

typedef struct vplmc_lightcut_plan vplmc_lightcut_plan;
int vplmc_lightcut_plan_create(const vplmc_light_tree *tree /* HOST */, int32_t n_samples, int32_t max_cut,
                               vplmc_lightcut_plan **out /* HOST */);
int vplmc_lightcut_plan_destroy(vplmc_lightcut_plan *plan);
int vplmc_lightcut_workspace_size(const vplmc_lightcut_plan *plan, size_t *bytes /* HOST */);
int vplmc_lightcut(vplmc_ctx *ctx, const vplmc_lightcut_plan *plan, const vplmc_points *points,
                   const vplmc_lights *vpls, const int32_t *sample_ids, double eps, float r_min, uint64_t seed,
                   void *workspace, size_t workspace_bytes, int32_t *n_cut, int32_t *cut_nodes,
                   int32_t *cut_offsets, int32_t *above_left, int32_t *above_right, float *rho);

/* ---- learned second-pass proposal ------------------------------------------
 * A 12 -> 128 -> 128 -> 1 GELU network predicting the log sampling density
 * of each (slice, column) from first-pass statistics and geometry; it
 * replaces g(j) = max C_j - min C_j (Sec. 5) as the column pdf when
 * params.flags has VPLMC_LEARNED.  Parameters are one FP32 vector of
 * vplmc_mlp_param_count() values, in the order W1[128][12], b1[128],
 * W2[128][128], b2[128], W3[128], b3; the kernels use the weights rounded to
 * bfloat16 and round both hidden activations to bfloat16.
 * Column weights become max(1, floor(2^24 exp(y_j - max y))) (FP64 from the
 * FP32 logits); a slice with a non-finite logit keeps the g weights and gets
 * VPLMC_SLICE_FALLBACK. */
int vplmc_mlp_param_count(void);
/* params: DEVICE, owned by the caller, must stay valid while renders use it; NULL removes the model. */
int vplmc_set_proposal(vplmc_ctx *ctx, const float *params);
/* y[r] for rows of 12 features (DEVICE float[rows][12] -> float[rows]). */
int vplmc_mlp_forward(vplmc_ctx *ctx, const float *params, int64_t rows, const float *features, float *y);
/* DEVICE scratch needed by vplmc_mlp_grad / vplmc_mlp_train_step for `rows` rows. */
int vplmc_mlp_scratch_size(int64_t rows, size_t *bytes /* HOST */);
/* grad = d(sum_r dy[r] y[r]) / d params (DEVICE float[param_count]). */
int vplmc_mlp_grad(vplmc_ctx *ctx, const float *params, int64_t rows, const float *features, const float *dy,
                   void *scratch, size_t scratch_bytes, float *grad);
/* One Adam step (lr, 0.9, 0.999, 1e-8, bias-corrected; step counts from 1) on params with moments m, v. */
int vplmc_mlp_adam(vplmc_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr);
/* Forward, loss sum over groups of KL(pstar || softmax(y)) (groups = rows
 * [group_offsets[g], group_offsets[g+1]), DEVICE int32), backward and Adam.
 * loss: DEVICE float, overwritten.  After the call the scratch begins with
 * this step's gradient (float[param_count]), then its logits y (float[rows])
 * and dloss/dy = softmax(y) - pstar (float[rows]), for inspection. */
int vplmc_mlp_train_step(vplmc_ctx *ctx, float *params, float *m, float *v, int32_t step, float lr, int64_t rows,
                         const float *features, const float *pstar, int32_t n_groups, const int32_t *group_offsets,
                         void *scratch, size_t scratch_bytes, float *loss);
/* Training targets from fully evaluated slices: pstar per (slice, column) in
 * the plan's column layout, p*_j ~ sigma_j + 3 mean(sigma), sigma_j the
 * standard deviation of R+G+B over the column.  lights: DEVICE float[9][n_clusters]
 * (vplmc_cluster_table); the workspace is used as scratch. */
int vplmc_proposal_targets(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points, const float *lights,
                           const int32_t *pt_ids, const int32_t *cl_ids, const vplmc_params *params, void *workspace,
                           size_t workspace_bytes, float *pstar);

/* ---- stage calls: the frame's kernels on inputs the caller places in the
 * workspace's public regions (parity tests, tools).  Plans without
 * coarsening only; each validates on the host, synchronises, and returns
 * VPLMC_EINVAL when a first-pass entry in OMEGA1 lies outside its slice or
 * repeats within it (nothing further is launched then). -------------------- */

/* Second pass (Sec. 5) of every slice given its first pass (OMEGA1: N1
 * entries per slice, packed i << 16 | j, any order) and its column weights
 * (WEIGHTS: uint32 per (slice, column), not all 0): OMEGA2 receives the
 * accepted entries in acceptance order and vplmc_read_stats their count and
 * the shortfall flag.  The inclusive prefix of the weights is kept in 64
 * bits, so any uint32 weights are exact. */
int vplmc_stage_pass2(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_params *params,
                      void *workspace, size_t workspace_bytes);

/* Completion (Appendix A) and factorised sum (Sec. 3, step 5) of every slice
 * from the samples in OMEGA1 / VAL1 (N1 distinct entries per slice with RGB
 * values; no second pass), with params.max_iter, tol, alpha0, beta0, gamma,
 * VPLMC_FIXED_ITERS and VPLMC_GIVEN_INIT (then X and Y hold the initial
 * factors, layouts as the X and Y regions).  Fills X, Y, SLICE_SCALE, the
 * per-slice stats and radiance float[n_points][3] (0 outside the slices). */
int vplmc_stage_adm(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_params *params,
                    const int32_t *pt_ids, int32_t n_points, void *workspace, size_t workspace_bytes,
                    float *radiance);

/* Factorised column sum I(s) = s0 X (Y e) (Sec. 3, step 5) of every slice
 * from the X, Y and SLICE_SCALE regions: radiance float[n_points][3]. */
int vplmc_stage_reduce(vplmc_ctx *ctx, const vplmc_plan *plan, const int32_t *pt_ids, int32_t n_points,
                       void *workspace, size_t workspace_bytes, float *radiance);

/* Every entry A(i, j) (Sec. 3) of slices [slice_begin, slice_end) of a plan
 * without coarsening: lights float[9][n_lights] as the LIGHTS region, cl_ids
 * indexing them; out float[sum m' n'][3], slice after slice, row-major (i, j). */
int vplmc_full_matrix(vplmc_ctx *ctx, const vplmc_plan *plan, const vplmc_points *points,
                      const float *lights, int32_t n_lights, const int32_t *pt_ids, const int32_t *cl_ids,
                      const vplmc_params *params, int32_t slice_begin, int32_t slice_end, float *out);

/* Philox4x64-10 (Salmon et al., SC'11): out[4k .. 4k+3] =
 * Philox(key, ctr[4k .. 4k+3]); ctr/out DEVICE uint64[4 n]. */
int vplmc_philox4x64(vplmc_ctx *ctx, uint64_t key0, uint64_t key1, const uint64_t *ctr,
                     int64_t n, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif /* VPLMC_H */
