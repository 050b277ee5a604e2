// Device state of the global light cut (Sec. 3, step 1; Sec. 6) and its
// launcher, shared by the C ABI and the kernels.
#ifndef VPLMC_LIGHTCUT_H
#define VPLMC_LIGHTCUT_H

#include "vplmc_internal.h"

namespace vplmc {

// Global light cut over the full light tree (n leaves, N = 2 n - 1 nodes):
// the tree as uploaded by its plan, the node table and the level-by-level
// state, all inside the caller's workspace.
constexpr int LC_UPDATE_CHUNK = 32;    // splits per chunk of the estimate update
constexpr int LC_ORDER_BLOCK = 1024;   // leaves per block of the output ordering

struct LightcutView {
    int32_t n = 0, S = 0, cap = 0, F = 0;                  // leaves, samples, cut cap, frontier capacity
    const int32_t *perm = nullptr, *left = nullptr, *right = nullptr;
    const int32_t *order = nullptr, *min_leaf = nullptr;   // split nodes by height; per node
    const int32_t *sample_ids = nullptr;
    int32_t *rep = nullptr;                                // per node
    float *lights = nullptr, *bbox = nullptr;              // 9 and 6 planes of N
    float *samp = nullptr;                                 // 9 planes of S: x y z nx ny nz M_r M_g M_b
    double *est = nullptr;                                 // S
    float *inv_est = nullptr;                              // S: 1 / est (inf where est = 0)
    double *part = nullptr;                                // per (split chunk, sample): estimate updates
    uint32_t *state = nullptr;                             // per node: 0 not reached, 1 in the cut, 2 split
    int32_t *front = nullptr;                              // [2][F] frontier of the level, by parity
    uint32_t *rho_f = nullptr;                             // [2][F] float bits of the frontier's ratios
    int32_t *split = nullptr;                              // cap: nodes split at the level
    int32_t *ctl = nullptr;                                // n_front[2], n_cut, n_split, done, output n_cut
    uint32_t *blk = nullptr;                               // [2][blocks of LC_ORDER_BLOCK leaves]: counts, then offsets
    int32_t *leafmark = nullptr;                           // n: cut node starting at each leaf, or -1
    int32_t *ren = nullptr;                                // per node: index in the output layout
};

int launch_lightcut(hipStream_t st, const LightcutView &v, const int32_t *level_off, int32_t height_max,
                    int32_t depth, const vplmc_points &pts, const vplmc_lights &vpls, double eps, float r_min,
                    uint64_t seed, int32_t *n_cut, int32_t *cut_nodes, int32_t *cut_offsets, int32_t *above_left,
                    int32_t *above_right, float *rho);

}  // namespace vplmc

#endif
