// Internal (non-ABI) declarations of libba: the device-resident problem, the
// build primitives and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "ba.h"
#include "ba_host.hpp"

namespace ba {

static inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// One K_vox wave group: up to 64 voxels with the same cluster count m, one
// voxel per lane; cluster k of lane l lives at cbase + 64 k + l.
struct GroupDesc {
    int64_t cbase;
    int32_t m;
    int32_t nvox;
    int32_t window;
    int32_t scan0;   // lowest scan of the group's clusters
    int32_t nscan;   // scans from scan0 to the highest one
    int32_t pad;
};

// Device-side Levenberg-Marquardt state of one window.
struct LMState {
    double mu, nu;
    double cost, cost_trial;
    double q, rho;
    double gnorm, maxdiag;
    double cost0;
    int32_t accepted, need_eval, info, done;   // done: 1 converged (||g|| < tol_g), 2 stalled
    int32_t iters, n_accepted, cur, rejects;   // rejects: rejected steps in a row
};

// One residual-pass block: `ng` consecutive groups served one wave each
// (split == 1), or one group whose clusters four waves share (split == 4).
struct VoxBlock {
    int32_t g0, ng, split, window;
};

// One pose chunk: `count` consecutive clusters of the pose-sorted layout,
// all observed by `pose`.
struct ChunkDesc {
    int64_t start;
    int32_t count;
    int32_t pose;
};


// Arguments of the per-window LM decision kernel.
struct DecideArgs {
    int32_t W;
    const int32_t *win_pose_ptr, *win_group_ptr;
    const double *pose_q;
    const int32_t *pose_info;
    const double *group_cost;
    LMState *lm;
    double *trace;
    int32_t it;
    int32_t max_rejects;
    const double *poses_trial;
    double *poses;
};

static constexpr int VSTATE = 8;    // doubles per voxel slot: u[3] mbar[3] 2/N lam0
static constexpr int NPART = 27;    // g[6] + Hpp[6] + Hpt[9] + Htt[6]

// Launch choices of the two evaluation passes (ba_tuning).
struct Tuning {
    int32_t vox_split = 4;   // waves sharing one 64-voxel group in the residual pass (0: per group, by its size)
    int32_t vox_grid = 0;    // 0: one block per group; k > 0: persistent grid of k blocks per CU
    int32_t pose_grid = 0;   // 0: one wave per chunk; k > 0: persistent grid of k blocks per CU
    int32_t chunk_len = 256; // clusters per derivative-pass chunk
};

static constexpr int32_t MIN_CHUNK = 32;   // smallest chunk length the chunk tables are sized for
static constexpr int32_t MAX_CHUNK = 1024; // longest chunk (the FP32 Hessian sums of a lane hold at most 16 terms)

struct Problem {
    int device = 0;
    int n_cu = 256;              // compute units of the device
    Tuning tune;
    int32_t tune_gen = 0;        // bumped on every tuning change (captured graphs depend on it)
    bool no_graph = false;       // ba_iterate launches eagerly (one-shot problems of the request server)
    std::vector<int64_t> h_pose_start;   // [n_poses+1] pose ranges of the pose-major layout
    int64_t chunk_cap = 0;       // capacity of chunks / partials (chunk descriptors)
    int32_t n_poses = 0, n_voxels_in = 0, n_windows = 1;
    int64_t n_clusters = 0;
    int32_t n_vox = 0;          // voxels with at least one cluster
    int32_t n_groups = 0;
    int64_t c_pad = 0;          // clusters incl. padding in the K_vox layout
    int32_t n_chunks = 0;
    int32_t chunk_len = 0;      // max clusters per pose chunk
    int32_t max_m = 0;
    int32_t prec = BA_PREC_F64;   // storage of the two iteration copies

    // K_vox layout (component-major SoA, length c_pad per component)
    double *v_mu = nullptr;     // [3][c_pad]
    double *v_S = nullptr;      // [6][c_pad]
    double *v_N = nullptr;      // [c_pad]
    int32_t *v_pose = nullptr;  // [c_pad]
    GroupDesc *groups = nullptr;
    VoxBlock *vblocks = nullptr;
    int32_t n_vblocks = 0;
    VoxBlock *vblocks_mix = nullptr;   // per-group split: 4 one-wave, 2 two-wave or 1 four-wave group per block
    int32_t n_vblocks_mix = 0;
    int32_t *slot_vox = nullptr; // slot -> input voxel id (-1 padding), n_groups*64
    double *vstate = nullptr;   // [2][n_groups*64][VSTATE]
    double *wave_cost = nullptr; // [n_groups]

    // precision form: the same two layouts in FP32, voxel-centred
    float *v_mu32 = nullptr, *v_S32 = nullptr, *v_N32 = nullptr;  // [3][c_pad], [6][c_pad], [c_pad]
    float *p_mu32 = nullptr, *p_S32 = nullptr, *p_N32 = nullptr;  // [3][C], [6][C], [C]
    double *v_ref = nullptr;      // [n_groups*64][4] reference point c_i of each voxel slot (xyz, pad)
    double *ref_poses = nullptr;  // [n_poses][12] poses that placed the references
    double *pdelta = nullptr;     // [n_poses][16] pose change of the evaluated poses: E (9), w = dt - E t0 (3)

    // pose-sorted layout (length n_clusters per component)
    double *p_mu = nullptr;     // [3][C]
    double *p_S = nullptr;      // [6][C]
    double *p_N = nullptr;      // [C]
    int32_t *p_slot = nullptr;  // [C]
    int32_t *p_cidx = nullptr;  // [C] (voxel, scan)-order index of each pose-major cluster
    ChunkDesc *chunks = nullptr;
    int32_t *chunk_ptr = nullptr; // [n_poses+1]
    double *partials = nullptr; // [n_chunks][NPART]

    // centred clusters in (voxel, scan) order, kept for export
    double *c_mu = nullptr, *c_S = nullptr, *c_N = nullptr; // [C][3], [C][6], [C]
    int32_t *c_vox = nullptr, *c_scan = nullptr;
    int32_t *c_slot = nullptr;                 // residual-pass slot of each cluster

    // windows
    int32_t *win_group_ptr = nullptr; // [n_windows+1]
    int32_t *win_pose_ptr = nullptr;  // [n_windows+1]
    int32_t *pose_window = nullptr;   // [n_poses]
    int32_t *h_win_pose_ptr = nullptr; // host copy

    // LM work buffers
    double *g = nullptr, *H = nullptr;       // [N][6], [N][36]
    double *dx = nullptr, *poses_trial = nullptr;
    double *pose_q = nullptr;                 // [N]
    int32_t *pose_info = nullptr;             // [N]
    LMState *lm = nullptr;                    // [n_windows]
    double *trace = nullptr;                  // [max_iters][n_windows][8]
    double *lm_init = nullptr;                // [n_windows][4] per-window LM start (ba_lm_options.resume)
    int32_t trace_cap = 0;

    // dense coupled path
    int64_t *win_dense_off = nullptr;         // [n_windows+1] offsets (doubles) of each window's dense H
    int64_t dense_total = 0;
    double *dense = nullptr;                  // per-window dense (6Nw)^2 matrices
    void *dense_state = nullptr;              // coupled-path plan and buffers
    void *iter_graph = nullptr;               // captured ba_iterate graph

    int64_t n_points = 0;
    DevArena mem;                             // every device allocation above
    ~Problem();
};

ba_status replan_chunks(Problem *P, int32_t chunk_len, hipStream_t s);
int64_t dense_device_bytes(const Problem *P);
ba_status dense_prepare(Problem *P);
double *dense_hvec(Problem *P);   // [C][6] pair vectors of the coupled form
ba_status build_from_points(const ba_points *pts, const ba_build_options *opt, Problem *P, DevArena &keep,
                            hipStream_t s);
ba_status build_from_sums(const ba_cluster_sums *cs, const ba_build_options *opt, Problem *P, DevArena &keep,
                          hipStream_t s);

// primitives
size_t scan_workspace_bytes(int64_t n);
hipError_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, void *ws, hipStream_t s);
size_t radix_sort_workspace_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int bits, void *ws, hipStream_t s);

}  // namespace ba

// The opaque handle of the C-ABI.
struct ba_problem {
    ba::Problem P;
};
