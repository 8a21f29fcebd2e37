/*
 * libba: one Levenberg-Marquardt iteration of majorization-minimization LiDAR
 * bundle adjustment on an AMD MI355X (gfx950).
 *
 * Method: Cai et al., "Accelerating Large-scale Bundle Adjustment for LiDAR
 * Mapping via Parallel Computing".  Sec. III states the problem: scan poses
 * T_j = (R_j, t_j) in SE(3), planar voxels i observed by scans j through point
 * clusters (N_ij, sum p, sum p p^T) (Eq. 2), the cost
 *     c(T) = sum_i lambda_min( P_i/N_i - v_i v_i^T / N_i^2 )          (Eq. 1)
 * and the MM surrogate of Eq. 3 that decouples the poses.  Sec. IV-C / Alg. 2
 * gives one iteration: residual (CalRes), Jacobian and Hessian per cluster
 * reduced by pose (CalJH), and a damped per-pose increment solve (Solver).
 *
 * Conventions shared by every entry point
 *   - Memory: array arguments marked "device" are device pointers owned by
 *     the caller (e.g. PyTorch tensors); "host" arrays are host memory.  A
 *     ba_problem owns the device-resident clusters and plan it builds; it is
 *     released by ba_problem_destroy.
 *   - Streams: work is enqueued on the given hipStream_t (0 = null stream).
 *     Calls marked "synchronous" return after the stream has drained.
 *   - Errors: every call returns a ba_status; BA_OK == 0, errors are
 *     negative.  No call aborts; ba_last_error() returns a thread-local text.
 *   - Pose layout: 12 doubles per scan, [R00 R01 R02 R10 R11 R12 R20 R21 R22
 *     t0 t1 t2] (row-major rotation, then translation); a point p of scan j
 *     maps to the world as R_j p + t_j.
 *   - Increment layout: 6 doubles per scan, [phi0 phi1 phi2 dt0 dt1 dt2] in
 *     the chart T (+) x = (Exp(phi) R, t + dt) (reading of the update
 *     "T_i <- T_i + Delta T" of Alg. 2, which does not fix the chart).
 *   - Symmetric 3x3 layout: [xx xy xz yy yz zz].
 *   - Determinism: identical inputs give bitwise identical outputs (fixed
 *     reduction orders, no floating-point atomics).
 */
#ifndef BA_H
#define BA_H

#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ba_status;
#define BA_OK 0
#define BA_E_ARG (-1)          /* invalid argument (null, size, label out of range, non-finite) */
#define BA_E_WORKSPACE (-2)    /* workspace smaller than required */
#define BA_E_HIP (-3)          /* a HIP runtime call failed; text in ba_last_error() */
#define BA_E_NOT_SPD (-4)      /* a factorization met a non-positive pivot */
#define BA_E_UNSUPPORTED (-5)  /* mode or size not supported */
#define BA_E_NOMEM (-6)        /* device allocation failed */
#define BA_E_BUDGET (-7)       /* a served request can never fit the server's device-memory budget */
#define BA_E_NOT_FOUND (-8)    /* unknown or already collected request id */
#define BA_E_CANCELLED (-9)    /* a served request was cancelled before it finished */

/* Cluster storage precision of a problem (ba_build_options.precision). */
#define BA_PREC_F64 0      /* clusters stored and evaluated in FP64 */
#define BA_PREC_F32 1      /* FP32 clusters centred on a per-voxel FP64 reference point (see ba_build_clusters) */

/* Hessian forms (mode arguments). */
#define BA_MODE_MM 0       /* Eq. 3 surrogate: block-diagonal, [N][6][6] full symmetric */
#define BA_MODE_COUPLED 1  /* Hessian of u^T A(T) u with u frozen: dense per window */
#define BA_MODE_EXACT 2    /* exact Hessian of Eq. 1 (diagnostic; FP64 problems): dense per window, the coupled
                            * one plus sum_l 2/(l0 - l_l) F^l F^l^T per voxel (l = 1, 2; gaps <= 1e-12 l2 dropped) */

typedef struct ba_problem ba_problem;

/* Raw body-frame points (Sec. IV-A: points with their pose index and voxel
 * index).  All arrays are device pointers of length n. */
typedef struct ba_points {
    int64_t n;
    const double *x, *y, *z;   /* device: coordinates in the observing scan's body frame */
    const int32_t *scan;       /* device: 0 <= scan < n_scans */
    const int32_t *voxel;      /* device: 0 <= voxel < n_voxels (one planar voxel per id) */
    int32_t n_scans;
    int32_t n_voxels;
} ba_points;

/* Clusters in the paper's interchange form (Eq. 2), any order, at most one per
 * (voxel, scan).  Device pointers of length n (sum: n x 3, sumsq: n x 6). */
typedef struct ba_cluster_sums {
    int64_t n;
    const int32_t *voxel, *scan;
    const int64_t *count;      /* device: N_ij >= 1 */
    const double *sum;         /* device: sum p (AoS, 3 per cluster) */
    const double *sumsq;       /* device: sum p p^T (AoS, 6 per cluster) */
    int32_t n_scans;
    int32_t n_voxels;
} ba_cluster_sums;

typedef struct ba_build_options {
    int32_t chunk_len;          /* clusters per pose chunk of the derivative pass: 0 = default (256), else 32..1024 */
    int32_t n_windows;          /* 0 or 1 = one problem; > 1 = independent windows (batched form) */
    const int32_t *scan_window; /* host, n_scans entries, non-decreasing window id per scan; NULL if n_windows <= 1 */
    int32_t precision;          /* BA_PREC_F64 (default) or BA_PREC_F32 */
    const double *ref_poses;    /* device [n_scans][12]; BA_PREC_F32 only: poses that place the voxel references */
} ba_build_options;

typedef struct ba_problem_info {
    int64_t n_points;       /* points consumed by the build (0 for the sums form) */
    int64_t n_clusters;     /* distinct (voxel, scan) clusters */
    int32_t n_voxels;       /* voxels with at least one cluster */
    int32_t n_scans;
    int32_t n_windows;
    int32_t max_m;          /* largest number of scans observing one voxel */
    int64_t device_bytes;   /* device memory held by the problem */
    int32_t n_wave_groups;  /* residual-pass wave groups (64 voxels of equal cluster count each) */
    int32_t n_pose_chunks;  /* derivative-pass chunks (clusters of one scan each) */
    int64_t padded_clusters; /* cluster slots of the wave-interleaved layout, incl. padding */
    int32_t precision;      /* BA_PREC_F64 or BA_PREC_F32 */
    int32_t cluster_bytes;  /* bytes of one stored cluster in each iteration copy (84 FP64, 44 FP32) */
} ba_problem_info;

typedef struct ba_lm_options {
    int32_t mode;        /* BA_MODE_MM or BA_MODE_COUPLED */
    int32_t max_iters;   /* iterations (solves, accepted or not) */
    double mu0;          /* initial damping (0 -> 1e-2) */
    double nu0;          /* initial damping growth (0 -> 2) */
    double tol_g;        /* stop a window once ||g||_2 < tol_g at its current poses (<= 0: never) */
    int32_t max_rejects; /* stop a window after this many rejected steps in a row (<= 0: never) */
    int32_t rejects0;    /* rejected steps in a row before this call (0; to resume a run exactly:
                          * the previous report's rejects_final) */
    double exact_below;  /* BA_MODE_COUPLED only: a window whose gradient norm at its current poses is below this
                          * takes the exact Hessian of Eq. 1 (BA_MODE_EXACT) for its step, the coupled one otherwise
                          * (FP64 problems; <= 0: never) */
    const double *resume; /* NULL, or host [n_windows][4]: per window mu0 (> 0), nu0 (> 0), rejects0 (>= 0) and a
                           * skip flag, in place of mu0 / nu0 / rejects0 above, so that each window of a batch resumes
                           * its own earlier run exactly; a window with a nonzero skip flag is left as it is (its
                           * poses unchanged, 0 iterations reported, its other report fields unspecified) */
} ba_lm_options;

typedef struct ba_lm_report {  /* one per window */
    int32_t iters;        /* solves run */
    int32_t n_accepted;
    int32_t converged;    /* ||g|| < tol_g reached */
    int32_t last_info;    /* solve failure of the last step: 0 none, a pivot index + 1, or -1 (dataflow wait gave up) */
    double cost_initial;
    double cost_final;
    double gnorm_final;   /* ||g|| at the last evaluated point */
    double mu_final;      /* damping mu after the last decision */
    int32_t stalled;      /* stopped after max_rejects rejections in a row */
    int32_t rejects_final; /* rejected steps in a row at the end of the call */
    double nu_final;      /* damping growth nu after the last decision: a later call with
                           * mu0 = mu_final, nu0 = nu_final and rejects0 = rejects_final
                           * continues the run exactly (the derivatives are re-evaluated at
                           * the same poses) */
} ba_lm_report;

/* Launch choices of the two evaluation passes.  They change the order in
 * which floating-point partial sums are combined (so results move at the
 * rounding level between settings), never what is computed; for one setting
 * results stay bitwise reproducible. */
typedef struct ba_tuning {
    int32_t vox_split;  /* waves sharing one 64-voxel group in the residual pass: 1, 2 or 4; 0: chosen per
                         * group by its clusters per voxel (1 up to 4, 2 up to 8, 4 beyond) */
    int32_t vox_grid;   /* residual pass: 0 = one block per group; 1..64 = persistent grid of that many blocks per CU */
    int32_t pose_grid;  /* derivative pass: 0 = one wavefront per chunk; 1..64 = persistent, blocks of 4 waves per CU */
    int32_t chunk_len;  /* clusters per derivative-pass chunk, 32..1024 */
} ba_tuning;

/* ---------------------------------------------------------------------- */

/* Text of a status code (static storage). */
const char *ba_status_str(ba_status s);
/* Thread-local description of the last error on this thread. */
const char *ba_last_error(void);

/*
 * ba_build_clusters — Sec. IV-A (L1 clustering and Index Mapper, Alg. 1):
 * group the points by (voxel, scan) with a stable device radix sort, reduce
 * each group into a point cluster (Eq. 2) kept in centred form
 * (N, mu = sum p / N, S = sum (p - mu)(p - mu)^T; compensated sums), and lay
 * out the static plan of the iteration: a voxel-major wave-interleaved copy
 * for the residual pass and a pose-major chunked copy for the derivative
 * pass (the paper's mappers M_v, M_s, built once).
 * pts: host struct of device arrays (not retained).  opt: may be NULL.
 * *out receives a new problem owned by the caller.  Synchronous.
 * Precision form (opt->precision == BA_PREC_F32): the iteration copies hold
 * each cluster as FP32 (N, mu - o, S), where o = R0_j^T (c_i - t0_j) is the
 * voxel's reference point c_i (its FP64 centroid at opt->ref_poses) seen
 * from scan j at its reference pose T0_j; the residual and derivative passes
 * then run their per-cluster arithmetic in FP32 on these voxel-centred
 * coordinates, accumulate in FP64, and keep the 3x3 eigensolve, the solves
 * and the SE(3) update in FP64.  The FP64 clusters stay available to
 * ba_problem_export_clusters.  Needs N_ij < 2^24 (BA_E_UNSUPPORTED).
 * Errors: BA_E_ARG for null pointers, n < 1, labels out of range, non-finite
 * coordinates or windows that a voxel straddles, an unknown precision or a
 * missing/non-finite ref_poses in the precision form; BA_E_NOMEM; BA_E_HIP.
 */
ba_status ba_build_clusters(const ba_points *pts, const ba_build_options *opt, ba_problem **out,
                            hipStream_t stream);

/* Same plan from clusters given as raw sums (Eq. 2); centring is done once
 * in double-double arithmetic.  Errors as above, plus BA_E_ARG for duplicate
 * (voxel, scan) pairs or counts < 1.  Synchronous. */
ba_status ba_build_clusters_from_sums(const ba_cluster_sums *cs, const ba_build_options *opt, ba_problem **out,
                                      hipStream_t stream);

ba_status ba_problem_destroy(ba_problem *p);
ba_status ba_problem_get_info(const ba_problem *p, ba_problem_info *info /* host */);

/* Export the centred clusters sorted by (voxel, scan).  Device outputs of
 * n_clusters entries (mu: 3 per cluster, S: 6 per cluster, AoS).  Any output
 * may be NULL.  Asynchronous. */
ba_status ba_problem_export_clusters(const ba_problem *p, int32_t *voxel, int32_t *scan, double *count,
                                     double *mu, double *S, hipStream_t stream);

/*
 * ba_eval_residual_grad_hessian — Alg. 2, CalRes and CalJH, at poses T:
 *   cost[w]  = sum over voxels of window w of lambda_min(A_i(T))        (Eq. 1)
 *   grad     = d c / d x for every scan (6 per scan)                   (Eq. 3 is tangent to Eq. 1)
 *   hess     = mode BA_MODE_MM: Hessian of the Eq. 3 surrogate, one full
 *              symmetric 6x6 block per scan ([N][36]);
 *              mode BA_MODE_COUPLED: Hessian of u^T A_i(T) u with u frozen
 *              (adds -2 h_j h_k^T pose-pair blocks), one dense row-major
 *              (6 N_w)^2 matrix per window, windows concatenated;
 *              mode BA_MODE_EXACT: the exact Hessian of Eq. 1 in the same
 *              layout (FP64 problems; BA_E_UNSUPPORTED for the precision
 *              form): a diagnostic, e.g. of the gauge null space.
 * poses: device [n_scans][12].  cost: device [n_windows].  grad: device
 * [n_scans][6].  hess: device, layout above (NULL: skip the Hessian and the
 * derivative pass entirely; grad must then be NULL too).  voxel_eig: device
 * [n_voxels_input][4] = (lambda_min, u) per input voxel id, or NULL (voxels
 * without clusters are left untouched).  Asynchronous.
 */
ba_status ba_eval_residual_grad_hessian(ba_problem *p, const double *poses, int32_t mode, double *cost,
                                        double *grad, double *hess, double *voxel_eig, hipStream_t stream);

/* Workspace needed by ba_solve_increment. */
size_t ba_solve_increment_workspace(int32_t mode, int32_t n_scans);

/*
 * ba_solve_increment — Alg. 2, Solver: solve (H + mu D) dx = -g, with
 * D = diag(H) floored at 1e-12 max_k H_kk (reading of "mu Diag(H)", which a
 * scan no voxel constrains would otherwise make singular).
 *   BA_MODE_MM: n_scans independent 6x6 LDL^T factorizations; hess is [N][36].
 *   BA_MODE_COUPLED (or BA_MODE_EXACT): one dense Cholesky of the (6N)^2
 *   row-major hess by 64 x 64 tiles on FP64 matrix cores: up to 6144 rows
 *   in one persistent dataflow launch for the factorization and forward
 *   substitution and one for the back substitution, larger ones blocked
 *   with one launch per step; hess is symmetric and only its lower
 *   triangle is read.
 * hess, grad: device inputs (unchanged).  dx: device [N][6] output.
 * info: device int32 output, 0, the 1-based index of the first
 * non-positive pivot, or -1 if a bounded wait of a dataflow launch gave
 * up (dx is zero unless info is 0).  ws: device workspace of at least
 * ba_solve_increment_workspace(mode, n_scans) bytes.  Asynchronous.
 */
ba_status ba_solve_increment(int32_t mode, int32_t n_scans, const double *hess, const double *grad, double mu,
                             double *dx, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ba_solve_increment_noalloc — for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): ba_solve_increment with its workspace taken from a
 * static device array of BA_STATIC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, so the call allocates nothing.
 * Arguments and results as ba_solve_increment (caller-owned device hess,
 * grad, dx, info; same kernels, bitwise the same results).  Errors:
 * BA_E_WORKSPACE (checked before any device call) when
 * ba_solve_increment_workspace(mode, n_scans) exceeds the static scratch
 * (MM: up to about 20M scans; coupled: up to 6 n_scans ~ 3100, i.e. about
 * 525 scans); BA_E_ARG, BA_E_UNSUPPORTED as ba_solve_increment; BA_E_HIP if
 * the scratch's device address cannot be obtained.  All calls on one GPU
 * share its scratch: calls that overlap on one GPU (concurrent streams) race
 * and must be ordered by the caller.  Asynchronous.
 */
#define BA_STATIC_SCRATCH_BYTES (80 << 20)
ba_status ba_solve_increment_noalloc(int32_t mode, int32_t n_scans, const double *hess, const double *grad,
                                     double mu, double *dx, int32_t *info, hipStream_t stream);

/*
 * ba_iterate — the LM optimizer of Fig. 1 run on the device: per iteration,
 * derivatives at the current poses (when they moved), the damped increment
 * solve, the trial poses T (+) dx, the trial cost (Eq. 1), the gain ratio
 * rho = (c - c_trial) / (-(g^T dx + dx^T H dx / 2)) and the damping update
 * (reading of the unprinted PredResReduction / Adjust: accept when rho > 0,
 * mu <- mu max(1/3, 1 - (2 rho - 1)^3), nu <- 2; otherwise mu <- mu nu,
 * nu <- 2 nu; a failed factorization is a rejected step).  Windows iterate
 * independently.
 * poses_inout: device [n_scans][12], updated in place.  rep: host array of
 * n_windows reports (may be NULL).  trace: host [max_iters][n_windows][8]
 * (cost, cost_trial, rho, mu, accepted, gnorm, info, q) or NULL.
 * The launches of a call are captured once into a HIP graph and replayed
 * by later calls with the same problem, poses pointer and options (set
 * BA_NO_GRAPH=1 in the environment to launch eagerly).
 * Synchronous (returns after the stream has drained).
 */
ba_status ba_iterate(ba_problem *p, double *poses_inout, const ba_lm_options *opt, ba_lm_report *rep,
                     double *trace, hipStream_t stream);

/* Current launch choices of a problem (host output). */
ba_status ba_problem_get_tuning(const ba_problem *p, ba_tuning *t);

/* Set the launch choices (host input; BA_E_ARG outside the ranges above).
 * Re-cuts the derivative-pass chunks when chunk_len changes and drops the
 * problem's captured ba_iterate graph.  Synchronous. */
ba_status ba_problem_set_tuning(ba_problem *p, const ba_tuning *t);

/*
 * ba_autotune — grid search over the launch choices on this problem: every
 * (vox_split, vox_grid) pair of the residual pass and every (chunk_len,
 * pose_grid) pair of the derivative pass is timed with HIP events over
 * `reps` evaluations at `poses` (device [n_scans][12]); the fastest of each
 * pass is applied to the problem and returned in *best (host, may be NULL).
 * Overwrites the problem's voxel state (as an evaluation does).  Synchronous.
 */
ba_status ba_autotune(ba_problem *p, const double *poses, int32_t reps, ba_tuning *best, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/*
 * Served form: a request server that keeps window problems resident on the
 * device while they iterate.  Requests are queued in arrival order; the head
 * of the queue is admitted as soon as a slot is free and its device footprint
 * (ba_request_footprint) fits, together with the requests already admitted,
 * in the budget.  Each slot owns a host thread and a HIP stream: it uploads
 * the request's clusters, builds its problem (ba_build_clusters_from_sums),
 * runs ba_iterate to the options' gradient tolerance or iteration cap, copies
 * the poses back and releases the device memory.  Requests that arrive while
 * others iterate are admitted as slots and memory free up, and their device
 * work overlaps with the running ones.  A request's result does not depend on
 * what else is served (every pass reduces in a fixed order per problem).
 */
typedef struct ba_server ba_server;

typedef struct ba_server_options {
    int64_t hbm_budget;    /* device bytes the admitted requests may reserve together (> 0) */
    int32_t slots;         /* requests on the device at once, 1..64 */
    int32_t precision;     /* BA_PREC_F64 or BA_PREC_F32 (references placed by each request's initial poses) */
    ba_lm_options lm;      /* LM options of every request (mode, max_iters, mu0, nu0, tol_g, max_rejects) */
    int32_t iters_per_check; /* LM iterations between cancellation checks (0: 10); the chunks resume
                              * each other exactly, so results do not depend on it */
    int32_t batch;         /* requests a slot fuses into one multi-window problem (0 or 1: one per problem);
                            * each window of the batch resumes its own run at every chunk, and a request is
                            * finished as soon as its window stops, so results do not depend on it */
} ba_server_options;

typedef struct ba_request {  /* raw-sum clusters of one window (Eq. 2); host arrays, copied on submit */
    int64_t n;
    const int32_t *voxel, *scan;
    const int64_t *count;
    const double *sum, *sumsq;     /* n x 3, n x 6 */
    int32_t n_scans, n_voxels;
    const double *poses_init;      /* n_scans x 12 */
} ba_request;

#define BA_REQ_QUEUED 0
#define BA_REQ_RUNNING 1
#define BA_REQ_DONE 2
#define BA_REQ_FAILED 3
#define BA_REQ_CANCELLED 4

typedef struct ba_request_status {
    int32_t state;         /* BA_REQ_* */
    ba_status status;      /* BA_OK, or the error of a failed request */
    double t_submit, t_admit, t_done;   /* seconds since the server was created (steady clock) */
    int64_t footprint;     /* device bytes reserved for the request */
    ba_lm_report report;
} ba_request_status;

/* Device bytes a request may hold at its peak (build temporaries, the
 * problem, the LM buffers and, in BA_MODE_COUPLED, the dense matrices);
 * an upper bound used for admission.  Host inputs. */
ba_status ba_request_footprint(const ba_request *req, int32_t mode, int32_t precision, int64_t *bytes);

/* Start a server on the current device.  *out receives the handle. */
ba_status ba_server_create(const ba_server_options *opt, ba_server **out);

/* Queue a request (inputs copied; the caller may free them on return).
 * *id receives its id.  BA_E_BUDGET if its footprint exceeds the budget;
 * BA_E_ARG for invalid sizes or labels. */
ba_status ba_server_submit(ba_server *s, const ba_request *req, int64_t *id);

/* Current status of a request (non-blocking; host output). */
ba_status ba_server_query(ba_server *s, int64_t id, ba_request_status *st);

/* Wait until request `id` has finished, copy its poses (host [n_scans][12],
 * may be NULL) and status, and forget the request.  BA_E_NOT_FOUND for an
 * unknown id. */
ba_status ba_server_wait(ba_server *s, int64_t id, double *poses_out, ba_request_status *st);

/* Cancel request `id`: a queued request leaves the queue at once; a running
 * one stops at its next check (every iters_per_check LM iterations) and keeps
 * the poses it reached.  Either way it ends in BA_REQ_CANCELLED and
 * ba_server_wait returns BA_E_CANCELLED with those poses (the initial ones if
 * it never ran).  A request that has already finished is not affected.  The
 * other requests' results do not change.  BA_E_NOT_FOUND for an unknown id. */
ba_status ba_server_cancel(ba_server *s, int64_t id);

/* Finish the running requests, drop the queued ones, stop the slots. */
ba_status ba_server_destroy(ba_server *s);

/*
 * Bottom-up multi-level voxelization and planar voxel selection (Sec. IV-A:
 * Eq. 4-5, Alg. 1 BottomUpVoxelization and Selection).  Turns unlabelled
 * body-frame points into the planar voxels the problem is built from:
 *   1. every point p of scan j is mapped to the world at the given poses,
 *      w = R_j p + t_j, each component evaluated as ((R_r0 p_x + R_r1 p_y) +
 *      R_r2 p_z) + t_r with every product and sum rounded on its own, and
 *      assigned the level-1 cell floor(w / d) per axis (Eq. 4);
 *   2. points of one scan in one cell form a cluster (N, sum p, sum p p^T) in
 *      the scan's body frame (Eq. 2);
 *   3. level k = 2..L halves the cell indices of level k-1 (floor, Eq. 5) and
 *      merges the clusters of one scan that share a parent cell;
 *   4. every cell of every level is tested: its clusters mapped by the poses
 *      give the voxel covariance (Eq. 1) with eigenvalues l0 <= l1 <= l2; the
 *      cell is kept when l0 < tau * l1 (the paper's test), it holds at
 *      least three points and l1 > 1e-10 * l2 (fewer points or a line span no
 *      plane; their l1 is only rounding), and at least min_scans scans observe
 *      it (min_scans is an option beyond the paper's rule; 0 or 1 leaves the
 *      planarity test alone);
 *   5. the kept cells of all levels are concatenated in (level, cell x, cell
 *      y, cell z) order and numbered 0..n_voxels-1 in that order; each keeps
 *      its clusters in scan order.
 * A point contributes to one cell per level, so a kept fine cell and its kept
 * parent both carry it (the multi-resolution features of Sec. IV-A).  The
 * exported clusters are the raw-sum input of ba_build_clusters_from_sums.
 * Sums are formed in a fixed order (bitwise reproducible).
 */
#define BA_VOXEL_MAX_LEVELS 16

typedef struct ba_voxel_map ba_voxel_map;

typedef struct ba_voxelize_options {
    double d;            /* edge of the level-1 cells, > 0 (the minimal resolution of Sec. IV-A) */
    int32_t levels;      /* L, 1..BA_VOXEL_MAX_LEVELS: level k has edge 2^(k-1) d */
    int32_t min_scans;   /* a kept cell is observed by at least this many scans (0 or 1: no requirement) */
    double tau;          /* planarity threshold, > 0: kept when l0 < tau * l1 */
} ba_voxelize_options;

typedef struct ba_voxel_map_info {
    int64_t n_points;
    int64_t n_clusters;   /* exported clusters (those of the kept cells) */
    int32_t n_voxels;     /* kept cells over all levels */
    int32_t levels;
    int32_t n_scans;
    int32_t n_batches;    /* batches of ba_voxelize_host (0 for ba_voxelize) */
    int64_t level_voxels[BA_VOXEL_MAX_LEVELS];         /* cells formed at each level */
    int64_t level_clusters[BA_VOXEL_MAX_LEVELS];       /* (cell, scan) clusters formed at each level */
    int64_t level_kept_voxels[BA_VOXEL_MAX_LEVELS];    /* cells kept at each level */
    int64_t level_kept_clusters[BA_VOXEL_MAX_LEVELS];  /* their clusters */
    int64_t device_bytes;                              /* device memory held by the map */
} ba_voxel_map_info;

/* Voxelize n body-frame points (device x, y, z, scan, length n; 0 <= scan <
 * n_scans) at the poses (device [n_scans][12]).  Synchronous.  On success
 * *out owns the kept clusters in device memory (release with
 * ba_voxel_map_destroy); on error *out is NULL.  Errors: BA_E_ARG (null
 * argument, n outside [1, 2^32), options out of range, a scan id out of
 * range, a non-finite world point or a cell index beyond 2^30 at edge d),
 * BA_E_UNSUPPORTED (the cloud's cell range and scan count need more than 64
 * key bits: use a larger d), BA_E_NOMEM, BA_E_HIP. */
ba_status ba_voxelize(const double *x, const double *y, const double *z, const int32_t *scan, int64_t n,
                      int32_t n_scans, const double *poses, const ba_voxelize_options *opt, ba_voxel_map **out,
                      hipStream_t stream);
/* Adaptive asynchronous loader (Sec. IV-A): the same voxelization for points
 * held in host memory, for clouds larger than device memory.  Device memory is
 * split by the ratio alpha: a point segment sized alpha x (free device memory)
 * holds two batches in flight, the rest holds clusters.  Batch b + 1 is staged
 * (when the host arrays are not pinned: copied into pinned buffers by a few
 * host threads) and transferred on a second stream while batch b is turned
 * into level-1 clusters; all batches' clusters of one (cell, scan) are then
 * merged by one sort (raw sums added in batch order), and the levels,
 * selection and export proceed as in ba_voxelize.  Cells, counts and kept
 * cells equal ba_voxelize's; sums agree to rounding (different addition
 * order).  Synchronous. */
typedef struct ba_stream_options {
    double alpha;           /* share of the free device memory for the point batches, (0, 1]; 0 -> 0.5 */
    int64_t batch_points;   /* points per batch (>= 1024); 0 -> derived from alpha */
} ba_stream_options;

/* x, y, z, scan: host arrays of length n (pinned or pageable); poses: device
 * [n_scans][12]; so may be NULL (defaults).  Errors as ba_voxelize, plus
 * BA_E_ARG for alpha outside (0, 1] or a negative batch size. */
ba_status ba_voxelize_host(const double *x, const double *y, const double *z, const int32_t *scan, int64_t n,
                           int32_t n_scans, const double *poses, const ba_voxelize_options *opt,
                           const ba_stream_options *so, ba_voxel_map **out, hipStream_t stream);
ba_status ba_voxel_map_get_info(const ba_voxel_map *m, ba_voxel_map_info *info);
/* Copy the kept clusters into caller-owned device arrays (any may be NULL to
 * skip it): voxel, scan [n_clusters] int32; count [n_clusters] int64; sum
 * [n_clusters][3] and sumsq [n_clusters][6] f64 (body frame, [xx xy xz yy yz
 * zz]); voxel_level [n_voxels] int32 (1..L); voxel_cell [n_voxels][3] int32
 * (the cell's integer indices at its level).  Clusters are ordered by (voxel,
 * scan).  Asynchronous on the stream. */
ba_status ba_voxel_map_export(const ba_voxel_map *m, int32_t *voxel, int32_t *scan, int64_t *count, double *sum,
                              double *sumsq, int32_t *voxel_level, int32_t *voxel_cell, hipStream_t stream);
ba_status ba_voxel_map_destroy(ba_voxel_map *m);

/*
 * Kernel timing (instrumentation, not part of the method): when enabled,
 * later calls record a pair of HIP events on their stream around each launch
 * of the residual kernel ("k_vox"), the derivative kernel ("k_pose"), the
 * diagonal-block factor ("k_potf2"), the matrix-core factorization kernels
 * ("k_trsm", "k_syrk"), the per-window MM increment solve ("k_window_solve_mm")
 * and the LM decision ("k_decide"); ba_iterate then
 * runs its launches eagerly instead of replaying a captured graph.
 * ba_profile_query waits for the recorded events and returns the summed
 * elapsed time and the launch count of one kernel; ba_profile_reset drops
 * the records.  Process-wide, guarded by a mutex.
 */
ba_status ba_profile_enable(int32_t on);
ba_status ba_profile_reset(void);
ba_status ba_profile_query(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
