// C-ABI entry points of libba (declared in include/ba.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ba.h"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"

namespace ba {
void dense_release(Problem *P);
void graph_release(Problem *P);
bool prof_enabled();
}


ba::Problem::~Problem() {
    graph_release(this);
    dense_release(this);
    delete[] h_win_pose_ptr;
}

namespace ba {

static thread_local char g_last_error[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
}

// dense coupled path (ba_dense.hip)
size_t dense_solve_workspace(int64_t n);
ba_status dense_assemble(Problem *P, const double *poses, double *hess_out, bool use_lm, hipStream_t s);
ba_status dense_assemble_exact(Problem *P, const double *poses, double *hess_out, bool use_lm, double exact_below,
                               hipStream_t s);
ba_status dense_solve(int64_t n, const double *A, const double *g, double mu, double *dx, int32_t *info, void *ws,
                      size_t ws_bytes, hipStream_t s);
ba_status dense_lm_step(Problem *P, const double *poses, double tol_g, hipStream_t s);
void launch_dense_gnorm(Problem *P, hipStream_t s, double tol_g = 0.0);
void dense_release(Problem *P);
ba_status dense_prepare(Problem *P);

// ---------------------------------------------------------------- profiling
// Event pairs recorded around kernel launches (eager launches only: a call
// made while profiling is enabled is not captured into a graph).  Elapsed
// times are summed per kernel name when queried.
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
static bool g_prof_on = false;
static std::vector<ProfRec> g_pending;
static std::vector<hipEvent_t> g_prof_pool;
static std::map<std::string, std::pair<double, int64_t>> g_prof_tot;
static std::mutex g_prof_mu;

static hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool prof_enabled() { return g_prof_on; }

void prof_begin(const char *name, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r;
    r.name = name;
    r.a = prof_event();
    r.b = prof_event();
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, s);
    g_pending.push_back(r);
}

void prof_end(hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_pending.empty()) (void)hipEventRecord(g_pending.back().b, s);
}

static void prof_add(const std::vector<ProfRec> &l) {
    for (const ProfRec &r : l) {
        if (hipEventSynchronize(r.b) != hipSuccess) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        auto &t = g_prof_tot[r.name];
        t.first += ms;
        t.second += 1;
    }
    (void)hipGetLastError();
}

// fold the eager records into the totals and recycle their events
static void prof_collect_pending() {
    prof_add(g_pending);
    for (auto &r : g_pending) {
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_pending.clear();
}


}  // namespace ba

using namespace ba;

namespace ba {

// Enqueue every launch of one ba_iterate call (stream-ordered, no host sync).
static ba_status enqueue_lm(Problem *P, double *poses, const ba_lm_options *opt, double *dtrace, double mu0, double nu0,
                            hipStream_t s) {
    const int iters = opt->max_iters;
    launch_lm_reset(P, mu0, nu0, opt->rejects0, opt->resume ? P->lm_init : nullptr, s);
    launch_vox(P, poses, true, false, s);
    launch_lm_cost(P, s);
    for (int it = 0; it < iters; it++) {
        if (opt->mode == BA_MODE_MM) {
            launch_pose_derivs(P, poses, true, P->g, P->H, s);
            launch_window_solve_mm(P, poses, opt->tol_g, s);
        } else {
            launch_pose_derivs(P, poses, true, P->g, P->H, s, true);
            if (opt->exact_below > 0.0) {
                // near convergence the exact Hessian: the switch reads the
                // gradient norm at the poses the matrix is built at
                launch_dense_gnorm(P, s);
                BA_TRY(dense_assemble_exact(P, poses, nullptr, true, opt->exact_below, s));
            } else {
                BA_TRY(dense_assemble(P, poses, nullptr, true, s));
            }
            BA_TRY(dense_lm_step(P, poses, opt->tol_g, s));
        }
        // trial residual, then the per-window decision and commit
        launch_vox(P, P->poses_trial, true, true, s);
        launch_decide(P, dtrace, it, poses, s, opt->max_rejects);
    }
    // derivatives at the final poses (windows whose last step was accepted),
    // so that the reported gradient norm belongs to the returned poses
    launch_pose_derivs(P, poses, true, P->g, P->H, s, opt->mode == BA_MODE_COUPLED);
    // the reported norm and convergence flag in the order the mode's in-loop
    // test forms them, so the two agree bitwise
    if (opt->mode == BA_MODE_MM) {
        launch_window_stats(P, opt->tol_g, s);
    } else {
        BA_TRY(dense_prepare(P));
        launch_dense_gnorm(P, s, opt->tol_g);
    }
    BA_HIP(hipGetLastError());
    return BA_OK;
}

struct IterGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    // key
    double *poses = nullptr, *trace = nullptr;
    int32_t mode = -1, iters = -1, tune_gen = -1, max_rejects = 0, rejects0 = 0;
    double mu0 = 0, nu0 = 0, tol_g = 0, exact_below = 0;
    bool per_window = false;   // start from P->lm_init (filled before each launch)
    ~IterGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

void graph_release(Problem *P) {
    delete (IterGraph *)P->iter_graph;
    P->iter_graph = nullptr;
}

static bool g_graphs_enabled() {
    const char *e = getenv("BA_NO_GRAPH");
    return !(e && e[0] == '1');
}

}  // namespace ba

extern "C" {

const char *ba_status_str(ba_status s) {
    switch (s) {
        case BA_OK: return "ok";
        case BA_E_ARG: return "invalid argument";
        case BA_E_WORKSPACE: return "workspace too small";
        case BA_E_HIP: return "HIP runtime error";
        case BA_E_NOT_SPD: return "matrix not positive definite";
        case BA_E_UNSUPPORTED: return "unsupported";
        case BA_E_NOMEM: return "out of device memory";
        case BA_E_BUDGET: return "request exceeds the device-memory budget";
        case BA_E_NOT_FOUND: return "unknown request";
        case BA_E_CANCELLED: return "request cancelled";
        default: return "unknown status";
    }
}

const char *ba_last_error(void) { return g_last_error; }

ba_status ba_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return BA_OK;
}

ba_status ba_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_collect_pending();
    g_prof_tot.clear();
    return BA_OK;
}

ba_status ba_profile_query(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel || !total_ms || !launches) {
        set_error("null argument to ba_profile_query");
        return BA_E_ARG;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_collect_pending();
    auto it = g_prof_tot.find(kernel);
    *total_ms = (it == g_prof_tot.end()) ? 0.0 : it->second.first;
    *launches = (it == g_prof_tot.end()) ? 0 : it->second.second;
    return BA_OK;
}

static ba_status build_common(ba_problem **out, hipStream_t stream,
                              ba_status (*fn)(const void *, const ba_build_options *, Problem *, DevArena &,
                                              hipStream_t),
                              const void *src, const ba_build_options *opt) {
    if (!out) {
        set_error("out is null");
        return BA_E_ARG;
    }
    *out = nullptr;
    if (opt && opt->n_windows > 1 && !opt->scan_window) {
        set_error("n_windows > 1 needs scan_window");
        return BA_E_ARG;
    }
    ba_problem *p = new (std::nothrow) ba_problem();
    if (!p) {
        set_error("host allocation failed");
        return BA_E_NOMEM;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete p;
        set_error("no HIP device");
        return BA_E_HIP;
    }
    p->P.device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        p->P.n_cu = ncu;
    ba_status st = fn(src, opt, &p->P, p->P.mem, stream);
    if (st != BA_OK) {
        (void)hipStreamSynchronize(stream);
        delete p;
        return st;
    }
    *out = p;
    return BA_OK;
}

static ba_status fn_points(const void *src, const ba_build_options *opt, Problem *P, DevArena &keep, hipStream_t s) {
    const ba_points *pts = (const ba_points *)src;
    P->n_points = pts->n;
    return build_from_points(pts, opt, P, keep, s);
}

static ba_status fn_sums(const void *src, const ba_build_options *opt, Problem *P, DevArena &keep, hipStream_t s) {
    return build_from_sums((const ba_cluster_sums *)src, opt, P, keep, s);
}

ba_status ba_build_clusters(const ba_points *pts, const ba_build_options *opt, ba_problem **out, hipStream_t stream) {
    if (!pts) {
        set_error("pts is null");
        return BA_E_ARG;
    }
    return build_common(out, stream, fn_points, pts, opt);
}

ba_status ba_build_clusters_from_sums(const ba_cluster_sums *cs, const ba_build_options *opt, ba_problem **out,
                                      hipStream_t stream) {
    if (!cs) {
        set_error("cs is null");
        return BA_E_ARG;
    }
    return build_common(out, stream, fn_sums, cs, opt);
}

ba_status ba_problem_destroy(ba_problem *p) {
    if (!p) return BA_OK;
    (void)hipDeviceSynchronize();
    delete p;
    return BA_OK;
}

ba_status ba_problem_get_info(const ba_problem *p, ba_problem_info *info) {
    if (!p || !info) {
        set_error("null argument");
        return BA_E_ARG;
    }
    const Problem &P = p->P;
    info->n_points = P.n_points;
    info->n_clusters = P.n_clusters;
    info->n_voxels = P.n_vox;
    info->n_scans = P.n_poses;
    info->n_windows = P.n_windows;
    info->max_m = P.max_m;
    info->device_bytes = (int64_t)P.mem.bytes + dense_device_bytes(&P);
    info->n_wave_groups = P.n_groups;
    info->n_pose_chunks = P.n_chunks;
    info->padded_clusters = P.c_pad;
    info->precision = P.prec;
    info->cluster_bytes = P.prec == BA_PREC_F32 ? 4 + 12 + 24 + 4 : 8 + 24 + 48 + 4;
    return BA_OK;
}

ba_status ba_problem_export_clusters(const ba_problem *p, int32_t *voxel, int32_t *scan, double *count, double *mu,
                                     double *S, hipStream_t stream) {
    if (!p) {
        set_error("null problem");
        return BA_E_ARG;
    }
    const Problem &P = p->P;
    const int64_t C = P.n_clusters;
    if (voxel) BA_HIP(hipMemcpyAsync(voxel, P.c_vox, sizeof(int32_t) * C, hipMemcpyDeviceToDevice, stream));
    if (scan) BA_HIP(hipMemcpyAsync(scan, P.c_scan, sizeof(int32_t) * C, hipMemcpyDeviceToDevice, stream));
    if (count) BA_HIP(hipMemcpyAsync(count, P.c_N, sizeof(double) * C, hipMemcpyDeviceToDevice, stream));
    if (mu) BA_HIP(hipMemcpyAsync(mu, P.c_mu, sizeof(double) * 3 * C, hipMemcpyDeviceToDevice, stream));
    if (S) BA_HIP(hipMemcpyAsync(S, P.c_S, sizeof(double) * 6 * C, hipMemcpyDeviceToDevice, stream));
    return BA_OK;
}

ba_status ba_eval_residual_grad_hessian(ba_problem *p, const double *poses, int32_t mode, double *cost, double *grad,
                                        double *hess, double *voxel_eig, hipStream_t stream) {
    if (!p || !poses || !cost) {
        set_error("null problem, poses or cost");
        return BA_E_ARG;
    }
    if (mode != BA_MODE_MM && mode != BA_MODE_COUPLED && mode != BA_MODE_EXACT) {
        set_error("unknown mode %d", mode);
        return BA_E_UNSUPPORTED;
    }
    if ((grad == nullptr) != (hess == nullptr)) {
        set_error("grad and hess must both be given or both be null");
        return BA_E_ARG;
    }
    Problem *P = &p->P;
    launch_vox(P, poses, false, false, stream);
    launch_window_cost(P, cost, stream);
    if (voxel_eig) launch_voxel_eig(P, voxel_eig, stream);
    if (grad) {
        double *Hmm = (mode == BA_MODE_MM) ? hess : P->H;
        if (mode == BA_MODE_EXACT && P->prec != BA_PREC_F64) {
            set_error("the exact Hessian is built for FP64 problems only");
            return BA_E_UNSUPPORTED;
        }
        if (mode != BA_MODE_MM) BA_TRY(dense_prepare(P));   // the derivative pass may fill its h vectors
        launch_pose_derivs(P, poses, false, grad, Hmm, stream, mode == BA_MODE_COUPLED);
        if (mode == BA_MODE_COUPLED) BA_TRY(dense_assemble(P, poses, hess, false, stream));
        if (mode == BA_MODE_EXACT) BA_TRY(dense_assemble_exact(P, poses, hess, false, 0.0, stream));
    }
    BA_HIP(hipGetLastError());
    return BA_OK;
}

size_t ba_solve_increment_workspace(int32_t mode, int32_t n_scans) {
    if (n_scans < 1) return 0;
    if (mode == BA_MODE_MM) return solve_mm_workspace(n_scans);
    if (mode == BA_MODE_COUPLED || mode == BA_MODE_EXACT) return dense_solve_workspace(6LL * n_scans);
    return 0;
}

ba_status ba_solve_increment(int32_t mode, int32_t n_scans, const double *hess, const double *grad, double mu,
                             double *dx, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (n_scans < 1 || !hess || !grad || !dx || !info || !(mu >= 0.0) || !std::isfinite(mu)) {
        set_error("invalid argument to ba_solve_increment");
        return BA_E_ARG;
    }
    const size_t need = ba_solve_increment_workspace(mode, n_scans);
    if (mode != BA_MODE_MM && mode != BA_MODE_COUPLED && mode != BA_MODE_EXACT) {
        set_error("unknown mode %d", mode);
        return BA_E_UNSUPPORTED;
    }
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
        return BA_E_WORKSPACE;
    }
    if (mode == BA_MODE_MM) {
        launch_solve_mm_plain(n_scans, hess, grad, mu, dx, info, ws, stream);
        BA_HIP(hipGetLastError());
        return BA_OK;
    }
    return dense_solve(6LL * n_scans, hess, grad, mu, dx, info, ws, ws_bytes, stream);
}

ba_status ba_iterate(ba_problem *p, double *poses_inout, const ba_lm_options *opt, ba_lm_report *rep, double *trace,
                     hipStream_t stream) {
    if (!p || !poses_inout || !opt) {
        set_error("null argument to ba_iterate");
        return BA_E_ARG;
    }
    if (opt->mode != BA_MODE_MM && opt->mode != BA_MODE_COUPLED) {
        set_error("unknown mode %d", opt->mode);
        return BA_E_UNSUPPORTED;
    }
    if (opt->max_iters < 0 || opt->rejects0 < 0) {
        set_error("max_iters < 0 or rejects0 < 0");
        return BA_E_ARG;
    }
    Problem *P = &p->P;
    if (opt->exact_below > 0.0 && (opt->mode != BA_MODE_COUPLED || P->prec != BA_PREC_F64)) {
        set_error("exact_below needs the coupled mode on an FP64 problem");
        return BA_E_UNSUPPORTED;
    }
    const int W = P->n_windows;
    const int iters = opt->max_iters;
    const double mu0 = opt->mu0 > 0 ? opt->mu0 : 1e-2;
    const double nu0 = opt->nu0 > 0 ? opt->nu0 : 2.0;
    if (opt->resume) {
        for (int w = 0; w < W; w++) {
            const double *r = opt->resume + 4 * w;
            if (!(r[0] > 0.0) || !(r[1] > 0.0) || !(r[2] >= 0.0) || r[2] > 2147483647.0 || r[2] != (double)(int32_t)r[2]) {
                set_error("resume entry of window %d out of range (mu0 %g, nu0 %g, rejects0 %g)", w, r[0], r[1], r[2]);
                return BA_E_ARG;
            }
        }
        if (!P->lm_init) BA_TRY(P->mem.alloc(&P->lm_init, 4LL * W));
        BA_HIP(hipMemcpyAsync(P->lm_init, opt->resume, sizeof(double) * 4 * W, hipMemcpyHostToDevice, stream));
    }
    if (opt->mode == BA_MODE_COUPLED) BA_TRY(dense_prepare(P));
    double *dtrace = nullptr;
    if (trace && iters > 0) {
        if (P->trace_cap < iters) {
            BA_TRY(P->mem.alloc(&P->trace, (int64_t)iters * W * 8));
            P->trace_cap = iters;
        }
        dtrace = P->trace;
    }
    // The whole call is captured once into a HIP graph and replayed while its
    // arguments stay the same (profiling records events, so it runs eagerly).
    bool done = false;
    if (g_graphs_enabled() && !prof_enabled() && !P->no_graph) {   // event records cannot be captured: profile eagerly
        IterGraph *G = (IterGraph *)P->iter_graph;
        const bool same = G && G->exec && G->poses == poses_inout && G->trace == dtrace && G->mode == opt->mode &&
                          G->iters == iters && G->mu0 == mu0 && G->nu0 == nu0 && G->tol_g == opt->tol_g &&
                          G->tune_gen == P->tune_gen && G->max_rejects == opt->max_rejects &&
                          G->rejects0 == opt->rejects0 && G->per_window == (opt->resume != nullptr) &&
                          G->exact_below == opt->exact_below;
        if (!same) {
            graph_release(P);
            G = new IterGraph();
            P->iter_graph = G;
            hipGraph_t graph = nullptr;
            bool ok = hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking) == hipSuccess &&
                      hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                ba_status st = enqueue_lm(P, poses_inout, opt, dtrace, mu0, nu0, G->cap);
                hipError_t e = hipStreamEndCapture(G->cap, &graph);
                ok = (st == BA_OK) && e == hipSuccess && graph &&
                     hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0) == hipSuccess;
            }
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (ok) {
                G->poses = poses_inout;
                G->trace = dtrace;
                G->mode = opt->mode;
                G->iters = iters;
                G->mu0 = mu0;
                G->nu0 = nu0;
                G->tol_g = opt->tol_g;
                G->tune_gen = P->tune_gen;
                G->max_rejects = opt->max_rejects;
                G->rejects0 = opt->rejects0;
                G->per_window = opt->resume != nullptr;
                G->exact_below = opt->exact_below;
            } else {
                graph_release(P);
                G = nullptr;
            }
        }
        if (G && G->exec) {
            BA_HIP(hipGraphLaunch(G->exec, stream));
            done = true;
        }
    }
    if (!done) BA_TRY(enqueue_lm(P, poses_inout, opt, dtrace, mu0, nu0, stream));
    std::vector<LMState> st(W);
    BA_HIP(hipMemcpyAsync(st.data(), P->lm, sizeof(LMState) * W, hipMemcpyDeviceToHost, stream));
    if (dtrace) BA_HIP(hipMemcpyAsync(trace, dtrace, sizeof(double) * (size_t)iters * W * 8, hipMemcpyDeviceToHost, stream));
    BA_HIP(hipStreamSynchronize(stream));
    if (rep) {
        for (int w = 0; w < W; w++) {
            rep[w].iters = st[w].iters;
            rep[w].n_accepted = st[w].n_accepted;
            rep[w].converged = st[w].done == 1;
            rep[w].stalled = st[w].done == 2;
            rep[w].rejects_final = st[w].rejects;
            rep[w].last_info = st[w].info;
            rep[w].cost_final = st[w].cost;
            rep[w].gnorm_final = st[w].gnorm;
            rep[w].mu_final = st[w].mu;
            rep[w].nu_final = st[w].nu;
            rep[w].cost_initial = st[w].cost0;
        }
    }
    return BA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- tuning
namespace ba {

static ba_status check_tuning(const ba_tuning *t) {
    if (!(t->vox_split == 0 || t->vox_split == 1 || t->vox_split == 2 || t->vox_split == 4) || t->vox_grid < 0 ||
        t->vox_grid > 64 ||
        t->pose_grid < 0 || t->pose_grid > 64 || t->chunk_len < MIN_CHUNK || t->chunk_len > MAX_CHUNK) {
        set_error("tuning out of range (vox_split %d, vox_grid %d, pose_grid %d, chunk_len %d)", t->vox_split,
                  t->vox_grid, t->pose_grid, t->chunk_len);
        return BA_E_ARG;
    }
    return BA_OK;
}

static ba_status apply_tuning(Problem *P, const ba_tuning *t, hipStream_t s) {
    BA_TRY(check_tuning(t));
    if (t->chunk_len != P->tune.chunk_len) BA_TRY(replan_chunks(P, t->chunk_len, s));
    P->tune.vox_split = t->vox_split;
    P->tune.vox_grid = t->vox_grid;
    P->tune.pose_grid = t->pose_grid;
    P->tune_gen++;
    graph_release(P);
    return BA_OK;
}

static ba_tuning export_tuning(const Problem *P) {
    ba_tuning t;
    t.vox_split = P->tune.vox_split;
    t.vox_grid = P->tune.vox_grid;
    t.pose_grid = P->tune.pose_grid;
    t.chunk_len = P->tune.chunk_len;
    return t;
}

// Mean time of `reps` launches of one pass (after one untimed launch).
static ba_status time_pass(Problem *P, const double *poses, bool vox, int reps, hipStream_t s, float *ms) {
    hipEvent_t a, b;
    BA_HIP(hipEventCreate(&a));
    BA_HIP(hipEventCreate(&b));
    auto launch = [&]() {
        if (vox)
            launch_vox(P, poses, false, false, s);
        else
            launch_pose_chunks(P, poses, false, s);
    };
    launch();
    hipError_t e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; r++) launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipGetLastError();
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        set_error("autotune timing failed: %s", hipGetErrorString(e));
        return BA_E_HIP;
    }
    *ms = t / (float)std::max(reps, 1);
    return BA_OK;
}

}  // namespace ba

extern "C" {

ba_status ba_problem_get_tuning(const ba_problem *p, ba_tuning *t) {
    if (!p || !t) {
        ba::set_error("null argument");
        return BA_E_ARG;
    }
    *t = ba::export_tuning(&p->P);
    return BA_OK;
}

ba_status ba_problem_set_tuning(ba_problem *p, const ba_tuning *t) {
    if (!p || !t) {
        ba::set_error("null argument");
        return BA_E_ARG;
    }
    return ba::apply_tuning(&p->P, t, 0);
}

ba_status ba_autotune(ba_problem *p, const double *poses, int32_t reps, ba_tuning *best, hipStream_t stream) {
    using namespace ba;
    if (!p || !poses || reps < 1) {
        set_error("null problem or poses, or reps < 1");
        return BA_E_ARG;
    }
    Problem *P = &p->P;
    ba_tuning cur = export_tuning(P);
    // residual pass: cluster split x grid
    const int splits[4] = {4, 2, 1, 0};
    const int vgrids[5] = {0, 1, 2, 4, 8};
    float best_ms = 1e30f;
    ba_tuning t = cur, win = cur;
    for (int sp : splits)
        for (int gr : vgrids) {
            t.vox_split = sp;
            t.vox_grid = gr;
            BA_TRY(apply_tuning(P, &t, stream));
            float ms = 0.f;
            BA_TRY(time_pass(P, poses, true, reps, stream, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                win.vox_split = sp;
                win.vox_grid = gr;
            }
        }
    t = win;
    BA_TRY(apply_tuning(P, &t, stream));
    // the derivative pass reads the voxel state of the residual pass
    launch_vox(P, poses, false, false, stream);
    const int chunks[5] = {256, 64, 128, 512, 1024};
    const int pgrids[4] = {0, 2, 4, 8};
    best_ms = 1e30f;
    for (int cl : chunks)
        for (int gr : pgrids) {
            t.chunk_len = cl;
            t.pose_grid = gr;
            BA_TRY(apply_tuning(P, &t, stream));
            float ms = 0.f;
            BA_TRY(time_pass(P, poses, false, reps, stream, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                win.chunk_len = cl;
                win.pose_grid = gr;
            }
        }
    BA_TRY(apply_tuning(P, &win, stream));
    if (best) *best = win;
    return BA_OK;
}

}  // extern "C"
