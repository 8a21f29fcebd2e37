// Served form: a request server over libba's problems (see include/ba.h).
//
// A FIFO queue of requests (host copies of their raw-sum clusters), a pool of
// slots (one host thread and one HIP stream each) and a device-memory budget.
// A free slot admits the head of the queue once its footprint fits next to
// the requests already admitted; it then builds the request's problem on its
// stream, runs the LM iteration, copies the poses out and releases the
// problem.  Slots run concurrently, so requests that arrive while others
// iterate start as soon as a slot and memory are free and their kernels
// overlap on the device with the running ones.
//
// Each slot keeps one device block (a slot arena, at most budget / slots
// bytes) that a request's build and LM buffers are carved from; it grows to
// the largest request the slot has served, so a steady request stream does
// no device allocation or release (hipFree synchronises the whole device).
// The LM runs in chunks of iters_per_check iterations, each resuming the last
// exactly (damping, damping growth and rejection count carried over), so a
// cancelled request stops at the next chunk boundary while the results of
// uncancelled ones are those of one uninterrupted run.
//
// With opt.batch > 1 a free slot admits up to that many queued requests (in
// queue order, while they fit the budget) and fuses them into one problem of
// independent windows: one launch per pass then serves all of them.  The LM
// runs in chunks with every window resuming its own run (per-window damping,
// growth and rejection count); a request is finished as soon as its window
// converges, stalls, uses its iterations or is cancelled, and its window is
// skipped from then on.  A window's arithmetic does not depend on the other
// windows of its problem, so every result equals the request's result alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ba.h"
#include "ba_internal.hpp"

namespace ba {

struct Request {
    int64_t id = 0;
    int64_t n = 0;
    int32_t n_scans = 0, n_voxels = 0;
    std::vector<int32_t> voxel, scan;
    std::vector<int64_t> count;
    std::vector<double> sum, sumsq, poses;   // poses: initial, then the result
    int64_t footprint = 0;
    ba_request_status st{};
    std::string error;   // text of a failure, handed to the waiting thread
    std::atomic<bool> cancel{false};
};

struct Server {
    ba_server_options opt{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // queue / budget / completion changes
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> all;
    int64_t next_id = 1;
    int64_t reserved = 0;
    bool stopping = false;
    std::vector<std::thread> slots;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Upper bound of the device bytes of one request (see ba_request_footprint).
static int64_t footprint_bytes(int64_t C, int64_t V, int64_t N, int32_t mode, int32_t prec) {
    // padding of the wave-interleaved copy: at most 63 slots per group of 64
    // voxels, each holding up to max_m clusters; bounded by 1/2 of C here
    const double cp = 1.5 * (double)C;
    const double ns = (double)V + 64.0 * ((double)V / 64.0 + 1.0);
    double b = 0.0;
    b += 40.0 * C;                                  // sort keys, values and workspace of the build
    b += 92.0 * C;                                  // centred clusters kept for export + slot
    b += (prec == BA_PREC_F32 ? (44.0 + 84.0) : 84.0) * cp;   // voxel-major copy (FP64 temporary in FP32 form)
    b += (prec == BA_PREC_F32 ? 44.0 : 84.0) * C;   // pose-major copy
    b += 16.0 * C + 8.0 * C;                        // scatter / gather tables of the build
    b += (16.0 + 27.0 * 8.0) * ((double)C / MIN_CHUNK + N + 1);   // chunk tables and partials
    b += ns * (2.0 * VSTATE * 8.0 + 4.0 + 32.0 + 8.0);            // voxel state, slot map, references, costs
    b += (double)N * (48.0 + 288.0 + 48.0 + 96.0 + 8.0 + 4.0 + 96.0 + 16.0);
    if (mode == BA_MODE_COUPLED) {
        const double n6 = 6.0 * (double)N;
        b += 8.0 * C * 10.0 + 48.0 * C;             // pose-pair lists (<= 10 pairs per cluster here) and h vectors
        b += 40.0 * C * 10.0;                       // the pair plan's sort keys, values and workspace (build time)
        b += 3.0 * n6 * n6 * 8.0;                   // the dense matrix and the factorization buffers
    }
    return (int64_t)(1.25 * b) + (16LL << 20);
}

static ba_status validate_request(const ba_request *r) {
    if (!r || r->n < 1 || r->n_scans < 1 || r->n_voxels < 1 || !r->voxel || !r->scan || !r->count || !r->sum ||
        !r->sumsq || !r->poses_init) {
        set_error("invalid request: null array or empty sizes");
        return BA_E_ARG;
    }
    return BA_OK;
}

// The LM of one request in chunks of opt.iters_per_check iterations, each
// resuming the previous one exactly; stops early once the request is
// cancelled, converged or stalled.  `rep` receives the whole run's report.
static ba_status run_lm_chunked(Server *S, Request &R, ba_problem *p, double *d_poses, ba_lm_report &rep,
                                bool &cancelled, hipStream_t stream) {
    ba_lm_options o = S->opt.lm;
    const int chunk = S->opt.iters_per_check > 0 ? S->opt.iters_per_check : 10;
    int left = o.max_iters;
    bool first = true;
    std::memset(&rep, 0, sizeof(rep));
    cancelled = false;
    while (left > 0) {
        if (R.cancel.load()) {
            cancelled = true;
            break;
        }
        o.max_iters = std::min(chunk, left);
        ba_lm_report r{};
        BA_TRY(ba_iterate(p, d_poses, &o, &r, nullptr, stream));
        if (first) rep.cost_initial = r.cost_initial;
        first = false;
        rep.iters += r.iters;
        rep.n_accepted += r.n_accepted;
        rep.converged = r.converged;
        rep.stalled = r.stalled;
        rep.last_info = r.last_info;
        rep.cost_final = r.cost_final;
        rep.gnorm_final = r.gnorm_final;
        rep.mu_final = r.mu_final;
        rep.nu_final = r.nu_final;
        rep.rejects_final = r.rejects_final;
        if (r.converged || r.stalled || r.iters < o.max_iters) break;
        left -= r.iters;
        o.mu0 = r.mu_final;
        o.nu0 = r.nu_final;
        o.rejects0 = r.rejects_final;
    }
    return BA_OK;
}

// One request, start to finish, on `stream`.
static ba_status run_request(Server *S, Request &R, hipStream_t stream, bool &cancelled) {
    const int64_t n = R.n;
    DevArena in;
    int32_t *d_vox, *d_scan;
    int64_t *d_cnt;
    double *d_sum, *d_sq, *d_poses;
    BA_TRY(in.alloc(&d_vox, n));
    BA_TRY(in.alloc(&d_scan, n));
    BA_TRY(in.alloc(&d_cnt, n));
    BA_TRY(in.alloc(&d_sum, 3 * n));
    BA_TRY(in.alloc(&d_sq, 6 * n));
    BA_TRY(in.alloc(&d_poses, 12LL * R.n_scans));
    BA_HIP(hipMemcpyAsync(d_vox, R.voxel.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_scan, R.scan.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_cnt, R.count.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_sum, R.sum.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_sq, R.sumsq.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_poses, R.poses.data(), sizeof(double) * 12 * R.n_scans, hipMemcpyHostToDevice, stream));
    ba_cluster_sums cs;
    cs.n = n;
    cs.voxel = d_vox;
    cs.scan = d_scan;
    cs.count = d_cnt;
    cs.sum = d_sum;
    cs.sumsq = d_sq;
    cs.n_scans = R.n_scans;
    cs.n_voxels = R.n_voxels;
    ba_build_options bo;
    std::memset(&bo, 0, sizeof(bo));
    bo.precision = S->opt.precision;
    bo.ref_poses = S->opt.precision == BA_PREC_F32 ? d_poses : nullptr;
    ba_problem *p = nullptr;
    BA_TRY(ba_build_clusters_from_sums(&cs, &bo, &p, stream));
    std::unique_ptr<ba_problem> own(p);
    p->P.no_graph = true;   // one-shot problem: launch eagerly rather than capture
    ba_lm_report rep{};
    ba_status st = run_lm_chunked(S, R, p, d_poses, rep, cancelled, stream);
    if (st == BA_OK) {
        R.st.report = rep;
        hipError_t e = hipMemcpyAsync(R.poses.data(), d_poses, sizeof(double) * 12 * R.n_scans,
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("copy of served poses failed: %s", hipGetErrorString(e));
            st = BA_E_HIP;
        }
    }
    (void)hipStreamSynchronize(stream);
    return st;
}

// Grows the slot's arena to hold a request of `need` bytes (never beyond the
// slot's share of the budget; larger requests allocate directly).
static void arena_reserve(Server *S, SlotArena &a, int64_t need) {
    const int64_t share = S->opt.hbm_budget / S->opt.slots;
    if ((int64_t)a.cap >= need || need > share) return;
    if (a.base) (void)hipFree(a.base);
    a.base = nullptr;
    a.cap = 0;
    void *q = nullptr;
    if (hipMalloc(&q, (size_t)need) == hipSuccess) {
        a.base = (char *)q;
        a.cap = (size_t)need;
    } else {
        (void)hipGetLastError();   // this request allocates directly instead
    }
}

// Marks a request finished (under the server lock) and drops its input copies.
static void finish_request(Server *S, Request &R, ba_status st, bool cancelled, const std::string &err) {
    std::lock_guard<std::mutex> lk(S->mu);
    R.error = err;
    R.st.status = cancelled ? BA_E_CANCELLED : st;
    R.st.state = cancelled ? BA_REQ_CANCELLED : (st == BA_OK ? BA_REQ_DONE : BA_REQ_FAILED);
    R.st.t_done = S->now();
    std::vector<int32_t>().swap(R.voxel);
    std::vector<int32_t>().swap(R.scan);
    std::vector<int64_t>().swap(R.count);
    std::vector<double>().swap(R.sum);
    std::vector<double>().swap(R.sumsq);
}

// Several requests as the windows of one problem, on `stream` (see above).
// Each request is finished (finish_request) as soon as its window stops;
// returns a status for the requests still open when the problem fails.
static ba_status run_batch(Server *S, std::vector<std::shared_ptr<Request>> &B, hipStream_t stream) {
    const int W = (int)B.size();
    int64_t n = 0;
    int32_t ns = 0, nv = 0;
    for (auto &R : B) {
        n += R->n;
        ns += R->n_scans;
        nv += R->n_voxels;
    }
    // concatenated inputs: voxel and scan ids shifted per request, one window per request
    std::vector<int32_t> vox(n), scan(n), win(ns);
    std::vector<int64_t> cnt(n);
    std::vector<double> sum(3 * n), sq(6 * n), poses(12LL * ns);
    std::vector<int32_t> s0(W + 1, 0);
    {
        int64_t o = 0;
        int32_t so = 0, vo = 0;
        for (int w = 0; w < W; w++) {
            const Request &R = *B[w];
            for (int64_t i = 0; i < R.n; i++) {
                vox[o + i] = R.voxel[i] + vo;
                scan[o + i] = R.scan[i] + so;
            }
            std::copy(R.count.begin(), R.count.end(), cnt.begin() + o);
            std::copy(R.sum.begin(), R.sum.end(), sum.begin() + 3 * o);
            std::copy(R.sumsq.begin(), R.sumsq.end(), sq.begin() + 6 * o);
            std::copy(R.poses.begin(), R.poses.end(), poses.begin() + 12LL * so);
            for (int32_t j = 0; j < R.n_scans; j++) win[so + j] = w;
            s0[w] = so;
            o += R.n;
            so += R.n_scans;
            vo += R.n_voxels;
        }
        s0[W] = so;
    }
    DevArena in;
    int32_t *d_vox, *d_scan;
    int64_t *d_cnt;
    double *d_sum, *d_sq, *d_poses;
    BA_TRY(in.alloc(&d_vox, n));
    BA_TRY(in.alloc(&d_scan, n));
    BA_TRY(in.alloc(&d_cnt, n));
    BA_TRY(in.alloc(&d_sum, 3 * n));
    BA_TRY(in.alloc(&d_sq, 6 * n));
    BA_TRY(in.alloc(&d_poses, 12LL * ns));
    BA_HIP(hipMemcpyAsync(d_vox, vox.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_scan, scan.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_cnt, cnt.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_sum, sum.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_sq, sq.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice, stream));
    BA_HIP(hipMemcpyAsync(d_poses, poses.data(), sizeof(double) * 12 * ns, hipMemcpyHostToDevice, stream));
    ba_cluster_sums cs;
    cs.n = n;
    cs.voxel = d_vox;
    cs.scan = d_scan;
    cs.count = d_cnt;
    cs.sum = d_sum;
    cs.sumsq = d_sq;
    cs.n_scans = ns;
    cs.n_voxels = nv;
    ba_build_options bo;
    std::memset(&bo, 0, sizeof(bo));
    bo.n_windows = W;
    bo.scan_window = win.data();
    bo.precision = S->opt.precision;
    bo.ref_poses = S->opt.precision == BA_PREC_F32 ? d_poses : nullptr;
    ba_problem *p = nullptr;
    BA_TRY(ba_build_clusters_from_sums(&cs, &bo, &p, stream));
    std::unique_ptr<ba_problem> own(p);
    p->P.no_graph = true;   // one-shot problem: launch eagerly rather than capture
    // chunked LM, every window resuming its own run
    ba_lm_options o = S->opt.lm;
    const int chunk = S->opt.iters_per_check > 0 ? S->opt.iters_per_check : 10;
    std::vector<double> resume(4LL * W);
    std::vector<ba_lm_report> acc(W), rep(W);
    std::vector<char> open(W, 1), first(W, 1);
    for (int w = 0; w < W; w++) {
        resume[4 * w] = o.mu0 > 0 ? o.mu0 : 1e-2;
        resume[4 * w + 1] = o.nu0 > 0 ? o.nu0 : 2.0;
        resume[4 * w + 2] = o.rejects0;
        std::memset(&acc[w], 0, sizeof(ba_lm_report));
    }
    auto close = [&](int w, bool cancelled) -> ba_status {
        Request &R = *B[w];
        R.st.report = acc[w];
        hipError_t e = hipMemcpyAsync(R.poses.data(), d_poses + 12LL * s0[w], sizeof(double) * 12 * R.n_scans,
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("copy of served poses failed: %s", hipGetErrorString(e));
            return BA_E_HIP;
        }
        finish_request(S, R, BA_OK, cancelled, std::string());
        open[w] = 0;
        return BA_OK;
    };
    int left = o.max_iters;
    for (;;) {
        for (int w = 0; w < W; w++)
            if (open[w] && B[w]->cancel.load()) BA_TRY(close(w, true));
        bool any = false;
        for (int w = 0; w < W; w++) any = any || open[w];
        if (!any) break;
        if (left <= 0) {
            for (int w = 0; w < W; w++)
                if (open[w]) BA_TRY(close(w, false));
            break;
        }
        for (int w = 0; w < W; w++) resume[4 * w + 3] = open[w] ? 0.0 : 1.0;
        o.max_iters = std::min(chunk, left);
        o.resume = resume.data();
        BA_TRY(ba_iterate(p, d_poses, &o, rep.data(), nullptr, stream));
        for (int w = 0; w < W; w++) {
            if (!open[w]) continue;
            const ba_lm_report &r = rep[w];
            ba_lm_report &a = acc[w];
            if (first[w]) a.cost_initial = r.cost_initial;
            first[w] = 0;
            a.iters += r.iters;
            a.n_accepted += r.n_accepted;
            a.converged = r.converged;
            a.stalled = r.stalled;
            a.last_info = r.last_info;
            a.cost_final = r.cost_final;
            a.gnorm_final = r.gnorm_final;
            a.mu_final = r.mu_final;
            a.nu_final = r.nu_final;
            a.rejects_final = r.rejects_final;
            resume[4 * w] = r.mu_final;
            resume[4 * w + 1] = r.nu_final;
            resume[4 * w + 2] = r.rejects_final;
            if (r.converged || r.stalled || r.iters < o.max_iters) BA_TRY(close(w, false));
        }
        left -= o.max_iters;
    }
    (void)hipStreamSynchronize(stream);
    return BA_OK;
}

static void slot_main(Server *S) {
    (void)hipSetDevice(S->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    const int batch = std::max(1, (int)S->opt.batch);
    SlotArena arena;
    for (;;) {
        std::vector<std::shared_ptr<Request>> B;
        int64_t need = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] {
                return S->stopping ||
                       (!S->queue.empty() && S->reserved + S->queue.front()->footprint <= S->opt.hbm_budget);
            });
            if (S->stopping) break;
            // the head, and the requests behind it while they fit (queue order);
            // requests admitted together share their admission time
            const double t_admit = S->now();
            while (!S->queue.empty() && (int)B.size() < batch &&
                   S->reserved + S->queue.front()->footprint <= S->opt.hbm_budget) {
                std::shared_ptr<Request> R = S->queue.front();
                S->queue.pop_front();
                S->reserved += R->footprint;
                need += R->footprint;
                R->st.state = BA_REQ_RUNNING;
                R->st.t_admit = t_admit;
                B.push_back(R);
            }
        }
        S->cv.notify_all();   // the next head may fit too
        ba_status st = BA_E_HIP;
        bool cancelled = false;
        if (have_stream) {
            arena_reserve(S, arena, need);
            arena.off = 0;
            tl_slot_arena = arena.base ? &arena : nullptr;
            if (B.size() == 1)
                st = run_request(S, *B[0], stream, cancelled);
            else
                st = run_batch(S, B, stream);
            tl_slot_arena = nullptr;
            arena.off = 0;   // the problem is released: the stream has drained
        }
        const std::string err = st == BA_OK ? std::string() : std::string(ba_last_error());
        for (auto &R : B) {
            bool open;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                open = R->st.state == BA_REQ_RUNNING;
            }
            // a batch finishes its requests itself; what is still open failed
            if (B.size() == 1 || open) finish_request(S, *R, B.size() == 1 ? st : (st == BA_OK ? BA_E_HIP : st),
                                                      B.size() == 1 && cancelled, err);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->reserved -= need;
        }
        S->cv.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(stream);
    if (arena.base) (void)hipFree(arena.base);
}

thread_local SlotArena *tl_slot_arena = nullptr;

}  // namespace ba

struct ba_server {
    ba::Server S;
};

extern "C" {

ba_status ba_request_footprint(const ba_request *req, int32_t mode, int32_t precision, int64_t *bytes) {
    using namespace ba;
    BA_TRY(validate_request(req));
    if (!bytes) {
        set_error("bytes is null");
        return BA_E_ARG;
    }
    *bytes = footprint_bytes(req->n, req->n_voxels, req->n_scans, mode, precision);
    return BA_OK;
}

ba_status ba_server_create(const ba_server_options *opt, ba_server **out) {
    using namespace ba;
    if (!opt || !out || opt->hbm_budget <= 0 || opt->slots < 1 || opt->slots > 64 || opt->iters_per_check < 0 ||
        (opt->precision != BA_PREC_F64 && opt->precision != BA_PREC_F32) ||
        (opt->lm.mode != BA_MODE_MM && opt->lm.mode != BA_MODE_COUPLED) || opt->lm.max_iters < 1 ||
        opt->batch < 0 || opt->batch > 256 || opt->lm.resume) {
        set_error("invalid server options");
        return BA_E_ARG;
    }
    ba_server *s = new (std::nothrow) ba_server();
    if (!s) {
        set_error("host allocation failed");
        return BA_E_NOMEM;
    }
    s->S.opt = *opt;
    s->S.t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->S.device) != hipSuccess) {
        delete s;
        set_error("no HIP device");
        return BA_E_HIP;
    }
    try {
        for (int i = 0; i < opt->slots; i++) s->S.slots.emplace_back(slot_main, &s->S);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->S.mu);
            s->S.stopping = true;
        }
        s->S.cv.notify_all();
        for (auto &t : s->S.slots) t.join();
        delete s;
        set_error("could not start the slot threads");
        return BA_E_NOMEM;
    }
    *out = s;
    return BA_OK;
}

ba_status ba_server_submit(ba_server *s, const ba_request *req, int64_t *id) {
    using namespace ba;
    if (!s || !id) {
        set_error("null server or id");
        return BA_E_ARG;
    }
    BA_TRY(validate_request(req));
    Server *S = &s->S;
    auto R = std::make_shared<Request>();
    R->n = req->n;
    R->n_scans = req->n_scans;
    R->n_voxels = req->n_voxels;
    for (int64_t i = 0; i < req->n; i++)
        if (req->voxel[i] < 0 || req->voxel[i] >= req->n_voxels || req->scan[i] < 0 || req->scan[i] >= req->n_scans) {
            set_error("request label out of range at %lld", (long long)i);
            return BA_E_ARG;
        }
    R->footprint = footprint_bytes(req->n, req->n_voxels, req->n_scans, S->opt.lm.mode, S->opt.precision);
    if (R->footprint > S->opt.hbm_budget) {
        set_error("request needs %lld device bytes, budget %lld", (long long)R->footprint,
                  (long long)S->opt.hbm_budget);
        return BA_E_BUDGET;
    }
    R->voxel.assign(req->voxel, req->voxel + req->n);
    R->scan.assign(req->scan, req->scan + req->n);
    R->count.assign(req->count, req->count + req->n);
    R->sum.assign(req->sum, req->sum + 3 * req->n);
    R->sumsq.assign(req->sumsq, req->sumsq + 6 * req->n);
    R->poses.assign(req->poses_init, req->poses_init + 12LL * req->n_scans);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            set_error("server is stopping");
            return BA_E_ARG;
        }
        R->id = S->next_id++;
        R->st.state = BA_REQ_QUEUED;
        R->st.status = BA_OK;
        R->st.footprint = R->footprint;
        R->st.t_submit = S->now();
        S->queue.push_back(R);
        S->all[R->id] = R;
        *id = R->id;
    }
    S->cv.notify_all();
    return BA_OK;
}

ba_status ba_server_query(ba_server *s, int64_t id, ba_request_status *st) {
    using namespace ba;
    if (!s || !st) {
        set_error("null argument");
        return BA_E_ARG;
    }
    std::lock_guard<std::mutex> lk(s->S.mu);
    auto it = s->S.all.find(id);
    if (it == s->S.all.end()) {
        set_error("unknown request %lld", (long long)id);
        return BA_E_NOT_FOUND;
    }
    *st = it->second->st;
    return BA_OK;
}

ba_status ba_server_wait(ba_server *s, int64_t id, double *poses_out, ba_request_status *st) {
    using namespace ba;
    if (!s) {
        set_error("null server");
        return BA_E_ARG;
    }
    Server *S = &s->S;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) {
        set_error("unknown request %lld", (long long)id);
        return BA_E_NOT_FOUND;
    }
    std::shared_ptr<Request> R = it->second;
    auto finished = [&] {
        return R->st.state == BA_REQ_DONE || R->st.state == BA_REQ_FAILED || R->st.state == BA_REQ_CANCELLED;
    };
    S->cv.wait(lk, [&] { return finished() || S->stopping; });
    if (!finished()) {
        set_error("server stopped before request %lld ran", (long long)id);
        return BA_E_ARG;
    }
    if (poses_out && (R->st.state == BA_REQ_DONE || R->st.state == BA_REQ_CANCELLED))
        std::memcpy(poses_out, R->poses.data(), sizeof(double) * R->poses.size());
    if (st) *st = R->st;
    S->all.erase(it);
    if (R->st.state == BA_REQ_DONE) return BA_OK;
    if (R->st.state == BA_REQ_CANCELLED) {
        set_error("request %lld was cancelled", (long long)id);
        return BA_E_CANCELLED;
    }
    set_error("served request %lld failed: %s", (long long)id, R->error.c_str());
    return R->st.status;
}

ba_status ba_server_cancel(ba_server *s, int64_t id) {
    using namespace ba;
    if (!s) {
        set_error("null server");
        return BA_E_ARG;
    }
    Server *S = &s->S;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(id);
        if (it == S->all.end()) {
            set_error("unknown request %lld", (long long)id);
            return BA_E_NOT_FOUND;
        }
        std::shared_ptr<Request> R = it->second;
        R->cancel.store(true);
        if (R->st.state == BA_REQ_QUEUED) {
            for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
                if ((*q)->id == id) {
                    S->queue.erase(q);
                    break;
                }
            R->st.state = BA_REQ_CANCELLED;
            R->st.status = BA_E_CANCELLED;
            R->st.t_done = S->now();
        }
    }
    S->cv.notify_all();
    return BA_OK;
}

ba_status ba_server_destroy(ba_server *s) {
    using namespace ba;
    if (!s) return BA_OK;
    {
        std::lock_guard<std::mutex> lk(s->S.mu);
        s->S.stopping = true;
        s->S.queue.clear();
    }
    s->S.cv.notify_all();
    for (auto &t : s->S.slots) t.join();
    delete s;
    return BA_OK;
}

}  // extern "C"
