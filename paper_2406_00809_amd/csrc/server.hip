// Solve server: continuous batching of FGMRES solves over resident systems.
//
// Systems (CSR, gamma, A-hat) and their trained networks are registered once
// and stay resident.  Requests (a right-hand side for a registered system)
// queue on the host; a worker thread admits them into slots (admission.hpp:
// slot count and HBM budget of the solve workspaces) whenever a slot and
// memory free up, and drives every busy slot through its restart cycles.
// Each slot has its own HIP stream, so the cycles of different requests run
// concurrently on the device; a slot's workspace (Krylov basis V, network
// outputs Z, activations, b, x) stays resident after its request finishes
// and is reused by the next request on the same system.  Every request runs
// the same kernels as a single fgmres_solve with x0 = 0, on buffers of its
// own, so its result does not depend on what else is in flight.
// Latency is stamped at submission and when the solution has reached host
// memory.
//
// Registered systems live at stable addresses (one heap object each): the
// worker keeps pointers to them while requests run, and registration may
// happen at any time.  A system's values can be replaced while the server
// runs (gnp_server_update_system, the evolving systems of Sec. 5): its
// queued requests wait, the running ones finish on the old values, then the
// values are replaced, the network is optionally trained further, and its
// requests are admitted again.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.hpp"
#include "solver.hpp"

namespace gnp {

using Clock = std::chrono::steady_clock;

struct SrvRequest {
    uint64_t ticket = 0;
    int sys_id = 0;
    std::vector<double> b;
    double rtol = 0.0;
    int maxiters = 0;
    Clock::time_point t_submit, t_done;
    std::vector<double> x;
    gnp_solve_info info{};
    gnp_status status = GNP_OK;
    std::string msg;
    bool done = false;
};

struct SrvWorkspace {
    int sys_id = 0;
    SolveCtx ctx;
    double *b_dev = nullptr, *x_dev = nullptr;  // device
    double *b_pin = nullptr, *x_pin = nullptr;  // pinned host staging
    size_t bytes = 0;                           // device bytes (HBM budget)
    uint64_t stamp = 0;
};

enum SlotPhase { PH_IDLE = 0, PH_BEGIN, PH_CYCLE, PH_COPYOUT };

struct SrvSystem;

struct SrvSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    SrvWorkspace *ws = nullptr;
    SrvRequest *req = nullptr;
    SrvSystem *sys = nullptr;  // the request's system (stable address)
    int phase = PH_IDLE;
    int it0 = 0;
};

struct SrvSystem {
    gnp_system *sys = nullptr;
    gnp_model *model = nullptr;
    size_t ws_bytes = 0;
    int active = 0;        // slots running a request of this system
    bool paused = false;   // an update is in progress: admit none of its requests
};

static gnp_status hip_ok(hipError_t e, const char *what) {
    return e == hipSuccess ? GNP_OK : check_hip(e, what);
}

static void ws_free(SrvWorkspace *w) {
    if (!w) return;
    solve_ctx_free(&w->ctx);
    if (w->b_dev) (void)hipFree(w->b_dev);
    if (w->x_dev) (void)hipFree(w->x_dev);
    if (w->b_pin) (void)hipHostFree(w->b_pin);
    if (w->x_pin) (void)hipHostFree(w->x_pin);
    delete w;
}

}  // namespace gnp

using namespace gnp;

struct gnp_server {
    int device = 0;
    int max_slots = 0, m = 0, max_iters = 0;
    gnp_precision prec = GNP_BF16;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::vector<std::unique_ptr<SrvSystem>> systems;
    std::deque<SrvRequest *> queue;
    std::unordered_map<uint64_t, SrvRequest *> requests;
    std::vector<SrvSlot> slots;
    std::vector<SrvWorkspace *> idle;
    AdmissionState adm;
    uint64_t next_ticket = 1, stamp = 0;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, converged = 0;
    int64_t ws_alloc = 0, ws_reuse = 0, ws_evict = 0;
    int busy = 0, max_busy = 0;
    size_t peak = 0;
    std::vector<double> latencies, conv_latencies;
    Clock::time_point t_first, t_last, t_last_conv;
};

namespace gnp {

static gnp_status ws_alloc(gnp_server *S, int sys_id, SrvWorkspace **out) {
    const SrvSystem &sy = *S->systems[sys_id];
    SrvWorkspace *w = new SrvWorkspace();
    w->sys_id = sys_id;
    w->bytes = sy.ws_bytes;
    const int64_t n = sy.sys->n;
    gnp_status st = solve_ctx_prepare(&w->ctx, sy.sys, S->m, S->max_iters, S->prec,
                                      sy.model ? sy.model->d : 0);
    if (st == GNP_OK) st = hip_ok(hipMalloc(&w->b_dev, sizeof(double) * n), "hipMalloc");
    if (st == GNP_OK) st = hip_ok(hipMalloc(&w->x_dev, sizeof(double) * n), "hipMalloc");
    if (st == GNP_OK)
        st = hip_ok(hipHostMalloc(&w->b_pin, sizeof(double) * n, hipHostMallocDefault),
                       "hipHostMalloc");
    if (st == GNP_OK)
        st = hip_ok(hipHostMalloc(&w->x_pin, sizeof(double) * n, hipHostMallocDefault),
                       "hipHostMalloc");
    if (st != GNP_OK) {
        ws_free(w);
        return st;
    }
    *out = w;
    return GNP_OK;
}

// Mark a request finished (called with the lock held).
static void finish_locked(gnp_server *S, SrvRequest *r, gnp_status st, const std::string &msg) {
    r->status = st;
    r->msg = msg;
    r->done = true;
    r->t_done = Clock::now();
    if (st == GNP_OK) {
        const double lat = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        ++S->completed;
        S->latencies.push_back(lat);
        S->t_last = r->t_done;
        if (r->info.converged) {
            ++S->converged;
            S->conv_latencies.push_back(lat);
            S->t_last_conv = r->t_done;
        }
    } else {
        ++S->failed;
    }
    S->cv_done.notify_all();
}

// Release a slot after its request ended: the workspace stays resident, idle.
static void release_slot_locked(gnp_server *S, SrvSlot &sl) {
    sl.ws->stamp = ++S->stamp;
    S->idle.push_back(sl.ws);
    sl.ws = nullptr;
    sl.req = nullptr;
    if (--sl.sys->active == 0) S->cv_done.notify_all();
    sl.sys = nullptr;
    sl.phase = PH_IDLE;
    --S->busy;
    S->cv_work.notify_all();
}

// Enqueue the start of a request on a slot (worker thread).
static gnp_status start_request(gnp_server *S, SrvSlot &sl) {
    SrvWorkspace *w = sl.ws;
    SrvRequest *r = sl.req;
    const int64_t n = sl.sys->sys->n;
    memcpy(w->b_pin, r->b.data(), sizeof(double) * n);
    GNP_HIP(hipMemcpyAsync(w->b_dev, w->b_pin, sizeof(double) * n, hipMemcpyHostToDevice, sl.st));
    GNP_HIP(hipMemsetAsync(w->x_dev, 0, sizeof(double) * n, sl.st));
    w->ctx.prec = S->prec;
    GNP_TRY(solve_begin(&w->ctx, w->b_dev, w->x_dev, S->m, r->rtol, r->maxiters, sl.st));
    GNP_HIP(hipEventRecord(sl.ev, sl.st));
    sl.phase = PH_BEGIN;
    return GNP_OK;
}

// Admit queued requests into free slots (worker thread, lock held).
static void admit_locked(gnp_server *S) {
    if (S->queue.empty()) return;
    int free_slots = S->max_slots - S->busy;
    // requests of systems being updated wait in the queue, in order
    std::vector<size_t> qmap;
    std::vector<AdmitItem> qv;
    qv.reserve(S->queue.size());
    for (size_t k = 0; k < S->queue.size(); ++k) {
        const SrvSystem &sy = *S->systems[S->queue[k]->sys_id];
        if (sy.paused) continue;
        qmap.push_back(k);
        qv.push_back({S->queue[k]->sys_id, sy.ws_bytes});
    }
    if (qv.empty()) return;
    std::vector<IdleItem> iv;
    for (SrvWorkspace *w : S->idle) iv.push_back({w->sys_id, w->bytes, w->stamp});
    const std::vector<AdmitDecision> plan = plan_admission(S->adm, free_slots, qv, iv);
    if (plan.empty()) return;
    std::vector<bool> q_taken(S->queue.size(), false), i_taken(S->idle.size(), false);
    for (const AdmitDecision &d : plan) {
        const size_t qk = qmap[d.qpos];
        SrvRequest *r = S->queue[qk];
        SrvSystem *sy = S->systems[r->sys_id].get();
        q_taken[qk] = true;
        if (d.kind == AdmitDecision::REJECT) {
            ++S->rejected;
            finish_locked(S, r,
                          GNP_ENOMEM,
                          "solve workspace of " + std::to_string(sy->ws_bytes) +
                              " bytes exceeds the HBM budget of " +
                              std::to_string(S->adm.budget) + " bytes");
            continue;
        }
        SrvWorkspace *w = nullptr;
        if (d.kind == AdmitDecision::REUSE) {
            w = S->idle[d.idle_pos];
            i_taken[d.idle_pos] = true;
            ++S->ws_reuse;
        } else {
            for (size_t k : d.evict) {
                i_taken[k] = true;
                ws_free(S->idle[k]);
                ++S->ws_evict;
            }
            if (ws_alloc(S, r->sys_id, &w) != GNP_OK) {
                S->adm.used -= sy->ws_bytes;
                finish_locked(S, r, GNP_ENOMEM, gnp_last_error());
                continue;
            }
            ++S->ws_alloc;
        }
        S->peak = std::max(S->peak, S->adm.used);
        SrvSlot *sl = nullptr;
        for (SrvSlot &c : S->slots)
            if (c.phase == PH_IDLE) {
                sl = &c;
                break;
            }
        sl->ws = w;
        sl->req = r;
        sl->sys = sy;
        ++sy->active;
        ++S->busy;
        S->max_busy = std::max(S->max_busy, S->busy);
        const gnp_status st = start_request(S, *sl);
        if (st != GNP_OK) {
            finish_locked(S, r, st, gnp_last_error());
            release_slot_locked(S, *sl);
        }
    }
    std::deque<SrvRequest *> q2;
    for (size_t k = 0; k < S->queue.size(); ++k)
        if (!q_taken[k]) q2.push_back(S->queue[k]);
    S->queue.swap(q2);
    std::vector<SrvWorkspace *> i2;
    for (size_t k = 0; k < S->idle.size(); ++k)
        if (!i_taken[k]) i2.push_back(S->idle[k]);
    S->idle.swap(i2);
}

// Advance a slot whose last enqueued stage has completed (worker thread).
// Returns the status of the request if it ended, GNP_EBUSY while it runs on.
static gnp_status advance(gnp_server *S, SrvSlot &sl, std::string &msg) {
    SrvWorkspace *w = sl.ws;
    SrvRequest *r = sl.req;
    const SrvSystem &sy = *sl.sys;  // stable: registration never moves it
    const int64_t n = sy.sys->n;
    const Ctl &h = *w->ctx.ctl_host;
    switch (sl.phase) {
        case PH_BEGIN:
            if (!std::isfinite(h.bnorm)) {
                msg = "b is not finite";
                return GNP_ENUMERIC;
            }
            if (h.bnorm == 0.0) {
                r->x.assign(n, 0.0);
                memset(&r->info, 0, sizeof(r->info));
                r->info.converged = 1;
                return GNP_OK;
            }
            break;
        case PH_CYCLE:
            if (h.solve_done) {
                if (h.nonfinite) {
                    msg = "non-finite value in the Arnoldi process";
                    return GNP_ENUMERIC;
                }
                if (hipMemcpyAsync(w->x_pin, w->x_dev, sizeof(double) * n,
                                   hipMemcpyDeviceToHost, sl.st) != hipSuccess ||
                    hipEventRecord(sl.ev, sl.st) != hipSuccess) {
                    msg = "copy of the solution failed";
                    return GNP_EDEVICE;
                }
                sl.phase = PH_COPYOUT;
                return GNP_EBUSY;
            }
            if (h.it <= sl.it0) {
                msg = "solver made no progress in a cycle";
                return GNP_EDEVICE;
            }
            break;
        case PH_COPYOUT:
            r->x.assign(w->x_pin, w->x_pin + n);
            solve_info_from(h, &r->info);
            return GNP_OK;
        default:
            msg = "slot in an unknown state";
            return GNP_EDEVICE;
    }
    // next restart cycle
    sl.it0 = h.it;
    gnp_status st = solve_next(&w->ctx, sy.model, w->b_dev, w->x_dev, S->m, r->maxiters, sl.st);
    if (st == GNP_OK) st = hip_ok(hipEventRecord(sl.ev, sl.st), "hipEventRecord");
    if (st != GNP_OK) {
        msg = gnp_last_error();
        return st;
    }
    sl.phase = PH_CYCLE;
    return GNP_EBUSY;
}

static void worker_main(gnp_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) {
                for (SrvRequest *r : S->queue)
                    finish_locked(S, r, GNP_EBUSY, "server shut down before the request started");
                S->queue.clear();
                if (S->busy == 0) break;
            } else {
                admit_locked(S);
            }
        }
        bool progressed = false;
        for (SrvSlot &sl : S->slots) {
            if (sl.phase == PH_IDLE) continue;
            const hipError_t e = hipEventQuery(sl.ev);
            if (e == hipErrorNotReady) continue;
            progressed = true;
            std::string msg;
            gnp_status st;
            if (e != hipSuccess) {
                st = GNP_EDEVICE;
                msg = std::string("HIP error '") + hipGetErrorString(e) + "' in a served solve";
            } else {
                st = advance(S, sl, msg);
            }
            if (st != GNP_EBUSY) {
                std::lock_guard<std::mutex> lk(S->mu);
                finish_locked(S, sl.req, st, msg);
                release_slot_locked(S, sl);
            }
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(S->mu);
            const bool can_admit = !S->queue.empty() && S->busy < S->max_slots;
            if (!S->stop && !can_admit)
                S->cv_work.wait_for(lk, std::chrono::microseconds(S->busy > 0 ? 20 : 2000));
        }
    }
}

static double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    // nearest rank
    size_t k = (size_t)ceil(p / 100.0 * (double)v.size());
    if (k < 1) k = 1;
    if (k > v.size()) k = v.size();
    return v[k - 1];
}

}  // namespace gnp

extern "C" {

gnp_status gnp_server_create(size_t hbm_budget, int max_slots, int m, int max_iters,
                             gnp_precision prec, gnp_server **out) {
    if (!out) return fail(GNP_EINVAL, "out is null");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 256) return fail(GNP_EINVAL, "max_slots must be in [1, 256]");
    if (m < 1 || m > 255) return fail(GNP_EINVAL, "m must be in [1, 255]");
    if (max_iters < 1) return fail(GNP_EINVAL, "max_iters must be >= 1");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    if (hbm_budget == 0) return fail(GNP_EINVAL, "hbm_budget must be > 0");
    gnp_server *S = new gnp_server();
    S->max_slots = max_slots;
    S->m = m;
    S->max_iters = max_iters;
    S->prec = prec;
    S->adm.budget = hbm_budget;
    S->slots.resize(max_slots);
    gnp_status st = hip_ok(hipGetDevice(&S->device), "hipGetDevice");
    for (int k = 0; k < max_slots && st == GNP_OK; ++k) {
        st = hip_ok(hipStreamCreateWithFlags(&S->slots[k].st, hipStreamNonBlocking),
                       "hipStreamCreate");
        if (st == GNP_OK)
            st = hip_ok(hipEventCreateWithFlags(&S->slots[k].ev, hipEventDisableTiming),
                           "hipEventCreate");
    }
    if (st != GNP_OK) {
        for (SrvSlot &sl : S->slots) {
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.st) (void)hipStreamDestroy(sl.st);
        }
        delete S;
        return st;
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return GNP_OK;
}

gnp_status gnp_server_register(gnp_server *S, gnp_system *sys, gnp_model *model, int *id) {
    if (!S || !sys || !id) return fail(GNP_EINVAL, "null argument");
    if (model && model->sys != sys) return fail(GNP_EINVAL, "model belongs to another system");
    auto sy = std::make_unique<SrvSystem>();
    sy->sys = sys;
    sy->model = model;
    sy->ws_bytes = solve_ctx_bytes(sys->n, S->m, S->max_iters, S->prec, model ? model->d : 0) +
                   2 * sizeof(double) * (size_t)sys->n;
    std::lock_guard<std::mutex> lk(S->mu);
    S->systems.push_back(std::move(sy));
    *id = (int)S->systems.size() - 1;
    return GNP_OK;
}

gnp_status gnp_server_workspace_bytes(gnp_server *S, int id, size_t *bytes) {
    if (!S || !bytes) return fail(GNP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (id < 0 || id >= (int)S->systems.size()) return fail(GNP_EINVAL, "unknown system id");
    *bytes = S->systems[id]->ws_bytes;
    return GNP_OK;
}

gnp_status gnp_server_submit(gnp_server *S, int id, const double *b_host, double rtol,
                             int maxiters, uint64_t *ticket) {
    if (!S || !b_host || !ticket) return fail(GNP_EINVAL, "null argument");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1 || maxiters > S->max_iters)
        return fail(GNP_EINVAL, "maxiters must be in [1, the server's max_iters]");
    SrvRequest *r = new SrvRequest();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (id < 0 || id >= (int)S->systems.size()) {
            delete r;
            return fail(GNP_EINVAL, "unknown system id");
        }
        if (S->stop) {
            delete r;
            return fail(GNP_EBUSY, "server is shutting down");
        }
        const int64_t n = S->systems[id]->sys->n;
        r->sys_id = id;
        r->b.assign(b_host, b_host + n);
        r->rtol = rtol;
        r->maxiters = maxiters;
        r->t_submit = Clock::now();
        r->ticket = S->next_ticket++;
        if (S->submitted == 0) S->t_first = r->t_submit;
        ++S->submitted;
        S->requests[r->ticket] = r;
        S->queue.push_back(r);
        *ticket = r->ticket;
    }
    S->cv_work.notify_all();
    return GNP_OK;
}

gnp_status gnp_server_poll(gnp_server *S, uint64_t ticket, double *x_host, gnp_solve_info *info,
                           double *latency_s) {
    if (!S) return fail(GNP_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->requests.find(ticket);
    if (it == S->requests.end()) return fail(GNP_EINVAL, "unknown or already collected ticket");
    SrvRequest *r = it->second;
    if (!r->done) return GNP_EBUSY;
    const gnp_status st = r->status;
    if (st == GNP_OK) {
        if (x_host) memcpy(x_host, r->x.data(), sizeof(double) * r->x.size());
        if (info) *info = r->info;
        if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    } else {
        fail(st, r->msg);
    }
    S->requests.erase(it);
    delete r;
    return st;
}

gnp_status gnp_server_drain(gnp_server *S, double timeout_s) {
    if (!S) return fail(GNP_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(timeout_s));
    const bool ok = S->cv_done.wait_until(lk, until, [&] { return S->queue.empty() && S->busy == 0; });
    return ok ? GNP_OK : fail(GNP_EBUSY, "requests still pending at the timeout");
}

gnp_status gnp_server_update_system(gnp_server *S, int id, const double *val,
                                    const gnp_train_opts *tune, double *loss_hist,
                                    int *best_step) {
    if (!S || !val) return fail(GNP_EINVAL, "null argument");
    SrvSystem *sy = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        if (id < 0 || id >= (int)S->systems.size()) return fail(GNP_EINVAL, "unknown system id");
        sy = S->systems[id].get();
        if (sy->paused) return fail(GNP_EBUSY, "an update of this system is in progress");
        if (tune && !sy->model) return fail(GNP_EINVAL, "fine-tuning needs a registered network");
        sy->paused = true;  // from now on its queued requests wait
        S->cv_done.wait(lk, [&] { return sy->active == 0; });
    }
    // no request of this system is in a slot: its matrix and network are ours
    gnp_status st = gnp_system_set_values(sy->sys, val, nullptr);
    if (st == GNP_OK && tune) st = gnp_train(sy->model, tune, nullptr, loss_hist, best_step,
                                             nullptr);
    const std::string msg = st == GNP_OK ? std::string() : std::string(gnp_last_error());
    {
        std::lock_guard<std::mutex> lk(S->mu);
        sy->paused = false;
    }
    S->cv_work.notify_all();
    return st == GNP_OK ? GNP_OK : fail(st, msg);
}

gnp_status gnp_server_get_stats(gnp_server *S, gnp_server_stats *o) {
    if (!S || !o) return fail(GNP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    memset(o, 0, sizeof(*o));
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->failed = S->failed;
    o->rejected = S->rejected;
    o->queued = (int64_t)S->queue.size();
    o->active = S->busy;
    o->max_active = S->max_busy;
    o->converged = S->converged;
    o->latency_p50_s = percentile(S->latencies, 50.0);
    o->latency_p99_s = percentile(S->latencies, 99.0);
    o->conv_latency_p50_s = percentile(S->conv_latencies, 50.0);
    o->conv_latency_p99_s = percentile(S->conv_latencies, 99.0);
    const double cspan = std::chrono::duration<double>(S->t_last_conv - S->t_first).count();
    o->converged_per_s = (S->converged > 0 && cspan > 0.0) ? (double)S->converged / cspan : 0.0;
    double sum = 0.0;
    for (double v : S->latencies) sum += v;
    o->latency_mean_s = S->latencies.empty() ? 0.0 : sum / (double)S->latencies.size();
    const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
    o->solves_per_s = (S->completed > 0 && span > 0.0) ? (double)S->completed / span : 0.0;
    o->hbm_budget = S->adm.budget;
    o->hbm_used = S->adm.used;
    o->hbm_peak = S->peak;
    o->workspaces_allocated = S->ws_alloc;
    o->workspaces_reused = S->ws_reuse;
    o->workspaces_evicted = S->ws_evict;
    return GNP_OK;
}

void gnp_server_destroy(gnp_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (SrvWorkspace *w : S->idle) ws_free(w);
    for (SrvSlot &sl : S->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (auto &kv : S->requests) delete kv.second;
    delete S;
}

}  // extern "C"
