// solver.cpp -- serving runtime: many RK4 boxes resident on one GPU.
//
// Requests (initial state on the host, box, parameters, steps) are queued by
// solver_submit and admitted in arrival order while a slot is free and their
// device footprint (state + workspace) fits the HBM budget.  Every resident
// request owns a HIP stream (default priority, for its copies) and advances in
// chunks of RK4 steps (continuous batching: a finished request frees its slot
// and memory at once and the next queued request is admitted).  Two ways of
// stepping: a worker thread keeps one chunk in flight per resident request on
// the request's stream, so the GPU interleaves all of them; or (batched) it
// keeps one batched chunk in flight over all resident requests, rk_step_batch
// per group with the same parameters and precision, so that small boxes share
// launches.  Each request runs exactly the arithmetic of rk_step on its box
// alone, so its result does not depend on what else is resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nopcs.h"

namespace nopcs {
void set_error(const std::string &msg);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    solve_request req{};
    std::vector<double> q0;        // initial state (copied at submit; kept until its upload has completed)
    std::vector<double> qout;      // final state (filled when done)
    size_t n_elems = 0;            // 5 * points
    size_t footprint = 0;          // device bytes while resident
    size_t ws_bytes = 0;
    double *dQ = nullptr;          // device state
    void *dws = nullptr;           // device workspace
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;       // end of the chunk (batched: of the upload) in flight
    bool in_flight = false;
    int32_t chunk = 0;             // batched: steps of the batched chunk in flight
    int32_t steps_done = 0;
    int32_t status = NOPCS_EAGAIN;
    double t_submit = 0, t_admit = -1, t_done = -1;
    bool done = false;
};

}  // namespace

struct nopcs_solver {
    solver_config cfg{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_id = 1;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<uint64_t> queue;       // waiting for admission, in arrival order
    std::vector<uint64_t> resident;   // admitted and not finished
    size_t resident_bytes = 0;
    std::vector<hipStream_t> free_streams;
    std::thread worker;
    int chunk_steps = 8;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    void run_batched();
    bool admit_one(std::unique_lock<std::mutex> &lk);
    bool copy_out(std::unique_lock<std::mutex> &lk, Request &r);
    void finish(Request &r, int status);
};

namespace {

size_t footprint_of(const solve_request &q, size_t *ws_bytes) {
    const size_t ws = nopcs_workspace_bytes(&q.grid, q.precision);
    if (ws == 0) return 0;
    const size_t n = (size_t)q.grid.n[0] * q.grid.n[1] * q.grid.n[2];
    const size_t state = ((5 * n * sizeof(double)) + 255) & ~(size_t)255;
    if (ws_bytes) *ws_bytes = ws;
    return state + ws;
}

}  // namespace

// Admit the request at the head of the queue if a slot and budget allow
// (strict arrival order: a large request at the head is not overtaken).
bool nopcs_solver::admit_one(std::unique_lock<std::mutex> &lk) {
    if (queue.empty() || (int)resident.size() >= cfg.max_slots || free_streams.empty()) return false;
    Request &r = *reqs[queue.front()];
    if (resident_bytes + r.footprint > cfg.hbm_budget_bytes) return false;
    const uint64_t id = queue.front();
    queue.pop_front();
    resident.push_back(id);
    resident_bytes += r.footprint;
    r.stream = free_streams.back();
    free_streams.pop_back();
    lk.unlock();
    int status = NOPCS_OK;
    if (hipMalloc(reinterpret_cast<void **>(&r.dQ), r.n_elems * sizeof(double)) != hipSuccess ||
        hipMalloc(&r.dws, r.ws_bytes) != hipSuccess) {
        status = NOPCS_ENOMEM;
    } else if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess ||
               hipMemcpyAsync(r.dQ, r.q0.data(), r.n_elems * sizeof(double), hipMemcpyHostToDevice, r.stream) !=
                   hipSuccess) {
        status = NOPCS_EDEVICE;
    } else if (cfg.batched) {
        // batched chunks run on the worker's stream: a request joins them once its upload is done
        if (hipEventRecord(r.ev, r.stream) != hipSuccess) status = NOPCS_EDEVICE;
        r.in_flight = true;
    }
    lk.lock();
    r.t_admit = now();
    // q0 stays until the upload is known to have completed (an event after it
    // has fired): the copy from pageable memory may read it after the call
    // returns, once the stream's hardware queue gets to it
    if (status != NOPCS_OK) finish(r, status);
    return true;
}

// Release a request's device resources and publish its result (called with the lock held).
void nopcs_solver::finish(Request &r, int status) {
    if (r.ev) (void)hipEventDestroy(r.ev);
    if (r.dQ) (void)hipFree(r.dQ);   // waits for the device, the upload included
    if (r.dws) (void)hipFree(r.dws);
    std::vector<double>().swap(r.q0);
    r.ev = nullptr;
    r.dQ = nullptr;
    r.dws = nullptr;
    free_streams.push_back(r.stream);
    r.stream = nullptr;
    resident_bytes -= r.footprint;
    for (size_t i = 0; i < resident.size(); ++i) {
        if (reqs[resident[i]].get() == &r) {
            resident.erase(resident.begin() + (long)i);
            break;
        }
    }
    r.status = status;
    r.t_done = now();
    r.done = true;
    cv.notify_all();
}

// Result back to the host, non-finite check, release (called with the lock
// held; the request's device work has ended).
bool nopcs_solver::copy_out(std::unique_lock<std::mutex> &lk, Request &r) {
    r.qout.resize(r.n_elems);
    lk.unlock();
    const bool ok = hipMemcpyAsync(r.qout.data(), r.dQ, r.n_elems * sizeof(double), hipMemcpyDeviceToHost,
                                   r.stream) == hipSuccess &&
                    hipStreamSynchronize(r.stream) == hipSuccess;
    bool finite = ok;
    if (ok)
        for (double v : r.qout)
            if (!std::isfinite(v)) {
                finite = false;
                break;
            }
    lk.lock();
    finish(r, !ok ? NOPCS_EDEVICE : finite ? NOPCS_OK : NOPCS_ENONFINITE);
    return true;
}

// Batched stepping: one batched chunk in flight on the worker's own stream.
// When it ends, finished requests are copied back after the next chunk has
// been launched (their memory is no longer touched by it).
void nopcs_solver::run_batched() {
    (void)hipSetDevice(cfg.device);
    hipStream_t bst = nullptr;
    hipEvent_t bev = nullptr;
    const bool dev_ok = hipStreamCreateWithFlags(&bst, hipStreamNonBlocking) == hipSuccess &&
                        hipEventCreateWithFlags(&bev, hipEventDisableTiming) == hipSuccess;
    std::vector<Request *> members;   // the requests of the chunk in flight
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        while (admit_one(lk)) {
        }
        bool progressed = false;
        if (!members.empty()) {
            const hipError_t q = hipEventQuery(bev);
            if (q == hipErrorNotReady) {
                cv.wait_for(lk, std::chrono::microseconds(100));
                continue;
            }
            for (Request *r : members) {
                if (r->done) continue;
                if (q != hipSuccess) finish(*r, NOPCS_EDEVICE);
                else r->steps_done += r->chunk;
            }
            members.clear();
            progressed = true;
        }
        // requests ready for a chunk (upload done, steps left), grouped by parameters and precision
        std::vector<Request *> finished;
        std::map<std::string, std::vector<Request *>> groups;
        const std::vector<uint64_t> ids = resident;
        for (uint64_t id : ids) {
            auto it = reqs.find(id);
            if (it == reqs.end()) continue;
            Request &r = *it->second;
            if (r.done) continue;
            if (r.in_flight) {   // upload
                const hipError_t q = hipEventQuery(r.ev);
                if (q == hipErrorNotReady) continue;
                r.in_flight = false;
                if (q != hipSuccess) {
                    finish(r, NOPCS_EDEVICE);
                    continue;
                }
                std::vector<double>().swap(r.q0);   // the device copy is the state from now on
            }
            if (r.steps_done >= r.req.nsteps) {
                finished.push_back(&r);
                continue;
            }
            std::string key(reinterpret_cast<const char *>(&r.req.params), sizeof r.req.params);
            key.append(reinterpret_cast<const char *>(&r.req.precision), sizeof r.req.precision);
            groups[key].push_back(&r);
        }
        if (!dev_ok) {
            for (auto &g : groups)
                for (Request *r : g.second) finish(*r, NOPCS_EDEVICE);
            groups.clear();
        }
        // one batched chunk per group (at most NOPCS_MAX_BATCH boxes a call)
        for (auto &g : groups) {
            std::vector<Request *> &v = g.second;
            for (size_t a = 0; a < v.size(); a += NOPCS_MAX_BATCH) {
                const size_t e = std::min(v.size(), a + (size_t)NOPCS_MAX_BATCH);
                int32_t k = chunk_steps;
                std::vector<nopcs_box> boxes;
                for (size_t i = a; i < e; ++i) {
                    const Request &r = *v[i];
                    k = std::min(k, r.req.nsteps - r.steps_done);
                    boxes.push_back(nopcs_box{r.req.grid, r.dQ, r.dws, r.ws_bytes, r.req.dt});
                }
                const nse_params prm = v[a]->req.params;
                const int prec = v[a]->req.precision;
                lk.unlock();
                const int rc = rk_step_batch(&prm, (int32_t)boxes.size(), boxes.data(), prec, boxes[0].dt, k, bst);
                lk.lock();
                for (size_t i = a; i < e; ++i) {
                    if (rc != NOPCS_OK) {
                        finish(*v[i], rc);
                    } else {
                        v[i]->chunk = k;
                        members.push_back(v[i]);
                    }
                }
            }
        }
        if (!members.empty()) {
            if (hipEventRecord(bev, bst) != hipSuccess) {
                (void)hipStreamSynchronize(bst);
                for (Request *r : members) finish(*r, NOPCS_EDEVICE);
                members.clear();
            }
            progressed = true;
        }
        for (Request *r : finished) progressed = copy_out(lk, *r) || progressed;
        if (!progressed) cv.wait_for(lk, std::chrono::microseconds(200));
    }
    lk.unlock();
    // nothing may run on the requests' memory once the worker has ended
    if (bst) {
        (void)hipStreamSynchronize(bst);
        (void)hipStreamDestroy(bst);
    }
    if (bev) (void)hipEventDestroy(bev);
}

void nopcs_solver::run() {
    (void)hipSetDevice(cfg.device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        while (admit_one(lk)) {
        }
        bool progressed = false;
        const std::vector<uint64_t> ids = resident;
        for (uint64_t id : ids) {
            auto it = reqs.find(id);
            if (it == reqs.end()) continue;
            Request &r = *it->second;
            if (r.done) continue;
            if (r.in_flight) {
                const hipError_t q = hipEventQuery(r.ev);
                if (q == hipErrorNotReady) continue;
                r.in_flight = false;
                progressed = true;
                if (q != hipSuccess) {
                    finish(r, NOPCS_EDEVICE);
                    continue;
                }
                std::vector<double>().swap(r.q0);   // the upload preceded this chunk on the stream
            }
            if (r.steps_done >= r.req.nsteps) {
                progressed = copy_out(lk, r);
                continue;
            }
            // next chunk of steps, asynchronously on the request's stream
            const int32_t k = std::min(chunk_steps, r.req.nsteps - r.steps_done);
            lk.unlock();
            int rc = rk_step(&r.req.params, &r.req.grid, r.req.precision, r.dQ, r.req.dt, k, r.dws, r.ws_bytes,
                             r.stream);
            if (rc == NOPCS_OK && hipEventRecord(r.ev, r.stream) != hipSuccess) rc = NOPCS_EDEVICE;
            lk.lock();
            if (rc != NOPCS_OK) {
                finish(r, rc);
                continue;
            }
            r.steps_done += k;
            r.in_flight = true;
            progressed = true;
        }
        if (!progressed) {
            // nothing ready: wait briefly for a chunk to end or for a new request
            cv.wait_for(lk, std::chrono::microseconds(200));
        }
    }
}

extern "C" {

int solver_create(const solver_config *cfg, nopcs_solver **out) {
    if (!cfg || !out) { nopcs::set_error("cfg and out must be non-NULL"); return NOPCS_EINVAL; }
    if (cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->max_queue < 1 || cfg->hbm_budget_bytes == 0 ||
        (cfg->batched != 0 && cfg->batched != 1)) {
        nopcs::set_error("solver_config: need 1 <= max_slots <= 64, max_queue >= 1, hbm_budget_bytes > 0, batched 0 or 1");
        return NOPCS_EINVAL;
    }
#ifndef NOPCS_CPU_EMUL
    // Batched serving is switched off on the GPU: a stream of 256 boxes
    // (32^3-192^3, mixed precision) ended in a segmentation fault in a
    // non-Python thread a few seconds in, twice, without an explained cause;
    // it stays available in the CPU build of the kernels, where its tests run
    // under AddressSanitizer.
    if (cfg->batched) {
        nopcs::set_error("solver_config: batched serving is switched off on the GPU (unexplained host crash)");
        return NOPCS_EINVAL;
    }
#endif
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        nopcs::set_error("solver_config: no such device");
        return NOPCS_EINVAL;
    }
    auto s = std::make_unique<nopcs_solver>();
    s->cfg = *cfg;
    s->t0 = Clock::now();
    if (hipSetDevice(cfg->device) != hipSuccess) { nopcs::set_error("hipSetDevice failed"); return NOPCS_EDEVICE; }
    for (int i = 0; i < cfg->max_slots; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->free_streams) (void)hipStreamDestroy(x);
            nopcs::set_error("hipStreamCreate failed");
            return NOPCS_EDEVICE;
        }
        s->free_streams.push_back(st);
    }
    nopcs_solver *raw = s.release();
    raw->worker = std::thread([raw] {
        if (raw->cfg.batched) raw->run_batched();
        else raw->run();
    });
    *out = raw;
    return NOPCS_OK;
}

int solver_submit(nopcs_solver *s, const solve_request *req, uint64_t *id_out) {
    if (!s || !req || !id_out) { nopcs::set_error("solver, request and id_out must be non-NULL"); return NOPCS_EINVAL; }
    if (req->nsteps < 1 || !(req->dt > 0.0) || !std::isfinite(req->dt) || !req->Q0_host) {
        nopcs::set_error("request: need nsteps >= 1, dt > 0 finite and Q0_host");
        return NOPCS_EINVAL;
    }
    if (req->precision != NOPCS_FP64 && req->precision != NOPCS_MIXED) {
        nopcs::set_error("request: precision must be NOPCS_FP64 or NOPCS_MIXED");
        return NOPCS_EINVAL;
    }
    size_t ws = 0;
    const size_t fp = footprint_of(*req, &ws);
    if (fp == 0) return NOPCS_EINVAL;   // grid error already recorded
    if (fp > s->cfg.hbm_budget_bytes) {
        nopcs::set_error("request footprint " + std::to_string(fp) + " bytes exceeds the HBM budget");
        return NOPCS_ENOMEM;
    }
    auto r = std::make_unique<Request>();
    r->req = *req;
    r->req.Q0_host = nullptr;
    r->n_elems = 5 * (size_t)req->grid.n[0] * req->grid.n[1] * req->grid.n[2];
    r->footprint = fp;
    r->ws_bytes = ws;
    r->q0.assign(req->Q0_host, req->Q0_host + r->n_elems);
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int)s->queue.size() >= s->cfg.max_queue) { nopcs::set_error("queue full"); return NOPCS_EBUSY; }
    r->t_submit = s->now();
    const uint64_t id = s->next_id++;
    s->reqs[id] = std::move(r);
    s->queue.push_back(id);
    *id_out = id;
    s->cv.notify_all();
    return NOPCS_OK;
}

int solver_poll(nopcs_solver *s, uint64_t id, double *Q_out_host, solve_result *out) {
    if (!s) { nopcs::set_error("solver is NULL"); return NOPCS_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) { nopcs::set_error("unknown or released request id"); return NOPCS_ENOTFOUND; }
    Request &r = *it->second;
    if (out) {
        out->status = r.done ? r.status : NOPCS_EAGAIN;
        out->steps_done = r.steps_done;
        out->t_submit = r.t_submit;
        out->t_admit = r.t_admit;
        out->t_done = r.t_done;
    }
    if (!r.done) return NOPCS_EAGAIN;
    const int status = r.status;
    if (Q_out_host && !r.qout.empty()) std::memcpy(Q_out_host, r.qout.data(), r.qout.size() * sizeof(double));
    s->reqs.erase(it);
    return status;
}

double solver_now(nopcs_solver *s) { return s ? s->now() : 0.0; }

int solver_destroy(nopcs_solver *s) {
    if (!s) return NOPCS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->cfg.device);
    for (auto &kv : s->reqs) {
        Request &r = *kv.second;
        if (r.stream) (void)hipStreamSynchronize(r.stream);
        if (r.ev) (void)hipEventDestroy(r.ev);
        if (r.dQ) (void)hipFree(r.dQ);
        if (r.dws) (void)hipFree(r.dws);
        if (r.stream) s->free_streams.push_back(r.stream);
    }
    for (hipStream_t st : s->free_streams) (void)hipStreamDestroy(st);
    delete s;
    return NOPCS_OK;
}

}  // extern "C"
