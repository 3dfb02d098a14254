// Continuous batching of general edit-distance queries (lvs_submit /
// lvs_poll): both strings encrypted (Algorithm 4, with Algorithm 3's
// equality), or one cleartext string against its Section 5 table, full or
// banded (Section 3.2).
//
// Each request runs the plan a lone call would run (the same jobs in the
// same steps, Section 6.2: the cells of one anti-diagonal are independent).
// A worker thread owns the device side: at every engine step it admits
// queued requests in arrival order while their device state fits a first-fit
// pool in the caller's arena, then gathers the next plan step of every
// admitted request, in arrival order and up to the step cap, into one key
// switch launch and one blind-rotation launch on the engine's own stream.  A
// plan step's bootstraps are independent, so the last request taken may run
// part of its step and finish it in the next engine step; a step larger than
// one device round is trimmed to whole rounds.  A request moves to its next
// plan step only when every bootstrap of the current one has run, so its
// results are bit-identical to the lone call, alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"
#include "plan.h"
#include "pool.h"

namespace lvs {

namespace {

struct EngineRequest {
    uint64_t ticket = 0;
    QuerySpec spec;
    size_t bytes = 0, off = 0;   // state block in the pool
    Plan plan;
    size_t step = 0;             // next plan step
    size_t taken = 0;            // bootstraps of that step already run
    bool filled = false;         // the plan's Enc(1) rows written
    bool done = false;
};

// Pool bytes of a request: what lvs_plan_create would carve from its
// workspace for this query (V, the row state, eq1 and eq9).
size_t request_bytes(const QuerySpec& q) { return std::max<size_t>(query_buffer_bytes(q), 256); }

}  // namespace

struct Engine : Handle {
    Context* C = nullptr;
    int encoding = LVS_ENC_ASCII7;
    size_t max_step = 0;
    hipStream_t stream = nullptr;
    Job* d_jobs = nullptr;
    uint64_t* d_part = nullptr;
    uint8_t* pool_base = nullptr;
    Pool pool;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<EngineRequest*> queue;
    std::vector<EngineRequest*> active;
    std::map<uint64_t, std::unique_ptr<EngineRequest>> all;
    int error = LVS_OK;
    std::string error_msg;
    uint64_t steps = 0, bootstraps = 0;

    bool has_work() const {
        if (!queue.empty()) return true;
        for (const EngineRequest* r : active)
            if (!r->done) return true;
        return false;
    }

    // Skips empty plan steps; a request with no step left is done.
    static void settle(EngineRequest* r) {
        while (r->step < r->plan.steps.size() && r->plan.steps[r->step].count == 0) r->step++;
        if (r->step >= r->plan.steps.size()) r->done = true;
    }

    void fail(hipError_t e, const char* what) {
        error = LVS_E_DEVICE;
        error_msg = std::string("lvs engine: ") + what + ": " + hipGetErrorString(e);
        for (EngineRequest* r : active) r->done = true;
    }

    void run() {
        std::vector<Job> jobs;
        std::unique_lock<std::mutex> lk(mu);
        if (hipSetDevice(C->device) != hipSuccess) {
            fail(hipErrorInvalidDevice, "hipSetDevice");
            cv.notify_all();
        }
        for (;;) {
            cv.wait(lk, [&] { return stop || (error == LVS_OK && has_work()); });
            if (stop) return;
            try {
                step(lk, jobs);
            } catch (const std::exception& ex) {
                // host allocation while admitting or gathering: the engine
                // stops with a sticky error instead of ending the process
                if (!lk.owns_lock()) lk.lock();
                error = LVS_E_NOMEM_HOST;
                error_msg = std::string("lvs engine: ") + ex.what();
                for (EngineRequest* r : active) r->done = true;
                cv.notify_all();
            }
        }
    }

    // One engine step (called with mu held; returns with it held).
    void step(std::unique_lock<std::mutex>& lk, std::vector<Job>& jobs) {
        struct Take {
            EngineRequest* r;
            size_t count;
        };
        {
            // admission in arrival order while the request's state fits
            std::vector<EngineRequest*> fresh;
            while (!queue.empty()) {
                EngineRequest* r = queue.front();
                size_t off;
                if (!pool.alloc(r->bytes, &off)) break;
                r->off = off;
                uint8_t* ws = pool_base + off;
                std::vector<QuerySpec> one{r->spec};
                assign_buffers(one, ws);
                build_edit_distance_plan(one, r->plan);
                queue.pop_front();
                active.push_back(r);
                fresh.push_back(r);
            }
            // the next plan step of every admitted request, within the cap
            std::vector<Take> takes;
            jobs.clear();
            for (EngineRequest* r : active) {
                if (r->done || r->step >= r->plan.steps.size()) continue;
                if (jobs.size() >= max_step) break;
                const PlanStep& st = r->plan.steps[r->step];
                const size_t n = std::min(st.count - r->taken, max_step - jobs.size());
                jobs.insert(jobs.end(), r->plan.jobs.begin() + long(st.off + r->taken),
                            r->plan.jobs.begin() + long(st.off + r->taken + n));
                takes.push_back({r, n});
            }
            const size_t cus = size_t(std::max(1, C->cus));
            const size_t round = jobs.size() <= size_t(C->latency_form_max) ? cus : 2 * cus;
            if (jobs.size() > round) {
                size_t cut = jobs.size() % round;
                while (cut > 0 && !takes.empty()) {
                    Take& t = takes.back();
                    const size_t d = std::min(cut, t.count);
                    t.count -= d;
                    cut -= d;
                    jobs.resize(jobs.size() - d);
                    if (t.count == 0) takes.pop_back();
                }
            }
            lk.unlock();
            hipError_t e = hipSuccess;
            const char* what = "";
            for (EngineRequest* r : fresh) {
                for (const auto& f : r->plan.fills) {
                    if (e != hipSuccess) break;
                    e = launch_trivial(f.first, int(f.second), 1, stream);
                    what = "fill";
                }
            }
            if (e == hipSuccess && !jobs.empty()) {
                const int B = int(jobs.size());
                what = "upload";
                e = hipMemcpyAsync(d_jobs, jobs.data(), sizeof(Job) * jobs.size(), hipMemcpyHostToDevice, stream);
                if (e == hipSuccess) {
                    what = "key switch";
                    e = launch_keyswitch_jobs(d_jobs, B, C->ksk, d_part, stream, keyswitch_splits(B, C->ks_tile),
                                              C->ks_tile);
                }
                if (e == hipSuccess) {
                    what = "blind rotation";
                    e = launch_blind_rotate_jobs(d_jobs, B, d_part, C->luts, C->bsk, C->tables, C->br_grid,
                                                 C->latency_form_max, C->latency_waves, stream,
                                                 keyswitch_splits(B, C->ks_tile), C->throughput_waves);
                }
            }
            if (e == hipSuccess) {
                what = "synchronize";
                e = hipStreamSynchronize(stream);   // the job list is reused; results are final
            }
            lk.lock();
            if (e != hipSuccess) {
                fail(e, what);
                cv.notify_all();
                return;
            }
            for (EngineRequest* r : fresh) {
                r->filled = true;
                settle(r);
            }
            if (!jobs.empty()) {
                steps++;
                bootstraps += jobs.size();
            }
            for (const Take& t : takes) {
                EngineRequest* r = t.r;
                r->taken += t.count;
                if (r->taken < r->plan.steps[r->step].count) continue;
                r->taken = 0;
                r->step++;
                settle(r);
            }
            cv.notify_all();
        }
    }
};

}  // namespace lvs

using namespace lvs;

namespace {

Engine* as_engine(lvs_engine* e) {
    auto* h = reinterpret_cast<Engine*>(e);
    return (h && h->kind == kEngine) ? h : nullptr;
}

int engine_fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

}  // namespace

extern "C" {

size_t lvs_engine_fixed_bytes(size_t max_step) {
    return align256(sizeof(Job) * max_step) + align256(sizeof(uint64_t) * keyswitch_part_words(int(max_step)));
}

int lvs_engine_query_bytes(const lvs_query* q, int encoding, size_t* bytes) {
    if (!q || !bytes) return engine_fail(LVS_E_INVAL, "lvs_engine_query_bytes: NULL argument");
    std::vector<QuerySpec> qs;
    const int rc = make_query_specs(q, 1, encoding, LVS_REFRESH_MIN, qs);
    if (rc) return rc;
    *bytes = request_bytes(qs[0]);
    return LVS_OK;
}

int lvs_engine_create(lvs_context* ctx, int encoding, size_t max_step, void* d_arena, size_t arena_bytes,
                      lvs_engine** out) {
    auto* C = reinterpret_cast<Context*>(ctx);
    if (!C || C->kind != kContext || !out) return engine_fail(LVS_E_INVAL, "lvs_engine_create: bad argument");
    if (encoding != LVS_ENC_ASCII7 && encoding != LVS_ENC_DNA2)
        return engine_fail(LVS_E_INVAL, "lvs_engine_create: unknown encoding");
    if (max_step == 0 || max_step > kMaxStep) return engine_fail(LVS_E_INVAL, "lvs_engine_create: max_step out of range");
    const size_t fixed = lvs_engine_fixed_bytes(max_step);
    if (!d_arena || arena_bytes < fixed || reinterpret_cast<uintptr_t>(d_arena) % 256)
        return engine_fail(LVS_E_NOMEM_DEVICE, "lvs_engine_create: arena too small or misaligned");
    auto E = std::unique_ptr<Engine>(new (std::nothrow) Engine());
    if (!E) return engine_fail(LVS_E_NOMEM_HOST, "lvs_engine_create: out of host memory");
    E->kind = kEngine;
    E->C = C;
    E->encoding = encoding;
    E->max_step = max_step;
    uint8_t* arena = reinterpret_cast<uint8_t*>(d_arena);
    E->d_jobs = reinterpret_cast<Job*>(arena);
    E->d_part = reinterpret_cast<uint64_t*>(arena + align256(sizeof(Job) * max_step));
    E->pool_base = arena + fixed;
    E->pool.init(arena_bytes - fixed);
    hipError_t e = hipSetDevice(C->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking);
    if (e != hipSuccess)
        return engine_fail(LVS_E_DEVICE, std::string("lvs_engine_create: ") + hipGetErrorString(e));
    try {
        Engine* raw = E.get();
        E->worker = std::thread([raw] { raw->run(); });
    } catch (...) {
        (void)hipStreamDestroy(E->stream);
        return engine_fail(LVS_E_NOMEM_HOST, "lvs_engine_create: cannot start the worker thread");
    }
    *out = reinterpret_cast<lvs_engine*>(E.release());
    return LVS_OK;
}

int lvs_submit(lvs_engine* eng, const lvs_query* q, size_t nq, uint64_t* tickets) {
    Engine* E = as_engine(eng);
    if (!E || !tickets || (!q && nq)) return engine_fail(LVS_E_INVAL, "lvs_submit: bad argument");
    std::vector<QuerySpec> qs;
    const int rc = make_query_specs(q, nq, E->encoding, E->C->refresh_every, qs);
    if (rc) return rc;
    for (const QuerySpec& s : qs) {
        const int lr = check_query_lengths(E->C, s.m, s.n, "lvs_submit");
        if (lr) return lr;
        if (s.trace || s.eq1_out || s.eq9_out)
            return engine_fail(LVS_E_INVAL, "lvs_submit: d_trace / d_eq1 / d_eq9 are for batch plans only");
    }
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->error) return engine_fail(E->error, E->error_msg);
    for (const QuerySpec& s : qs)
        if (request_bytes(s) > E->pool.total())
            return engine_fail(LVS_E_NOMEM_DEVICE, "lvs_submit: a query can never fit in the engine's arena");
    std::vector<std::unique_ptr<EngineRequest>> made;
    for (QuerySpec& s : qs) {
        auto r = std::unique_ptr<EngineRequest>(new (std::nothrow) EngineRequest());
        if (!r) return engine_fail(LVS_E_NOMEM_HOST, "lvs_submit: out of host memory");
        r->spec = std::move(s);
        r->bytes = request_bytes(r->spec);
        made.push_back(std::move(r));
    }
    for (size_t k = 0; k < made.size(); ++k) {
        EngineRequest* r = made[k].get();
        r->ticket = E->next_ticket++;
        tickets[k] = r->ticket;
        E->queue.push_back(r);
        E->all[r->ticket] = std::move(made[k]);
    }
    E->cv.notify_all();
    return LVS_OK;
}

int lvs_poll(lvs_engine* eng, uint64_t ticket, int wait, int* done) {
    Engine* E = as_engine(eng);
    if (!E || !done) return engine_fail(LVS_E_INVAL, "lvs_poll: bad argument");
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->all.find(ticket);
    if (it == E->all.end()) return engine_fail(LVS_E_INVAL, "lvs_poll: unknown ticket");
    EngineRequest* r = it->second.get();
    if (wait) E->cv.wait(lk, [&] { return r->done || E->error != LVS_OK; });
    if (E->error) return engine_fail(E->error, E->error_msg);
    *done = r->done ? 1 : 0;
    if (!r->done) return LVS_OK;
    E->pool.release(r->off, r->bytes);
    E->active.erase(std::remove(E->active.begin(), E->active.end(), r), E->active.end());
    E->all.erase(it);
    return LVS_OK;
}

int lvs_engine_stats(lvs_engine* eng, uint64_t* steps, uint64_t* bootstraps, size_t* active, size_t* queued) {
    Engine* E = as_engine(eng);
    if (!E) return engine_fail(LVS_E_INVAL, "lvs_engine_stats: bad engine");
    std::lock_guard<std::mutex> lk(E->mu);
    if (steps) *steps = E->steps;
    if (bootstraps) *bootstraps = E->bootstraps;
    size_t na = 0;
    for (const EngineRequest* r : E->active) na += !r->done;
    if (active) *active = na;
    if (queued) *queued = E->queue.size();
    return LVS_OK;
}

void lvs_engine_free_impl(void* h) {
    auto* E = reinterpret_cast<Engine*>(h);
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->stop = true;
    }
    E->cv.notify_all();
    if (E->worker.joinable()) E->worker.join();
    if (E->stream) (void)hipStreamDestroy(E->stream);
    delete E;
}

}  // extern "C"
