// Serving: continuous batching of encrypted name queries against a cleartext
// list of names (Section 5's setting of one encrypted query against a large
// cleartext database: preprocess the query once, then one bootstrap per cell
// for every name).
//
// Each request goes through three phases: the preprocessing table's two
// bootstrap rounds (eq1, then eq9 = T[c][i]; over wide symbols, Section
// 4.2, the chunk sub-equalities and one round per merging level, each level's
// group sums run just before its round), then the anti-diagonals
// s = 2 .. m + max(n_k) of one DP instance per name, all instances of the
// request advancing together, with a refresh round (Section 3.1) after every
// refresh-th diagonal.  An engine step gathers the ready bootstraps of
// the admitted requests in arrival order (any mix of phases and tables, the
// last one possibly with part of its round, the step trimmed to whole device
// rounds) into one key-switch launch and one blind-rotation launch.
// Requests are admitted in
// arrival order when their device buffers fit in the caller's arena, and join
// at the next step boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"
#include "plan.h"
#include "pool.h"

namespace lvs {

namespace {

constexpr size_t W = kCtWords;
constexpr uint64_t kOne = uint64_t(1) << kDeltaLog;

enum Phase { kQueued, kPre1, kPre2, kPreWide, kDp, kDone };

struct Request {
    uint64_t ticket = 0;
    size_t m = 0;
    std::vector<uint64_t> host_query;   // [m][2][W] until admitted
    Phase phase = kQueued;
    size_t s = 2;                        // current anti-diagonal in the DP phase
    bool refreshing = false;             // the round refreshes the differences of diagonal s
    size_t off = 0, bytes = 0;           // block in the pool
    uint64_t* A = nullptr;               // [m][2][W]
    uint64_t* eq1 = nullptr;             // [alen][m][W]
    uint64_t* T = nullptr;               // [alen][m][W]
    uint64_t* V = nullptr;               // [names][m+1][W]
    uint64_t* H = nullptr;               // [sum n_k][W] results
    // wide symbols: the table's equality plan (jobs point into the block) and
    // the next of its steps to run
    Plan pre;
    size_t pre_step = 0;
    // bootstraps of the current phase already run (a phase's bootstraps are
    // independent, so a step may run part of them), and the phase's jobs,
    // generated when its first part is taken
    size_t taken = 0;
    std::vector<Job> phase_jobs;
    const SumOp* phase_sum = nullptr;
};

// Pool bytes of one request: the query, the preprocessing buffers (ASCII: the
// eq1 table; wide: the merging levels), the table T, one DP frontier per name
// and the result rows.
size_t request_block_bytes(size_t m, size_t alen, size_t c, size_t n_names, size_t total_len) {
    const size_t qsyms = c ? c : 2;
    const size_t pre = c ? wide_buffer_bytes(alen * m, c) : align256(sizeof(uint64_t) * alen * m * W);
    return align256(sizeof(uint64_t) * m * qsyms * W) + pre + align256(sizeof(uint64_t) * alen * m * W) +
           align256(sizeof(uint64_t) * n_names * (m + 1) * W) + align256(sizeof(uint64_t) * total_len * W);
}

// Table entry p = sym * m + i of a wide request against the alphabet.
struct WideTableSrc {
    const uint64_t* A;
    const uint64_t* alphabet;
    size_t m, c;
};
WideChunkInput wide_table_chunk(const void* ctx, size_t p, size_t k) {
    const auto* s = static_cast<const WideTableSrc*>(ctx);
    const size_t sym = p / s->m, i = p % s->m;
    return {s->A + (i * s->c + k) * W, nullptr, uint32_t((s->alphabet[sym] >> (4 * k)) & 15u)};
}

}  // namespace

struct Server : Handle {
    Context* C = nullptr;
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    size_t max_step = 0;
    // names
    std::vector<size_t> name_len, name_start;  // first result row of every name
    std::vector<int32_t> cols;                 // concatenated alphabet index of every name symbol
    size_t total_len = 0, max_len = 0;
    size_t refresh = 0;                        // noise-refresh interval (anti-diagonals, 0: off)
    std::vector<uint8_t> sym_lo, sym_hi;       // alphabet symbols (4-bit, 3-bit)
    size_t alen = 0;
    size_t c = 0;                              // chunks of a wide symbol (0: ASCII)
    std::vector<uint64_t> alpha_wide;          // wide alphabet
    // device regions
    Job* d_jobs = nullptr;
    uint64_t* d_part = nullptr;
    Pool pool;
    uint8_t* pool_base = nullptr;
    // requests
    uint64_t next_ticket = 1;
    std::deque<Request*> queue;                // arrival order, not admitted yet
    std::vector<Request*> active;              // admitted, arrival order
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Job> jobs;
    uint64_t steps = 0, bootstraps = 0;

    size_t query_syms() const { return c ? c : 2; }

    size_t request_bytes(size_t m) const { return request_block_bytes(m, alen, c, name_len.size(), total_len); }

    void carve(Request* r) {
        uint8_t* p = pool_base + r->off;
        const size_t m = r->m;
        r->A = reinterpret_cast<uint64_t*>(p);
        p += align256(sizeof(uint64_t) * m * query_syms() * W);
        if (c) {
            // the merging levels, then T, which the plan's last round writes
            uint8_t* levels = p;
            p += wide_buffer_bytes(alen * m, c);
            r->T = reinterpret_cast<uint64_t*>(p);
            const WideTableSrc src{r->A, alpha_wide.data(), m, c};
            r->pre = Plan();
            r->pre_step = 0;
            build_wide_equality(r->pre, alen * m, c, wide_table_chunk, &src, r->T, levels);
        } else {
            r->eq1 = reinterpret_cast<uint64_t*>(p);
            p += align256(sizeof(uint64_t) * alen * m * W);
            r->T = reinterpret_cast<uint64_t*>(p);
        }
        p += align256(sizeof(uint64_t) * alen * m * W);
        r->V = reinterpret_cast<uint64_t*>(p);
        p += align256(sizeof(uint64_t) * name_len.size() * (m + 1) * W);
        r->H = reinterpret_cast<uint64_t*>(p);
    }

    // Jobs of one request's current phase; *sum receives the group sums
    // that must run before them (wide merging levels), if any.
    void gather(Request* r, std::vector<Job>& out, const SumOp** sum) const {
        const size_t m = r->m;
        *sum = nullptr;
        if (r->phase == kPreWide) {
            const PlanStep* st = &r->pre.steps[r->pre_step];
            if (st->sum >= 0) {
                *sum = &r->pre.sums[size_t(st->sum)];
                st = &r->pre.steps[r->pre_step + 1];
            }
            out.insert(out.end(), r->pre.jobs.begin() + long(st->off), r->pre.jobs.begin() + long(st->off + st->count));
            return;
        }
        if (r->phase == kPre1 || r->phase == kPre2) {
            for (size_t a = 0; a < alen; ++a)
                for (size_t i = 0; i < m; ++i) {
                    Job J{};
                    if (r->phase == kPre1) {     // z1 = x1 - c1, eq1 = PBS(z1; LUT_eq)
                        J.src[0] = r->A + (i * 2) * W;
                        J.coef[0] = 1;
                        J.delta = uint64_t(0) - uint64_t(sym_lo[a]) * kOne;
                        J.lut = LVS_LUT_EQ;
                        J.dst[0] = r->eq1 + (a * m + i) * W;
                    } else {                     // z2 = 2 (x2 - c2) + 1 - eq1, T = PBS(z2; LUT_eq9)
                        J.src[0] = r->A + (i * 2 + 1) * W;
                        J.src[1] = r->eq1 + (a * m + i) * W;
                        J.coef[0] = 2;
                        J.coef[1] = -1;
                        J.delta = kOne - 2 * uint64_t(sym_hi[a]) * kOne;
                        J.lut = LVS_LUT_EQ9;
                        J.dst[0] = r->T + (a * m + i) * W;
                    }
                    out.push_back(J);
                }
            return;
        }
        // DP: every name's cells (i, s - i) on anti-diagonal s
        const size_t s = r->s;
        for (size_t k = 0; k < name_len.size(); ++k) {
            const size_t n = name_len[k];
            if (n == 0 || s > m + n) continue;
            uint64_t* V = r->V + k * (m + 1) * W;
            uint64_t* H = r->H + name_start[k] * W - W;     // H[j] = h[latest i, j], j >= 1
            const int32_t* col = cols.data() + name_start[k];
            const size_t i_lo = (s > n + 1) ? s - n : 1;
            const size_t i_hi = std::min(m, s - 1);
            if (r->refreshing) {
                // the v and h written on diagonal s, in place through the identity table
                if (s >= m + n) continue;
                for (size_t i = i_lo; i <= i_hi; ++i)
                    for (uint64_t* x : {V + i * W, H + (s - i) * W}) {
                        Job J{};
                        J.src[0] = x;
                        J.coef[0] = 1;
                        J.lut = LVS_LUT_REFRESH;
                        J.dst[2] = x;
                        out.push_back(J);
                    }
                continue;
            }
            for (size_t i = i_lo; i <= i_hi; ++i) {
                const size_t j = s - i;
                const uint64_t* v_in = (j == 1) ? nullptr : V + i * W;
                const uint64_t* h_in = (i == 1) ? nullptr : H + j * W;
                Job J{};
                J.src[0] = v_in;
                J.src[1] = h_in;
                J.src[2] = r->T + (size_t(col[j - 1]) * m + (i - 1)) * W;
                J.coef[0] = -1;
                J.coef[1] = 3;
                J.coef[2] = 1;
                J.delta = 4 * kOne - (v_in ? 0 : kOne) + (h_in ? 0 : 3 * kOne);
                J.lut = LVS_LUT_MIN;
                J.dst[0] = V + i * W;
                J.sub[0] = h_in;
                J.sub_delta[0] = h_in ? 0 : kOne;
                J.dst[1] = H + j * W;
                J.sub[1] = v_in;
                J.sub_delta[1] = v_in ? 0 : kOne;
                out.push_back(J);
            }
        }
    }

    void advance(Request* r) const {
        if (r->phase == kPreWide) {
            r->pre_step += (r->pre.steps[r->pre_step].sum >= 0) ? 2 : 1;
            if (r->pre_step >= r->pre.steps.size()) {
                r->pre = Plan();
                r->phase = kDp;
                r->s = 2;
            }
        } else if (r->phase == kPre1) r->phase = kPre2;
        else if (r->phase == kPre2) { r->phase = kDp; r->s = 2; }
        else if (r->phase == kDp) {
            // a refresh round follows diagonal s when some name still has cells past it
            if (!r->refreshing && refresh > 0 && r->s % refresh == 0 && r->s < r->m + max_len) {
                r->refreshing = true;
                return;
            }
            r->refreshing = false;
            r->s++;
            if (r->s > r->m + max_len) r->phase = kDone;
        }
    }
};

}  // namespace lvs

using namespace lvs;

namespace {

thread_local std::string g_srv_error;

Server* as_srv(lvs_server* s) {
    auto* h = reinterpret_cast<Server*>(s);
    return (h && h->kind == kServer) ? h : nullptr;
}

#define SRV_FAIL(code, msg)   \
    do {                      \
        set_error(msg);       \
        return (code);        \
    } while (0)

#define SRV_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) SRV_FAIL(LVS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

size_t lvs_server_fixed_bytes(size_t max_step) {
    return align256(sizeof(Job) * max_step) + align256(sizeof(uint64_t) * keyswitch_part_words(int(max_step)));
}

size_t lvs_server_request_bytes(const uint8_t* names, const size_t* name_lens, size_t n_names, size_t alen,
                                size_t m) {
    (void)names;
    size_t total = 0;
    for (size_t k = 0; k < n_names; ++k) total += name_lens[k];
    return request_block_bytes(m, alen, 0, n_names, total);
}

size_t lvs_server_request_bytes_wide(const size_t* name_lens, size_t n_names, size_t alen, size_t m,
                                     unsigned width) {
    if (width < 1 || width > 64) return 0;
    size_t total = 0;
    for (size_t k = 0; k < n_names; ++k) total += name_lens[k];
    return request_block_bytes(m, alen, (width + 3) / 4, n_names, total);
}

}  // extern "C"

namespace {

// The part of server creation shared by the ASCII and the wide form: checks,
// arena layout and the name table (every name symbol's alphabet index).
template <typename Sym>
int create_server(lvs_context* ctx, const Sym* names, const size_t* name_lens, size_t n_names, const Sym* alphabet,
                  size_t alen, size_t max_step, void* d_arena, size_t arena_bytes, size_t chunks, const char* fn,
                  lvs_server** out) {
    auto* C = reinterpret_cast<Context*>(ctx);
    if (!C || C->kind != kContext || !out || (!names && n_names) || (!name_lens && n_names) || !alphabet || !alen)
        SRV_FAIL(LVS_E_INVAL, std::string(fn) + ": bad argument");
    if (max_step == 0 || max_step > kMaxStep) SRV_FAIL(LVS_E_INVAL, std::string(fn) + ": max_step out of range");
    const size_t fixed = lvs_server_fixed_bytes(max_step);
    if (!d_arena || arena_bytes < fixed || reinterpret_cast<uintptr_t>(d_arena) % 256)
        SRV_FAIL(LVS_E_NOMEM_DEVICE, std::string(fn) + ": arena too small or misaligned");
    auto S = std::unique_ptr<Server>(new (std::nothrow) Server());
    if (!S) SRV_FAIL(LVS_E_NOMEM_HOST, std::string(fn) + ": out of host memory");
    S->kind = kServer;
    S->C = C;
    S->arena = reinterpret_cast<uint8_t*>(d_arena);
    S->arena_bytes = arena_bytes;
    S->max_step = max_step;
    S->refresh = C->refresh_every;
    S->alen = alen;
    S->c = chunks;
    if (chunks) {
        S->alpha_wide.assign(alphabet, alphabet + alen);
    } else {
        for (size_t a = 0; a < alen; ++a) {
            S->sym_lo.push_back(uint8_t(alphabet[a] & 15));
            S->sym_hi.push_back(uint8_t(alphabet[a] >> 4));
        }
    }
    size_t pos = 0;
    for (size_t k = 0; k < n_names; ++k) {
        const size_t n = name_lens[k];
        if (n > 4096) SRV_FAIL(LVS_E_INVAL, std::string(fn) + ": name longer than 4096");
        S->name_len.push_back(n);
        S->name_start.push_back(S->total_len);
        for (size_t j = 0; j < n; ++j) {
            const Sym* hit = std::find(alphabet, alphabet + alen, names[pos + j]);
            if (hit == alphabet + alen) SRV_FAIL(LVS_E_ALPHABET, std::string(fn) + ": name symbol not in the alphabet");
            S->cols.push_back(int32_t(hit - alphabet));
        }
        pos += n;
        S->total_len += n;
        S->max_len = std::max(S->max_len, n);
    }
    S->d_jobs = reinterpret_cast<Job*>(S->arena);
    S->d_part = reinterpret_cast<uint64_t*>(S->arena + align256(sizeof(Job) * max_step));
    S->pool_base = S->arena + fixed;
    S->pool.init(arena_bytes - fixed);
    *out = reinterpret_cast<lvs_server*>(S.release());
    return LVS_OK;
}

}  // namespace

extern "C" {

int lvs_server_create(lvs_context* ctx, const uint8_t* names, const size_t* name_lens, size_t n_names,
                      const uint8_t* alphabet, size_t alen, size_t max_step, void* d_arena, size_t arena_bytes,
                      lvs_server** out) {
    for (size_t a = 0; alphabet && a < alen; ++a)
        if (alphabet[a] >= 128) SRV_FAIL(LVS_E_ALPHABET, "lvs_server_create: alphabet symbol >= 128");
    return create_server(ctx, names, name_lens, n_names, alphabet, alen, max_step, d_arena, arena_bytes, 0,
                         "lvs_server_create", out);
}

int lvs_server_create_wide(lvs_context* ctx, const uint64_t* names, const size_t* name_lens, size_t n_names,
                           const uint64_t* alphabet, size_t alen, unsigned width, size_t max_step, void* d_arena,
                           size_t arena_bytes, lvs_server** out) {
    if (width < 1 || width > 64) SRV_FAIL(LVS_E_INVAL, "lvs_server_create_wide: width must be 1..64");
    for (size_t a = 0; alphabet && a < alen; ++a)
        if (width < 64 && (alphabet[a] >> width))
            SRV_FAIL(LVS_E_ALPHABET, "lvs_server_create_wide: alphabet symbol wider than width bits");
    return create_server(ctx, names, name_lens, n_names, alphabet, alen, max_step, d_arena, arena_bytes,
                         (width + 3) / 4, "lvs_server_create_wide", out);
}

int lvs_server_submit(lvs_server* srv, const uint64_t* h_query, size_t m, uint64_t* ticket) {
    Server* S = as_srv(srv);
    if (!S || !ticket || (!h_query && m)) SRV_FAIL(LVS_E_INVAL, "lvs_server_submit: bad argument");
    if (m == 0 || m > 4096) SRV_FAIL(LVS_E_INVAL, "lvs_server_submit: query length must be 1..4096");
    if (S->refresh == 0 && std::min(m, S->max_len) > size_t(LVS_MAX_DEPTH_NO_REFRESH))
        SRV_FAIL(LVS_E_NOISE_BUDGET, "lvs_server_submit: min(m, name length) exceeds the noise budget with refresh off");
    if (S->request_bytes(m) > S->pool.total())
        SRV_FAIL(LVS_E_NOMEM_DEVICE, "lvs_server_submit: the request can never fit in the arena");
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!r) SRV_FAIL(LVS_E_NOMEM_HOST, "lvs_server_submit: out of host memory");
    r->ticket = S->next_ticket++;
    r->m = m;
    r->host_query.assign(h_query, h_query + m * S->query_syms() * W);
    S->queue.push_back(r.get());
    *ticket = r->ticket;
    S->all[r->ticket] = std::move(r);
    return LVS_OK;
}

int lvs_server_step(lvs_server* srv, size_t* active, size_t* queued, size_t* step_jobs) {
    Server* S = as_srv(srv);
    if (!S) SRV_FAIL(LVS_E_INVAL, "lvs_server_step: bad server");
    Context* C = S->C;
    SRV_HIP(hipSetDevice(C->device));
    // admission in arrival order while the request's buffers fit
    while (!S->queue.empty()) {
        Request* r = S->queue.front();
        size_t off;
        if (!S->pool.alloc(S->request_bytes(r->m), &off)) break;
        r->off = off;
        r->bytes = S->request_bytes(r->m);
        S->carve(r);
        SRV_HIP(hipMemcpyAsync(r->A, r->host_query.data(), r->host_query.size() * 8, hipMemcpyHostToDevice,
                               C->stream));
        r->phase = S->c ? kPreWide : kPre1;
        S->queue.pop_front();
        S->active.push_back(r);
    }
    // gather the admitted requests' ready bootstraps in arrival order, within
    // the step cap; the last request may contribute part of its phase
    struct Take {
        Request* r;
        size_t count, total;
        const SumOp* sum;
    };
    std::vector<Take> takes;
    S->jobs.clear();
    for (Request* r : S->active) {
        if (r->phase == kDone) continue;
        if (S->jobs.size() >= S->max_step) break;
        if (r->taken == 0) {                 // a new phase (or one no step has run yet)
            r->phase_jobs.clear();
            S->gather(r, r->phase_jobs, &r->phase_sum);
        }
        const size_t total = r->phase_jobs.size();
        const size_t n = std::min(total - r->taken, S->max_step - S->jobs.size());
        S->jobs.insert(S->jobs.end(), r->phase_jobs.begin() + long(r->taken),
                       r->phase_jobs.begin() + long(r->taken + n));
        takes.push_back({r, n, total, r->taken == 0 ? r->phase_sum : nullptr});
    }
    // end the step on a whole device round (one bootstrap per CU, two in the
    // four-wave form): the bootstraps of a partial last round wait for the
    // next step, taken off the latest requests
    const size_t cus = size_t(std::max(1, C->cus));
    const size_t round = S->jobs.size() <= size_t(C->latency_form_max) ? cus : 2 * cus;
    if (S->jobs.size() > round) {
        size_t cut = S->jobs.size() % round;
        while (cut > 0 && !takes.empty()) {
            Take& t = takes.back();
            const size_t d = std::min(cut, t.count);
            t.count -= d;
            cut -= d;
            S->jobs.resize(S->jobs.size() - d);
            if (t.count == 0) takes.pop_back();
        }
    }
    // the merging levels' group sums feed this step's bootstraps (once, with
    // the first part of their round)
    for (const Take& t : takes)
        if (t.sum)
            SRV_HIP(launch_group_sum(t.sum->in, t.sum->out, t.sum->items, t.sum->cnt, t.sum->groups, t.sum->group,
                                     C->cus, C->stream));
    if (!S->jobs.empty()) {
        const int B = int(S->jobs.size());
        SRV_HIP(hipMemcpyAsync(S->d_jobs, S->jobs.data(), sizeof(Job) * S->jobs.size(), hipMemcpyHostToDevice,
                               C->stream));
        {
            TimedLaunch t(C, kProfKeySwitch, uint64_t(B));
            SRV_HIP(launch_keyswitch_jobs(S->d_jobs, B, C->ksk, S->d_part, C->stream, keyswitch_splits(B, C->ks_tile),
                                          C->ks_tile));
        }
        {
            TimedLaunch t(C, br_profile_id(C, B), uint64_t(B));
            SRV_HIP(launch_blind_rotate_jobs(S->d_jobs, B, S->d_part, C->luts, C->bsk, C->tables, C->br_grid,
                                             C->latency_form_max, C->latency_waves, C->stream,
                                             keyswitch_splits(B, C->ks_tile), C->throughput_waves));
        }
        SRV_HIP(hipStreamSynchronize(C->stream));   // the job list is reused by the next step
        S->steps++;
        S->bootstraps += S->jobs.size();
    }
    for (const Take& t : takes) {
        t.r->taken += t.count;
        if (t.r->taken < t.total) continue;
        t.r->taken = 0;
        S->advance(t.r);
    }
    // requests with no name work left are done as well
    for (Request* r : S->active)
        if (r->phase == kDp && r->s > r->m + S->max_len) r->phase = kDone;
    size_t na = 0;
    for (Request* r : S->active) na += (r->phase != kDone);
    if (active) *active = na;
    if (queued) *queued = S->queue.size();
    if (step_jobs) *step_jobs = S->jobs.size();
    return LVS_OK;
}

int lvs_server_poll(lvs_server* srv, uint64_t ticket, uint64_t* h_out, int* done) {
    Server* S = as_srv(srv);
    if (!S || !done) SRV_FAIL(LVS_E_INVAL, "lvs_server_poll: bad argument");
    auto it = S->all.find(ticket);
    if (it == S->all.end()) SRV_FAIL(LVS_E_INVAL, "lvs_server_poll: unknown ticket");
    Request* r = it->second.get();
    *done = r->phase == kDone;
    if (!*done || !h_out) return LVS_OK;
    SRV_HIP(hipSetDevice(S->C->device));
    SRV_HIP(hipMemcpy(h_out, r->H, sizeof(uint64_t) * S->total_len * W, hipMemcpyDeviceToHost));
    S->pool.release(r->off, r->bytes);
    S->active.erase(std::remove(S->active.begin(), S->active.end(), r), S->active.end());
    S->all.erase(it);
    return LVS_OK;
}

int lvs_server_stats(const lvs_server* srv, uint64_t* steps, uint64_t* bootstraps) {
    auto* S = reinterpret_cast<const Server*>(srv);
    if (!S || S->kind != kServer) SRV_FAIL(LVS_E_INVAL, "lvs_server_stats: bad server");
    if (steps) *steps = S->steps;
    if (bootstraps) *bootstraps = S->bootstraps;
    return LVS_OK;
}

void lvs_server_free_impl(void* h) { delete reinterpret_cast<Server*>(h); }

}  // extern "C"
