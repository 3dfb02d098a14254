// Wide symbols (Section 4.2 of arXiv 2508.14568): the hybrid of the 4-bit
// subtraction equality with Algorithm 2's merging, for symbols of up to 64
// bits, and the edit distances built on it.
//
// A symbol of w bits is c = ceil(w / 4) ciphertexts of 4-bit chunks.  The
// equality of a pair is one plan: a step with the c sub-equality bootstraps
// of every pair, then per merging level a linear step (group sums) and a
// step with one bootstrap per group.  The edit distances run the same
// bootstraps inside the main loop instead, each diagonal's equality just in
// time for it (and earlier where a step has room), as Algorithm 4 runs the
// equality inside its loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"
#include "plan.h"

using namespace lvs;

namespace {

constexpr size_t W = kCtWords;

#define WIDE_FAIL(code, msg) \
    do {                     \
        set_error(msg);      \
        return (code);       \
    } while (0)

#define WIDE_HIP(expr)                                                                                  \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) WIDE_FAIL(LVS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

Context* ctx_of(lvs_context* c) {
    auto* h = reinterpret_cast<Context*>(c);
    return (h && h->kind == kContext) ? h : nullptr;
}

size_t chunks_of(unsigned width) { return (width >= 1 && width <= 64) ? (width + 3) / 4 : 0; }

uint32_t chunk_value(uint64_t v, size_t k) { return uint32_t((v >> (4 * k)) & 15u); }

// Both strings encrypted: pair p = i * n + j.
struct PairSrc {
    const uint64_t* A;
    const uint64_t* B;
    size_t n, c;
};
WideChunkInput pair_chunk(const void* ctx, size_t p, size_t k) {
    const auto* s = static_cast<const PairSrc*>(ctx);
    const size_t i = p / s->n, j = p % s->n;
    return {s->A + (i * s->c + k) * W, s->B + (j * s->c + k) * W, 0};
}

// Preprocessing: entry p = s * m + i against the cleartext alphabet[s].
struct TableSrc {
    const uint64_t* A;
    const uint64_t* alphabet;
    size_t m, c;
};
WideChunkInput table_chunk(const void* ctx, size_t p, size_t k) {
    const auto* s = static_cast<const TableSrc*>(ctx);
    const size_t sym = p / s->m, i = p % s->m;
    return {s->A + (i * s->c + k) * W, nullptr, chunk_value(s->alphabet[sym], k)};
}

int run(Context* C, Plan& P, uint8_t* ws) {
    WIDE_HIP(upload_plan(P, ws, C->stream));
    WIDE_HIP(run_plan(C, P));
    return LVS_OK;
}

// The main loop over an eq9 matrix (the same query form as
// lvs_edit_distance_eq9), with the refresh interval given.
QuerySpec eq9_query(const uint64_t* eq9, size_t m, size_t n, uint64_t* h_last, size_t refresh) {
    QuerySpec q;
    q.m = m;
    q.n = n;
    q.eq9_in = eq9 ? eq9 : reinterpret_cast<const uint64_t*>(16);
    q.h_last = h_last;
    q.refresh = refresh;
    return q;
}

// Several queries: query k's eq9 matrix starts at pair first[k].
struct MultiSrc {
    std::vector<size_t> first;     // first pair of every query, then the total
    std::vector<const uint64_t*> A, B;
    std::vector<size_t> n;
    size_t c;
};
// The queries of a wide plan; refresh is the interval the plan uses.
int wide_specs(const lvs_query* x, size_t nq, size_t refresh, std::vector<QuerySpec>& qs, MultiSrc& src,
               size_t c) {
    qs.assign(nq, QuerySpec());
    src.first.assign(1, 0);
    src.A.clear();
    src.B.clear();
    src.n.clear();
    src.c = c;
    for (size_t k = 0; k < nq; ++k) {
        const lvs_query& y = x[k];
        if (std::max(y.m, y.n) > size_t(LVS_MAX_LEN)) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide: string longer than LVS_MAX_LEN");
        if (y.d_table || (!y.d_a && y.m) || (!y.d_b && y.n))
            WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide: every query needs both strings encrypted");
        if (y.d_eq1 || y.d_eq9) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide: d_eq1 / d_eq9 are not kept for wide symbols");
        QuerySpec& s = qs[k];
        s.m = y.m;
        s.n = y.n;
        s.refresh = refresh;
        s.trace = y.d_trace;
        s.eq9_in = reinterpret_cast<const uint64_t*>(16);   // set once the workspace is carved
        if (y.banded) {
            s.band = long(std::min<size_t>(y.ell, y.m + y.n));
            s.path = y.d_path;
            if (!y.d_path && y.m + y.n) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide: NULL band path");
        } else {
            s.h_last = y.d_h_last;
            if (!y.d_h_last && y.n) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide: NULL result buffer");
        }
        src.A.push_back(y.d_a);
        src.B.push_back(y.d_b);
        src.n.push_back(std::max<size_t>(y.n, 1));
        src.first.push_back(src.first.back() + y.m * y.n);
    }
    return LVS_OK;
}

size_t wide_plan_bytes(const std::vector<QuerySpec>& qs, size_t pairs, size_t c) {
    size_t b = align256(sizeof(uint64_t) * std::max<size_t>(pairs, 1) * W) + wide_interleaved_bytes(pairs, c);
    size_t jobs = wide_jobs(pairs, c);
    for (const auto& q : qs) {
        b += query_buffer_bytes(q);
        jobs += query_jobs(q);
    }
    return b + plan_bytes(jobs, wide_step_bound(qs, c));
}

// The interleaved plan of qs (eq9 matrices carved from ws at first[k]).
void build_wide_plan(std::vector<QuerySpec>& qs, const MultiSrc& src, size_t c, size_t quantum, uint8_t*& ws,
                     Plan& P) {
    uint64_t* eq9 = reinterpret_cast<uint64_t*>(ws);
    ws += align256(sizeof(uint64_t) * std::max<size_t>(src.first.back(), 1) * W);
    std::vector<WideQuery> wq;
    for (size_t k = 0; k < qs.size(); ++k) {
        qs[k].eq9_in = eq9 + src.first[k] * W;
        wq.push_back({src.A[k], src.B[k], eq9 + src.first[k] * W});
    }
    assign_buffers(qs, ws);
    build_wide_edit_distance_plan(qs, wq, c, quantum, wide_step_bound(qs, c), ws, P);
}

}  // namespace

extern "C" {

size_t lvs_wide_chunks(unsigned width) { return chunks_of(width); }

size_t lvs_wide_pbs_per_pair(unsigned width) {
    const size_t c = chunks_of(width);
    return c ? wide_jobs(1, c) : 0;
}

int lvs_encrypt_symbols(const lvs_client_key* ck, const uint64_t* syms, size_t len, unsigned width, uint64_t seed,
                        uint64_t* h_out) {
    auto* c = reinterpret_cast<const ClientKey*>(ck);
    if (!c || c->kind != kClientKey || (!syms && len) || (!h_out && len))
        WIDE_FAIL(LVS_E_INVAL, "lvs_encrypt_symbols: bad argument");
    const size_t nc = chunks_of(width);
    if (!nc) WIDE_FAIL(LVS_E_INVAL, "lvs_encrypt_symbols: width must be 1..64");
    for (size_t i = 0; i < len; ++i)
        if (width < 64 && (syms[i] >> width))
            WIDE_FAIL(LVS_E_ALPHABET, "lvs_encrypt_symbols: symbol wider than width bits");
    for (size_t i = 0; i < len; ++i)
        for (size_t k = 0; k < nc; ++k) encrypt(*c, chunk_value(syms[i], k), seed, i * nc + k, h_out + (i * nc + k) * W);
    return LVS_OK;
}

size_t lvs_equality_wide_workspace_bytes(size_t m, size_t n, unsigned width) {
    const size_t c = chunks_of(width);
    return wide_buffer_bytes(m * n, c) + plan_bytes(wide_jobs(m * n, c), wide_max_step(m * n, c));
}

int lvs_equality_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, unsigned width,
                      uint64_t* d_eq9, void* d_work, size_t work_bytes) {
    Context* C = ctx_of(ctx);
    const size_t c = chunks_of(width);
    if (!C || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_equality_wide: bad context or width");
    if (m == 0 || n == 0) return LVS_OK;
    if (!d_a || !d_b || !d_eq9 || !d_work) WIDE_FAIL(LVS_E_INVAL, "lvs_equality_wide: NULL buffer");
    if (std::max(m, n) > size_t(LVS_MAX_LEN)) WIDE_FAIL(LVS_E_INVAL, "lvs_equality_wide: string longer than LVS_MAX_LEN");
    if (work_bytes < lvs_equality_wide_workspace_bytes(m, n, width))
        WIDE_FAIL(LVS_E_NOMEM_DEVICE, "lvs_equality_wide: workspace too small");
    WIDE_HIP(hipSetDevice(C->device));
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    const PairSrc src{d_a, d_b, n, c};
    Plan P;
    build_wide_equality(P, m * n, c, pair_chunk, &src, d_eq9, ws);
    return run(C, P, ws);
}

size_t lvs_edit_distance_wide_workspace_bytes(size_t m, size_t n, unsigned width) {
    const size_t c = chunks_of(width);
    const std::vector<QuerySpec> qs{eq9_query(nullptr, m, n, nullptr, LVS_REFRESH_MIN)};
    return wide_plan_bytes(qs, m * n, c);
}

int lvs_edit_distance_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n,
                           unsigned width, uint64_t* d_h_last, void* d_work, size_t work_bytes) {
    Context* C = ctx_of(ctx);
    const size_t c = chunks_of(width);
    if (!C || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_edit_distance_wide: bad context or width");
    if ((!d_a && m) || (!d_b && n) || (!d_h_last && n)) WIDE_FAIL(LVS_E_INVAL, "lvs_edit_distance_wide: NULL buffer");
    if (std::max(m, n) > size_t(LVS_MAX_LEN))
        WIDE_FAIL(LVS_E_INVAL, "lvs_edit_distance_wide: string longer than LVS_MAX_LEN");
    if (C->refresh_every == 0 && std::min(m, n) > size_t(LVS_MAX_DEPTH_NO_REFRESH))
        WIDE_FAIL(LVS_E_NOISE_BUDGET, "lvs_edit_distance_wide: min(m, n) exceeds the noise budget with refresh off");
    WIDE_HIP(hipSetDevice(C->device));
    if (n == 0) return LVS_OK;
    if (m == 0) {
        WIDE_HIP(launch_trivial(d_h_last, int(n), 1, C->stream));
        return LVS_OK;
    }
    if (!d_work || work_bytes < lvs_edit_distance_wide_workspace_bytes(m, n, width))
        WIDE_FAIL(LVS_E_NOMEM_DEVICE, "lvs_edit_distance_wide: workspace too small");
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    std::vector<QuerySpec> qs{eq9_query(nullptr, m, n, d_h_last, C->refresh_every)};
    MultiSrc src;
    src.first = {0, m * n};
    src.A = {d_a};
    src.B = {d_b};
    src.n = {n};
    src.c = c;
    Plan P;
    build_wide_plan(qs, src, c, size_t(std::max(1, C->cus)), ws, P);
    return run(C, P, ws);
}

int lvs_plan_wide_workspace_bytes(const lvs_query* queries, size_t nq, unsigned width, size_t* bytes) {
    const size_t c = chunks_of(width);
    if (!bytes || (!queries && nq) || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_wide_workspace_bytes: bad argument");
    std::vector<QuerySpec> qs;
    MultiSrc src;
    const int rc = wide_specs(queries, nq, LVS_REFRESH_MIN, qs, src, c);
    if (rc) return rc;
    *bytes = wide_plan_bytes(qs, src.first.back(), c);
    return LVS_OK;
}

int lvs_plan_create_wide(lvs_context* ctx, const lvs_query* queries, size_t nq, unsigned width, int flags,
                         void* d_work, size_t work_bytes, lvs_plan** out) {
    Context* C = ctx_of(ctx);
    const size_t c = chunks_of(width);
    if (!C || !out || (!queries && nq) || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_create_wide: bad argument");
    std::vector<QuerySpec> qs;
    MultiSrc src;
    int rc = wide_specs(queries, nq, C->refresh_every, qs, src, c);
    if (rc) return rc;
    for (const auto& q : qs)
        if (C->refresh_every == 0 && std::min(q.m, q.n) > size_t(LVS_MAX_DEPTH_NO_REFRESH))
            WIDE_FAIL(LVS_E_NOISE_BUDGET, "lvs_plan_create_wide: min(m, n) exceeds the noise budget with refresh off");
    const size_t pairs = src.first.back();
    if (!d_work || work_bytes < wide_plan_bytes(qs, pairs, c))
        WIDE_FAIL(LVS_E_NOMEM_DEVICE, "lvs_plan_create_wide: workspace too small");
    if (reinterpret_cast<uintptr_t>(d_work) % 256) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_create_wide: misaligned workspace");
    WIDE_HIP(hipSetDevice(C->device));
    auto* H = new (std::nothrow) PlanHandle();
    if (!H) WIDE_FAIL(LVS_E_NOMEM_HOST, "lvs_plan_create_wide: out of host memory");
    H->kind = kPlan;
    H->C = C;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    build_wide_plan(qs, src, c, size_t(std::max(1, C->cus)), ws, H->P);
    hipError_t e = upload_plan(H->P, ws, C->stream);
    if (e == hipSuccess && (flags & LVS_PLAN_GRAPH)) e = capture_plan(C, H->P);
    if (e != hipSuccess) {
        if (H->P.graph) (void)hipGraphExecDestroy(H->P.graph);
        delete H;
        WIDE_FAIL(LVS_E_DEVICE, std::string("lvs_plan_create_wide: ") + hipGetErrorString(e));
    }
    *out = reinterpret_cast<lvs_plan*>(H);
    return LVS_OK;
}

int lvs_plan_verify_wide(const lvs_query* queries, size_t nq, unsigned width, size_t round, size_t refresh,
                         size_t* steps, size_t* jobs, size_t* rounds, size_t* violations) {
    const size_t c = chunks_of(width);
    if ((!queries && nq) || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_plan_verify_wide: bad argument");
    if (refresh != 0 && (refresh < LVS_REFRESH_MIN || refresh > LVS_REFRESH_MAX))
        WIDE_FAIL(LVS_E_INVAL, "lvs_plan_verify_wide: bad refresh interval");
    std::vector<QuerySpec> qs;
    MultiSrc src;
    const int rc = wide_specs(queries, nq, refresh, qs, src, c);
    if (rc) return rc;
    // workspace buffers at addresses above every caller address; nothing is dereferenced
    uintptr_t top = 0;
    for (size_t k = 0; k < nq; ++k)
        for (uintptr_t a : {uintptr_t(queries[k].d_a), uintptr_t(queries[k].d_b), uintptr_t(queries[k].d_h_last),
                            uintptr_t(queries[k].d_path), uintptr_t(queries[k].d_trace)})
            top = std::max(top, a);
    uint8_t* ws = reinterpret_cast<uint8_t*>((top + (uintptr_t(1) << 40)) & ~uintptr_t(255));
    Plan P;
    build_wide_plan(qs, src, c, std::max<size_t>(round, 1), ws, P);
    size_t nr = 0;
    const size_t bad = verify_plan(P, round, wide_step_bound(qs, c), &nr);
    if (steps) *steps = P.steps.size();
    if (jobs) *jobs = P.jobs.size();
    if (rounds) *rounds = nr;
    if (violations) *violations = bad;
    return LVS_OK;
}

size_t lvs_preprocess_wide_workspace_bytes(size_t m, size_t alen, unsigned width) {
    return lvs_equality_wide_workspace_bytes(alen, m, width);
}

int lvs_preprocess_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, unsigned width, const uint64_t* alphabet,
                        size_t alen, uint64_t* d_table, void* d_work, size_t work_bytes) {
    Context* C = ctx_of(ctx);
    const size_t c = chunks_of(width);
    if (!C || !c) WIDE_FAIL(LVS_E_INVAL, "lvs_preprocess_wide: bad context or width");
    if (m == 0 || alen == 0) return LVS_OK;
    if (!d_a || !alphabet || !d_table || !d_work) WIDE_FAIL(LVS_E_INVAL, "lvs_preprocess_wide: NULL buffer");
    if (m > size_t(LVS_MAX_LEN)) WIDE_FAIL(LVS_E_INVAL, "lvs_preprocess_wide: string longer than LVS_MAX_LEN");
    for (size_t s = 0; s < alen; ++s)
        if (width < 64 && (alphabet[s] >> width))
            WIDE_FAIL(LVS_E_ALPHABET, "lvs_preprocess_wide: alphabet symbol wider than width bits");
    if (work_bytes < lvs_preprocess_wide_workspace_bytes(m, alen, width))
        WIDE_FAIL(LVS_E_NOMEM_DEVICE, "lvs_preprocess_wide: workspace too small");
    WIDE_HIP(hipSetDevice(C->device));
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    const TableSrc src{d_a, alphabet, m, c};
    Plan P;
    build_wide_equality(P, alen * m, c, table_chunk, &src, d_table, ws);
    return run(C, P, ws);
}

}  // extern "C"
