// Static bootstrap schedules ("plans") shared by the plain, batched and
// serving paths.
#pragma once

#include <hip/hip_runtime_api.h>

#include <vector>

#include "launch.h"
#include "lvs_internal.h"

namespace lvs {

constexpr size_t kMaxStep = 65536;   // bootstraps per launch

struct Context;

// One edit distance of a plan.
struct QuerySpec {
    int encoding = LVS_ENC_ASCII7;
    const uint64_t* A = nullptr;   // [m][nsym][W] encrypted string a
    size_t m = 0;
    const uint64_t* B = nullptr;   // [n][nsym][W] encrypted string b (both encrypted)
    size_t n = 0;
    const uint64_t* table = nullptr;        // [alen][m][W] preprocessing table (cleartext b)
    std::vector<int32_t> cols;              // table row of b_j (cleartext b)
    const uint64_t* eq9_in = nullptr;       // [m][n][W] given equality matrix (Algorithm 1)
    uint64_t* h_last = nullptr;             // [n][W] result; doubles as H[1..n]
    uint64_t* trace = nullptr;              // optional [m][n][W] record of every M
    uint64_t* eq1_out = nullptr;            // optional caller buffers for eq1 / eq9 (both encrypted):
    uint64_t* eq9_out = nullptr;            //   used instead of workspace when set
    // Algorithm 1's band (Section 3.2): only cells with |i - j| <= band are
    // bootstrapped (band < 0: every cell); the result is then the m + n
    // differences of the diagonal path, written to path ([m+n][W]).
    long band = -1;
    uint64_t* path = nullptr;
    // Section 3.1's noise refresh: the v and h written on anti-diagonals
    // s = refresh, 2 refresh, ... (s < m + n) are bootstrapped again through
    // the identity table before diagonal s + 1 reads them (0: never).
    size_t refresh = 0;
    // workspace buffers assigned by assign_buffers()
    uint64_t* V = nullptr;                  // [m+1][W]
    uint64_t* eq1 = nullptr;                // [m][n][W] (ASCII, both encrypted)
    uint64_t* eq9 = nullptr;                // [m][n][W] (both encrypted)
    uint64_t* H = nullptr;                  // [n][W] row state when there is no h_last (band)
};

// Whether cell (i, j) (1-based) is bootstrapped.
inline bool in_band(const QuerySpec& q, size_t i, size_t j) {
    return q.band < 0 || (i > j ? i - j : j - i) <= size_t(q.band);
}

// Cells of an m x n matrix with |i - j| <= band (every cell if band < 0).
size_t band_cells(size_t m, size_t n, long band);

// Cells of anti-diagonal s (i + j = s) that the query bootstraps.
size_t diagonal_cells(const QuerySpec& q, size_t s);

// Whether the differences written on anti-diagonal s are refreshed.
inline bool refresh_due(const QuerySpec& q, size_t s) {
    return q.refresh > 0 && s >= 2 && s % q.refresh == 0 && s < q.m + q.n;
}

// A step is a batch of bootstraps (jobs off .. off + count), or, with
// sum >= 0, the linear group sums Plan::sums[sum].
struct PlanStep {
    size_t off, count;
    int sum = -1;
};

// Linear step: out[item][g] = sum of in[item][k] over the g-th group of
// `group` consecutive k < cnt (launch_group_sum).
struct SumOp {
    const uint64_t* in;
    uint64_t* out;
    size_t items;
    int cnt, groups, group;
};

struct Plan {
    std::vector<std::pair<uint64_t*, size_t>> fills;   // rows set to Enc(1) at the start of every run
    std::vector<Job> jobs;
    std::vector<PlanStep> steps;
    std::vector<SumOp> sums;
    size_t max_step = 0;
    Job* d_jobs = nullptr;
    uint64_t* d_part = nullptr;
    hipGraphExec_t graph = nullptr;
    size_t pbs() const { return jobs.size(); }
};

// A plan handle of the C ABI (lvs_plan): the context it runs on and the plan.
struct PlanHandle : Handle {
    Context* C = nullptr;
    Plan P;
};

// Bytes of per-query workspace (V, eq1, eq9) and of a plan's jobs/partials.
size_t query_buffer_bytes(const QuerySpec& q);
size_t plan_bytes(size_t njobs, size_t max_step);
size_t align256(size_t x);

// Bootstraps a query contributes and its largest step.
size_t query_jobs(const QuerySpec& q);

// Carves V / eq1 / eq9 of every query from ws (advancing it).
void assign_buffers(std::vector<QuerySpec>& qs, uint8_t*& ws);

// Builds the jobs: equality steps (both encrypted), then one step per
// anti-diagonal s = 2 .. max(m + n) holding every query's cells on it, each
// followed by a refresh step when some query's refresh is due after it.
// quantum: bootstraps the device runs at once (0: no filling); cap: the
// largest step the workspace was sized for.  step_diag, if given, receives
// per main-loop step its anti-diagonal t, or -t - 1 for the refresh step
// after diagonal t.
void build_edit_distance_plan(const std::vector<QuerySpec>& qs, Plan& P, bool with_dp = true, size_t quantum = 0,
                              size_t cap = 0, std::vector<long>* step_diag = nullptr);

// Jobs of the Section 5 table: T[c][i] = Enc(9 [a_i = S_c]).
void build_preprocess_plan(const uint64_t* A, size_t m, int encoding, const std::vector<uint8_t>& syms_lo,
                           const std::vector<uint8_t>& syms_hi, uint64_t* table, uint64_t* eq1, Plan& P);

// Independent bootstraps d_out[b] = PBS(d_in[b]).
void build_pbs_plan(const uint64_t* in, const uint8_t* lut_ids, int lut, size_t B, uint64_t* out, Plan& P);

// Section 4.2's hybrid equality of `pairs` symbol pairs of c 4-bit chunks:
// chunk_input(p, k) returns a job whose inputs form x_k - y_k of pair p; the
// result Enc(9 [x = y]) of pair p goes to out + p * W.  ws is advanced past
// the level buffers (wide_buffer_bytes).
struct WideChunkInput {
    const uint64_t* a;      // encrypted chunk of x
    const uint64_t* b;      // encrypted chunk of y, or null: y_k is `clear`
    uint32_t clear;
};
size_t wide_buffer_bytes(size_t pairs, size_t c);
size_t wide_jobs(size_t pairs, size_t c);
size_t wide_max_step(size_t pairs, size_t c);
void build_wide_equality(Plan& P, size_t pairs, size_t c, WideChunkInput (*chunk)(const void*, size_t, size_t),
                         const void* ctx, uint64_t* out, uint8_t*& ws);

// Wide-symbol edit distances as one plan: the hybrid equality of every
// in-band pair interleaved with the main loop.  qs are main-loop queries
// (eq9_in = wq[k].eq9, buffers assigned); wq[k] gives query k's chunk
// ciphertexts ([m][c][W], [n][c][W]) and its writable eq9 matrix.  Slot t
// runs the cells of anti-diagonal t; diagonal s's chunk sub-equalities run by
// slot s - 1 - levels, merging level l at slot s - 1 - levels + l (group
// sums first), so its eq9 is ready at slot s - 1.  quantum > 0 fills each
// slot's last partial device round with chunk sub-equalities of later
// diagonals, never past cap (0: no bound); no step exceeds
// wide_step_bound(qs, c) when cap is that bound.  ws is advanced past the
// level buffers (wide_interleaved_bytes(pairs, c), pairs = every query's m n
// at most).
struct WideQuery {
    const uint64_t* A;
    const uint64_t* B;
    uint64_t* eq9;
};
size_t wide_levels(size_t c);
size_t wide_interleaved_bytes(size_t pairs, size_t c);
size_t wide_step_bound(const std::vector<QuerySpec>& qs, size_t c);
void build_wide_edit_distance_plan(const std::vector<QuerySpec>& qs, const std::vector<WideQuery>& wq, size_t c,
                                   size_t quantum, size_t cap, uint8_t*& ws, Plan& P);

// Host-side schedule check (nothing dereferenced): the number of reads of a
// word the plan writes before any earlier step wrote it, of in-step races
// (two writers, or a subtrahend another job writes) and of steps above cap
// (0: no bound); *rounds = sum over bootstrap steps of ceil(count / round).
size_t verify_plan(const Plan& P, size_t round, size_t cap, size_t* rounds);

// Splits oversized steps, uploads the jobs into ws (advancing it) and
// reserves the key-switch partial sums.
hipError_t upload_plan(Plan& P, uint8_t*& ws, hipStream_t st);

// Enqueues every step (or the captured graph).
hipError_t run_plan(Context* C, const Plan& P);

// Enqueues steps first .. first + count - 1 (never the graph); the plan's
// Enc(1) fills run first when first is 0.
hipError_t run_plan_steps(Context* C, const Plan& P, size_t first, size_t count);

// Captures the plan's launches into a graph executable.
hipError_t capture_plan(Context* C, Plan& P);

// Query specs of C-ABI queries, checking buffers, lengths and alphabets
// (capi.cpp); refresh is the interval the queries use.
int make_query_specs(const lvs_query* q, size_t nq, int encoding, size_t refresh, std::vector<QuerySpec>& qs);
// LVS_E_INVAL past LVS_MAX_LEN, LVS_E_NOISE_BUDGET past the no-refresh depth
// when the context's refresh is off (capi.cpp).
int check_query_lengths(const Context* C, size_t m, size_t n, const char* fn);

}  // namespace lvs
