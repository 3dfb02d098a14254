// Launch-shape tuning of the blind rotation.
//
// The blind rotation has four forms (one eight-wave or one sixteen-wave
// workgroup per CU; two eight-wave or two four-wave workgroups per CU) and an
// optional persistent grid.  Which is faster depends on how a batch fills the device,
// so the autotuner times every form, and a persistent grid, on batches around
// the CU count and keeps the fastest shape per batch size.  Its inputs are zero
// ciphertexts: the work of a bootstrap does not depend on the values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"
#include "plan.h"

using namespace lvs;

namespace {

#define TUNE_FAIL(code, msg) \
    do {                     \
        set_error(msg);      \
        return (code);       \
    } while (0)

#define TUNE_HIP(expr)                                                                                  \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) TUNE_FAIL(LVS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

Context* ctx_of(lvs_context* c) {
    auto* h = reinterpret_cast<Context*>(c);
    return (h && h->kind == kContext) ? h : nullptr;
}

// Batch sizes timed: half the CUs up to four times the CUs.
std::vector<int> tune_batches(int cus, size_t max_batch) {
    std::vector<int> out;
    for (int b : {cus / 2, cus, cus + cus / 4, 2 * cus, 4 * cus})
        if (b >= 1 && size_t(b) <= max_batch && (out.empty() || b > out.back())) out.push_back(b);
    if (out.empty()) out.push_back(int(max_batch));
    return out;
}

struct Candidate {
    int form, grid;
};

}  // namespace

extern "C" {

size_t lvs_autotune_workspace_bytes(size_t max_batch) {
    const size_t b = std::max<size_t>(max_batch, 1);
    return 2 * align256(sizeof(uint64_t) * b * kCtWords) + plan_bytes(b, b);
}

int lvs_context_get_tuning(const lvs_context* ctx, lvs_tuning* out) {
    Context* C = ctx_of(const_cast<lvs_context*>(ctx));
    if (!C || !out) TUNE_FAIL(LVS_E_INVAL, "lvs_context_get_tuning: bad argument");
    out->br_grid = C->br_grid;
    out->latency_form_max = C->latency_form_max;
    out->latency_waves = C->latency_waves;
    out->throughput_waves = C->throughput_waves;
    out->ks_tile = C->ks_tile;
    return LVS_OK;
}

int lvs_context_set_tuning(lvs_context* ctx, const lvs_tuning* t) {
    Context* C = ctx_of(ctx);
    if (!C || !t) TUNE_FAIL(LVS_E_INVAL, "lvs_context_set_tuning: bad argument");
    if (t->br_grid < 0 || t->latency_form_max < 0) TUNE_FAIL(LVS_E_INVAL, "lvs_context_set_tuning: negative value");
    if (t->latency_waves != 0 && t->latency_waves != 8 && t->latency_waves != 16)
        TUNE_FAIL(LVS_E_INVAL, "lvs_context_set_tuning: latency_waves must be 8 or 16");
    if (t->throughput_waves != 0 && t->throughput_waves != 4 && t->throughput_waves != 8)
        TUNE_FAIL(LVS_E_INVAL, "lvs_context_set_tuning: throughput_waves must be 4 or 8");
    if (t->ks_tile != 0 && t->ks_tile != 4 && t->ks_tile != 8 && t->ks_tile != 16)
        TUNE_FAIL(LVS_E_INVAL, "lvs_context_set_tuning: ks_tile must be 4, 8 or 16");
    C->br_grid = t->br_grid;
    C->latency_form_max = t->latency_form_max;
    C->latency_waves = t->latency_waves ? t->latency_waves : 8;
    C->throughput_waves = t->throughput_waves ? t->throughput_waves : 8;
    C->ks_tile = t->ks_tile ? t->ks_tile : 8;
    return LVS_OK;
}

int lvs_autotune(lvs_context* ctx, size_t max_batch, void* d_work, size_t work_bytes, lvs_tuning* best,
                 lvs_tune_sample* samples, size_t max_samples, size_t* n_samples) {
    Context* C = ctx_of(ctx);
    if (!C || !d_work) TUNE_FAIL(LVS_E_INVAL, "lvs_autotune: bad argument");
    if (max_batch == 0 || max_batch > kMaxStep) TUNE_FAIL(LVS_E_INVAL, "lvs_autotune: max_batch out of range");
    if (work_bytes < lvs_autotune_workspace_bytes(max_batch))
        TUNE_FAIL(LVS_E_NOMEM_DEVICE, "lvs_autotune: workspace too small");
    if (reinterpret_cast<uintptr_t>(d_work) % 256) TUNE_FAIL(LVS_E_INVAL, "lvs_autotune: workspace misaligned");
    TUNE_HIP(hipSetDevice(C->device));
    const hipStream_t st = C->stream;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    uint64_t* in = reinterpret_cast<uint64_t*>(ws);
    ws += align256(sizeof(uint64_t) * max_batch * kCtWords);
    uint64_t* out = reinterpret_cast<uint64_t*>(ws);
    ws += align256(sizeof(uint64_t) * max_batch * kCtWords);
    TUNE_HIP(launch_fill_u64(in, max_batch * kCtWords, 0, st));

    hipEvent_t e0 = nullptr, e1 = nullptr;
    TUNE_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        TUNE_FAIL(LVS_E_DEVICE, "lvs_autotune: hipEventCreate failed");
    }
    struct Result {
        int batch, form, grid;
        double ms;
    };
    std::vector<Result> res;
    hipError_t err = hipSuccess;
    const int cus = std::max(1, C->cus);
    for (int B : tune_batches(cus, max_batch)) {
        Plan P;
        build_pbs_plan(in, nullptr, LVS_LUT_EQ, size_t(B), out, P);
        uint8_t* w = ws;
        err = upload_plan(P, w, st);
        if (err == hipSuccess) err = launch_keyswitch_jobs(P.d_jobs, B, C->ksk, P.d_part, st);
        // forms: 1 / 3 one eight- / sixteen-wave workgroup per CU, 2 / 4 two
        // four- / eight-wave workgroups per CU
        std::vector<Candidate> cands{{1, B}, {3, B}, {2, B}, {4, B}};
        if (B >= 2 * cus) {
            cands.push_back({2, 2 * cus});
            cands.push_back({4, 2 * cus});
        }
        for (const Candidate& c : cands) {
            if (err != hipSuccess) break;
            const bool two = c.form == 2 || c.form == 4;
            const int lf = two ? 0 : INT_MAX;
            const int waves = c.form == 3 ? 16 : 8;
            const int tw = c.form == 2 ? 4 : 8;
            // one launch to warm caches, then two timed
            err = launch_blind_rotate_jobs(P.d_jobs, B, P.d_part, C->luts, C->bsk, C->tables, c.grid, lf, waves, st, 0,
                                           tw);
            if (err == hipSuccess) err = hipEventRecord(e0, st);
            for (int r = 0; r < 2 && err == hipSuccess; ++r)
                err = launch_blind_rotate_jobs(P.d_jobs, B, P.d_part, C->luts, C->bsk, C->tables, c.grid, lf, waves,
                                               st, 0, tw);
            if (err == hipSuccess) err = hipEventRecord(e1, st);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess) res.push_back({B, c.form, c.grid, double(ms) / 2});
        }
        // the key switch at each tile size (form 5, grid = the tile)
        for (int tile : {4, 8, 16}) {
            if (err != hipSuccess) break;
            const int ns = keyswitch_splits(B, tile);
            err = launch_keyswitch_jobs(P.d_jobs, B, C->ksk, P.d_part, st, ns, tile);
            if (err == hipSuccess) err = hipEventRecord(e0, st);
            for (int r = 0; r < 2 && err == hipSuccess; ++r)
                err = launch_keyswitch_jobs(P.d_jobs, B, C->ksk, P.d_part, st, ns, tile);
            if (err == hipSuccess) err = hipEventRecord(e1, st);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess) res.push_back({B, 5, tile, double(ms) / 2});
        }
        if (err != hipSuccess) break;
    }
    (void)hipEventDestroy(e0);   // a failed measurement is reported below
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) TUNE_FAIL(LVS_E_DEVICE, std::string("lvs_autotune: ") + hipGetErrorString(err));

    auto time_of = [&](int B, int form, int grid) {
        for (const auto& r : res)
            if (r.batch == B && r.form == form && r.grid == grid) return r.ms;
        return -1.0;
    };
    // the one-per-CU form and the two-per-CU form with the smaller total
    // time over the batches tried, then the one-per-CU form until the
    // two-per-CU form is more than 1% faster, in increasing batch order (if it
    // never is, the one-per-CU form takes every size)
    lvs_tuning t{};
    const std::vector<int> tried_b = tune_batches(cus, max_batch);
    double t8 = 0, t16 = 0, t4x2 = 0, t8x2 = 0;
    for (int B : tried_b) {
        t8 += time_of(B, 1, B);
        t16 += time_of(B, 3, B);
        t4x2 += time_of(B, 2, B);
        t8x2 += time_of(B, 4, B);
    }
    const int lat = t16 < t8 ? 3 : 1;
    const int thr = t4x2 < t8x2 ? 2 : 4;
    t.latency_waves = lat == 3 ? 16 : 8;
    t.throughput_waves = thr == 2 ? 4 : 8;
    t.latency_form_max = 0;
    for (size_t k = 0; k < tried_b.size(); ++k) {
        const int B = tried_b[k];
        if (time_of(B, lat, B) > 1.01 * time_of(B, thr, B)) break;
        t.latency_form_max = (k + 1 == tried_b.size()) ? INT_MAX : B;
    }
    // a persistent grid only if it wins by more than 1% at every batch that tried it
    bool tried = false, wins = true;
    for (const auto& r : res)
        if (r.grid != r.batch && r.form == thr) {
            tried = true;
            wins = wins && r.ms < 0.99 * time_of(r.batch, thr, r.batch);
        }
    t.br_grid = (tried && wins) ? 2 * cus : 0;
    // the key-switch tile with the smallest total time over the batches tried
    double best_ks = -1;
    t.ks_tile = 8;
    for (int tile : {4, 8, 16}) {
        double tot = 0;
        for (int B : tried_b) tot += time_of(B, 5, tile);
        if (best_ks < 0 || tot < best_ks) {
            best_ks = tot;
            t.ks_tile = tile;
        }
    }
    C->ks_tile = t.ks_tile;
    C->br_grid = t.br_grid;
    C->latency_form_max = t.latency_form_max;
    C->latency_waves = t.latency_waves;
    C->throughput_waves = t.throughput_waves;
    if (best) *best = t;
    if (n_samples) *n_samples = res.size();
    for (size_t k = 0; k < res.size() && samples && k < max_samples; ++k)
        samples[k] = lvs_tune_sample{res[k].batch, res[k].form, res[k].grid, res[k].ms};
    return LVS_OK;
}

size_t lvs_microbench_workspace_bytes(const lvs_context* ctx) {
    Context* C = ctx_of(const_cast<lvs_context*>(ctx));
    return C ? sizeof(uint32_t) * 256 * size_t(8 * std::max(1, C->cus)) : 0;
}

int lvs_microbench_modmul(lvs_context* ctx, int iters, void* d_work, size_t work_bytes, double* ms,
                          double* int_muls) {
    Context* C = ctx_of(ctx);
    if (!C || !d_work || !ms || !int_muls || iters <= 0) TUNE_FAIL(LVS_E_INVAL, "lvs_microbench_modmul: bad argument");
    if (work_bytes < lvs_microbench_workspace_bytes(ctx))
        TUNE_FAIL(LVS_E_INVAL, "lvs_microbench_modmul: workspace too small");
    TUNE_HIP(hipSetDevice(C->device));
    const int blocks = 8 * std::max(1, C->cus);   // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    uint32_t* out = reinterpret_cast<uint32_t*>(d_work);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TUNE_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch_modmul_probe(out, blocks, std::min(iters, 64), C->stream);   // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, C->stream);
    if (err == hipSuccess) err = launch_modmul_probe(out, blocks, iters, C->stream);
    if (err == hipSuccess) err = hipEventRecord(e1, C->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) TUNE_FAIL(LVS_E_DEVICE, std::string("lvs_microbench_modmul: ") + hipGetErrorString(err));
    *ms = t;
    *int_muls = double(blocks) * 256.0 * double(iters) * modmul_probe_muls_per_thread_iter();
    return LVS_OK;
}

int lvs_microbench_copy(lvs_context* ctx, const void* d_src, void* d_dst, size_t bytes, int reps, double* ms) {
    Context* C = ctx_of(ctx);
    if (!C || !d_src || !d_dst || !ms || reps <= 0 || bytes % 16 ||
        reinterpret_cast<uintptr_t>(d_src) % 16 || reinterpret_cast<uintptr_t>(d_dst) % 16)
        TUNE_FAIL(LVS_E_INVAL, "lvs_microbench_copy: bad argument");
    TUNE_HIP(hipSetDevice(C->device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TUNE_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch_copy_probe(d_src, d_dst, bytes, std::max(1, C->cus), C->stream);
    if (err == hipSuccess) err = hipEventRecord(e0, C->stream);
    for (int r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_copy_probe(d_src, d_dst, bytes, std::max(1, C->cus), C->stream);
    if (err == hipSuccess) err = hipEventRecord(e1, C->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (err != hipSuccess) TUNE_FAIL(LVS_E_DEVICE, std::string("lvs_microbench_copy: ") + hipGetErrorString(err));
    *ms = double(t) / reps;
    return LVS_OK;
}

}  // extern "C"
