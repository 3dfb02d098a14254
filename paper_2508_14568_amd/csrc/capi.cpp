// C ABI of liblvs: keys, device context, bootstrap batches and the plain
// anti-diagonal edit-distance driver (Algorithm 4 of arXiv 2508.14568 with the
// Section 6.2 observation that cells of one anti-diagonal are independent).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <set>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "context.h"
#include "launch.h"
#include "lvs_internal.h"
#include "plan.h"

namespace lvs {

namespace {

thread_local std::string g_error = "no error";

constexpr size_t kAlign = 256;
constexpr size_t kMaxLen = LVS_MAX_LEN;
constexpr size_t W = kCtWords;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct ArenaLayout {
    size_t bsk, ksk, tw, luts, total;
};

ArenaLayout arena_layout() {
    ArenaLayout L{};
    size_t off = 0;
    L.bsk = off;
    off = align_up(off + sizeof(uint32_t) * size_t(kSmallN) * kPrimes * 4 * kN);
    L.ksk = off;
    off = align_up(off + sizeof(uint64_t) * size_t(kKsRows) * kSmallWords);
    L.tw = off;
    off = align_up(off + sizeof(uint32_t) * (4 * size_t(kPrimes) * kN + 2 * kPrimes));
    L.luts = off;
    off = align_up(off + sizeof(uint64_t) * size_t(LVS_LUT_SLOTS) * kN);
    L.total = off;
    return L;
}

// Test polynomial of a 16-entry table: coefficient t holds f(t / 128) * 2^59,
// then the polynomial is multiplied by X^-64 so each value's box is centred.
void build_test_poly(const int32_t f16[16], uint64_t* out) {
    std::vector<uint64_t> v(kN);
    const int box = kN / 16;
    for (int t = 0; t < kN; ++t) v[t] = uint64_t(uint32_t(f16[t / box]) & 31u) << kDeltaLog;
    const int half = box / 2;
    for (int t = 0; t < kN; ++t) out[t] = (t + half < kN) ? v[t + half] : uint64_t(0) - v[t + half - kN];
}

#define LVS_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
            return LVS_E_DEVICE;                                                           \
        }                                                                                  \
    } while (0)

#define LVS_REQUIRE(cond, code, msg) \
    do {                             \
        if (!(cond)) {               \
            set_error(msg);          \
            return (code);           \
        }                            \
    } while (0)

Context* as_ctx(lvs_context* c) {
    auto* h = reinterpret_cast<Context*>(c);
    return (h && h->kind == kContext) ? h : nullptr;
}
const ClientKey* as_ck(const lvs_client_key* c) {
    auto* h = reinterpret_cast<const ClientKey*>(c);
    return (h && h->kind == kClientKey) ? h : nullptr;
}
const ServerKey* as_sk(const lvs_server_key* c) {
    auto* h = reinterpret_cast<const ServerKey*>(c);
    return (h && h->kind == kServerKey) ? h : nullptr;
}

int nsym_of(int encoding) { return encoding == LVS_ENC_ASCII7 ? 2 : 1; }

// ------------------------------------------------------------- plans

bool valid_encoding(int e) { return e == LVS_ENC_ASCII7 || e == LVS_ENC_DNA2; }

// Uploads and runs a plan built for one call; ws must hold plan_bytes().
int execute(Context* C, Plan& P, uint8_t* ws) {
    LVS_HIP(upload_plan(P, ws, C->stream));
    LVS_HIP(run_plan(C, P));
    return LVS_OK;
}

// Bound of a wavefront plan's largest step: a diagonal holds at most
// min(m, n) cells of a query, each step the cells of one diagonal plus one
// equality stage of each of the next two, a refresh step two bootstraps per
// cell of a diagonal.
size_t max_step_of(const std::vector<QuerySpec>& qs) {
    size_t step = 0;
    for (const auto& q : qs) {
        const size_t w = std::min(q.m, q.n);
        const bool eq = q.B && !q.eq9_in;
        const size_t k = eq ? (q.encoding == LVS_ENC_ASCII7 ? 3 : 2) : 1;
        step += std::max<size_t>(k, q.refresh ? 2 : 1) * w;
    }
    return step;
}

// Section 3.1: with refresh off the differences' noise grows with min(m, n),
// which is then bounded; the string lengths are bounded in any case.
int check_lengths(const Context* C, size_t m, size_t n, const char* fn) {
    LVS_REQUIRE(std::max(m, n) <= kMaxLen, LVS_E_INVAL, std::string(fn) + ": string longer than LVS_MAX_LEN");
    LVS_REQUIRE(C->refresh_every > 0 || std::min(m, n) <= size_t(LVS_MAX_DEPTH_NO_REFRESH), LVS_E_NOISE_BUDGET,
                std::string(fn) + ": min(m, n) exceeds the noise budget with refresh off");
    return LVS_OK;
}

#define LVS_CHECK_LENGTHS(C, m, n, fn)                  \
    do {                                                \
        const int rc_ = check_lengths((C), (m), (n), fn); \
        if (rc_) return rc_;                            \
    } while (0)

// Bootstraps the device runs at once for steps of up to cap bootstraps: one
// per CU in the eight-wave form, two per CU in the four-wave form.
size_t round_of(const Context* C, size_t cap) {
    const size_t cus = size_t(std::max(1, C->cus));
    return cap <= size_t(C->latency_form_max) ? cus : 2 * cus;
}

size_t plan_ws(const std::vector<QuerySpec>& qs) {
    size_t b = 0, jobs = 0;
    for (const auto& q : qs) {
        b += query_buffer_bytes(q);
        jobs += query_jobs(q);
    }
    return b + plan_bytes(jobs, max_step_of(qs));
}

}  // namespace

int check_query_lengths(const Context* C, size_t m, size_t n, const char* fn) { return check_lengths(C, m, n, fn); }

void set_error(const std::string& msg) { g_error = msg; }

bool params_supported(const lvs_params& p) {
    return p.n_lwe == uint32_t(kSmallN) && p.glwe_k == 1 && p.poly_N == uint32_t(kN) &&
           p.pbs_base_log == uint32_t(kPbsBaseLog) && p.pbs_level == 1 && p.ks_base_log == uint32_t(kKsBaseLog) &&
           p.ks_level == uint32_t(kKsLevel);
}

}  // namespace lvs

using namespace lvs;

extern "C" {

const char* lvs_last_error(void) { return g_error.c_str(); }

int lvs_params_default(lvs_params* out) {
    LVS_REQUIRE(out, LVS_E_INVAL, "lvs_params_default: out is NULL");
    out->n_lwe = kSmallN;
    out->glwe_k = 1;
    out->poly_N = kN;
    out->pbs_base_log = kPbsBaseLog;
    out->pbs_level = 1;
    out->ks_base_log = kKsBaseLog;
    out->ks_level = kKsLevel;
    out->lwe_noise_q64 = 130415703530680ULL;   // 7.069849454709433e-06 * 2^64
    out->glwe_noise_q64 = 5424ULL;             // 2.9403601535432533e-16 * 2^64
    return LVS_OK;
}

size_t lvs_ct_words(void) { return kCtWords; }

int lvs_keygen(const lvs_params* params, uint64_t seed, lvs_client_key** ck, lvs_server_key** sk) {
    LVS_REQUIRE(params && ck && sk, LVS_E_INVAL, "lvs_keygen: NULL argument");
    LVS_REQUIRE(params_supported(*params), LVS_E_PARAMS, "lvs_keygen: unsupported parameter set");
    ClientKey* c = new (std::nothrow) ClientKey();
    ServerKey* s = new (std::nothrow) ServerKey();
    if (!c || !s) {
        delete c;
        delete s;
        set_error("lvs_keygen: out of host memory");
        return LVS_E_NOMEM_HOST;
    }
    c->kind = kClientKey;
    s->kind = kServerKey;
    try {
        keygen(*params, seed, *c, *s);
    } catch (const std::bad_alloc&) {
        delete c;
        delete s;
        set_error("lvs_keygen: out of host memory");
        return LVS_E_NOMEM_HOST;
    }
    *ck = reinterpret_cast<lvs_client_key*>(c);
    *sk = reinterpret_cast<lvs_server_key*>(s);
    return LVS_OK;
}

int lvs_lwe_encrypt(const lvs_client_key* ck, uint32_t mu, uint64_t seed, uint64_t index, uint64_t* h_ct) {
    const ClientKey* c = as_ck(ck);
    LVS_REQUIRE(c && h_ct, LVS_E_INVAL, "lvs_lwe_encrypt: bad argument");
    LVS_REQUIRE(mu < 32, LVS_E_INVAL, "lvs_lwe_encrypt: mu must be in 0..31");
    encrypt(*c, mu, seed, index, h_ct);
    return LVS_OK;
}

int lvs_lwe_decrypt(const lvs_client_key* ck, const uint64_t* h_ct, uint32_t* mu, int64_t* phase_err) {
    const ClientKey* c = as_ck(ck);
    LVS_REQUIRE(c && h_ct && mu, LVS_E_INVAL, "lvs_lwe_decrypt: bad argument");
    const uint64_t ph = phase(*c, h_ct);
    const uint32_t v = uint32_t((((ph >> (kDeltaLog - 1)) + 1) >> 1) & 31u);
    *mu = v;
    if (phase_err) *phase_err = int64_t(ph - (uint64_t(v) << kDeltaLog));
    return LVS_OK;
}

int lvs_encrypt_string(const lvs_client_key* ck, const uint8_t* s, size_t len, int encoding, uint64_t seed,
                       uint64_t* h_out) {
    const ClientKey* c = as_ck(ck);
    LVS_REQUIRE(c && (s || len == 0) && (h_out || len == 0), LVS_E_INVAL, "lvs_encrypt_string: bad argument");
    LVS_REQUIRE(encoding == LVS_ENC_ASCII7 || encoding == LVS_ENC_DNA2, LVS_E_INVAL, "unknown encoding");
    const int ns = nsym_of(encoding);
    for (size_t i = 0; i < len; ++i)
        LVS_REQUIRE(encoding == LVS_ENC_ASCII7 ? s[i] < 128 : s[i] < 4, LVS_E_ALPHABET,
                    "lvs_encrypt_string: symbol outside the alphabet");
    for (size_t i = 0; i < len; ++i) {
        uint32_t sym[2];
        if (encoding == LVS_ENC_ASCII7) {
            sym[0] = s[i] & 15u;
            sym[1] = s[i] >> 4;
        } else {
            sym[0] = s[i];
        }
        for (int r = 0; r < ns; ++r) encrypt(*c, sym[r], seed, i * ns + r, h_out + (i * ns + r) * W);
    }
    return LVS_OK;
}

int lvs_decrypt_distance(const lvs_client_key* ck, const uint64_t* h_last, size_t m, size_t n, int64_t* out) {
    const ClientKey* c = as_ck(ck);
    LVS_REQUIRE(c && (h_last || n == 0) && out, LVS_E_INVAL, "lvs_decrypt_distance: bad argument");
    int64_t d = int64_t(m);
    for (size_t j = 0; j < n; ++j) {
        const uint64_t ph = phase(*c, h_last + j * W);
        uint32_t v = uint32_t((((ph >> (kDeltaLog - 1)) + 1) >> 1) & 31u);
        d += (v >= 16) ? int64_t(v) - 32 : int64_t(v);
    }
    *out = d;
    return LVS_OK;
}

int lvs_key_export(const lvs_client_key* ck, const lvs_server_key* sk, int kind, void* buf, size_t* len) {
    LVS_REQUIRE(len, LVS_E_INVAL, "lvs_key_export: len is NULL");
    const ClientKey* c = as_ck(ck);
    const ServerKey* s = as_sk(sk);
    const void* src = nullptr;
    size_t bytes = 0;
    if (kind == 0 && c) { src = c->s.data(); bytes = c->s.size(); }
    else if (kind == 1 && c) { src = c->S.data(); bytes = c->S.size(); }
    else if (kind == 2 && s) { src = s->bsk.data(); bytes = s->bsk.size() * 8; }
    else if (kind == 3 && s) { src = s->ksk.data(); bytes = s->ksk.size() * 8; }
    else { set_error("lvs_key_export: bad kind or handle"); return LVS_E_INVAL; }
    if (buf) {
        LVS_REQUIRE(*len >= bytes, LVS_E_INVAL, "lvs_key_export: buffer too small");
        std::memcpy(buf, src, bytes);
    }
    *len = bytes;
    return LVS_OK;
}

int lvs_context_bytes(const lvs_params* params, size_t* bytes) {
    LVS_REQUIRE(params && bytes, LVS_E_INVAL, "lvs_context_bytes: NULL argument");
    LVS_REQUIRE(params_supported(*params), LVS_E_PARAMS, "lvs_context_bytes: unsupported parameter set");
    *bytes = arena_layout().total;
    return LVS_OK;
}

int lvs_context_create(const lvs_server_key* sk, int device, void* hip_stream, void* d_arena, size_t arena_bytes,
                       lvs_context** out) {
    const ServerKey* s = as_sk(sk);
    LVS_REQUIRE(s && out && d_arena, LVS_E_INVAL, "lvs_context_create: NULL argument");
    LVS_REQUIRE(reinterpret_cast<uintptr_t>(d_arena) % kAlign == 0, LVS_E_INVAL,
                "lvs_context_create: arena must be 256-byte aligned");
    const ArenaLayout L = arena_layout();
    LVS_REQUIRE(arena_bytes >= L.total, LVS_E_NOMEM_DEVICE, "lvs_context_create: arena too small");
    LVS_HIP(hipSetDevice(device));
    Context* C = new (std::nothrow) Context();
    LVS_REQUIRE(C, LVS_E_NOMEM_HOST, "lvs_context_create: out of host memory");
    C->kind = kContext;
    C->p = s->p;
    C->device = device;
    C->stream = reinterpret_cast<hipStream_t>(hip_stream);
    C->arena = reinterpret_cast<uint8_t*>(d_arena);
    C->arena_bytes = arena_bytes;
    C->bsk = reinterpret_cast<uint32_t*>(C->arena + L.bsk);
    C->ksk = reinterpret_cast<uint64_t*>(C->arena + L.ksk);
    C->tw = reinterpret_cast<uint32_t*>(C->arena + L.tw);
    C->luts = reinterpret_cast<uint64_t*>(C->arena + L.luts);
    const PrimeTables& T = prime_tables();
    const size_t tn = size_t(kPrimes) * kN;
    std::vector<uint32_t> tw(4 * tn + 2 * kPrimes);
    for (size_t k = 0; k < tn; ++k) {
        tw[2 * k] = T.fwd[k];
        tw[2 * k + 1] = T.fwd_shoup[k];
        tw[2 * tn + 2 * k] = T.inv[k];
        tw[2 * tn + 2 * k + 1] = T.inv_shoup[k];
    }
    for (int r = 0; r < kPrimes; ++r) {
        tw[4 * tn + r] = T.bsk_scale[r];
        tw[4 * tn + kPrimes + r] = uint32_t((uint64_t(T.bsk_scale[r]) << 32) / T.p[r]);
    }
    C->tables = DevTables{C->tw, C->tw + 2 * tn, C->tw + 4 * tn, C->tw + 4 * tn + kPrimes};
    auto fail = [&](int code) { delete C; return code; };
    hipError_t e = hipDeviceGetAttribute(&C->cus, hipDeviceAttributeMultiprocessorCount, device);
    C->latency_form_max = INT_MAX;     // the eight-wave form: faster at every batch size measured
    if (e == hipSuccess) e = prepare_kernels();
    if (e == hipSuccess) e = static_scratch_setup(device);
    if (e == hipSuccess) e = hipMemcpy(C->tw, tw.data(), tw.size() * 4, hipMemcpyHostToDevice);
    // the 64-bit bootstrapping key is staged in the key-switching key's slot
    if (e == hipSuccess) e = hipMemcpy(C->ksk, s->bsk.data(), s->bsk.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_bsk_convert(C->ksk, C->bsk, C->tables, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(C->ksk, s->ksk.data(), s->ksk.size() * 8, hipMemcpyHostToDevice);
    std::vector<uint64_t> luts(size_t(LVS_LUT_SLOTS) * kN, 0);
    const int32_t f_eq[16] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int32_t f_eq9[16] = {9, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    // 1 + min(-eq, dv, dh) under key (1 - dv) + 3 (1 + dh) + 9 eq: the value is 1
    // exactly when eq = 0, dh >= 0 and dv >= 0, i.e. keys 3, 4, 6, 7.
    const int32_t f_min[16] = {0, 0, 0, 1, 1, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0};
    build_test_poly(f_eq, &luts[size_t(LVS_LUT_EQ) * kN]);
    build_test_poly(f_eq9, &luts[size_t(LVS_LUT_EQ9) * kN]);
    build_test_poly(f_min, &luts[size_t(LVS_LUT_MIN) * kN]);
    // the identity on the differences -1, 0, 1: an input of -1 (= 31) reads -f(15)
    const int32_t f_refresh[16] = {0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1};
    build_test_poly(f_refresh, &luts[size_t(LVS_LUT_REFRESH) * kN]);
    // Algorithm 2's merging test, with the group sum offset so its maximum reads 15
    const int32_t f_max[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1};
    const int32_t f_max9[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 9};
    build_test_poly(f_max, &luts[size_t(LVS_LUT_MAX) * kN]);
    build_test_poly(f_max9, &luts[size_t(LVS_LUT_MAX9) * kN]);
    if (e == hipSuccess) e = hipMemcpy(C->luts, luts.data(), luts.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error(std::string("lvs_context_create: ") + hipGetErrorString(e));
        return fail(LVS_E_DEVICE);
    }
    *out = reinterpret_cast<lvs_context*>(C);
    return LVS_OK;
}

int lvs_context_set_stream(lvs_context* ctx, void* hip_stream) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_context_set_stream: bad context");
    C->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return LVS_OK;
}

int lvs_context_set_lut(lvs_context* ctx, int slot, const int32_t f16[16]) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C && f16, LVS_E_INVAL, "lvs_context_set_lut: bad argument");
    LVS_REQUIRE(slot >= LVS_LUT_USER && slot < LVS_LUT_SLOTS, LVS_E_INVAL, "lvs_context_set_lut: bad slot");
    std::vector<uint64_t> poly(kN);
    build_test_poly(f16, poly.data());
    LVS_HIP(hipSetDevice(C->device));
    LVS_HIP(hipMemcpyAsync(C->luts + size_t(slot) * kN, poly.data(), kN * 8, hipMemcpyHostToDevice, C->stream));
    LVS_HIP(hipStreamSynchronize(C->stream));
    return LVS_OK;
}

int lvs_context_set_refresh(lvs_context* ctx, size_t every) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_context_set_refresh: bad context");
    LVS_REQUIRE(every == 0 || (every >= LVS_REFRESH_MIN && every <= LVS_REFRESH_MAX), LVS_E_INVAL,
                "lvs_context_set_refresh: interval must be 0 or LVS_REFRESH_MIN..LVS_REFRESH_MAX");
    C->refresh_every = every;
    return LVS_OK;
}

int lvs_context_get_refresh(const lvs_context* ctx, size_t* every) {
    Context* C = as_ctx(const_cast<lvs_context*>(ctx));
    LVS_REQUIRE(C && every, LVS_E_INVAL, "lvs_context_get_refresh: bad argument");
    *every = C->refresh_every;
    return LVS_OK;
}

int lvs_sync(lvs_context* ctx) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_sync: bad context");
    LVS_HIP(hipStreamSynchronize(C->stream));
    return LVS_OK;
}

size_t lvs_pbs_workspace_bytes(size_t B) { return plan_bytes(std::max<size_t>(B, 1), std::max<size_t>(B, 1)); }

int lvs_pbs_batch(lvs_context* ctx, const uint64_t* d_in, const uint8_t* lut_ids, int lut_id, size_t B,
                  uint64_t* d_out, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_pbs_batch: bad context");
    if (B == 0) return LVS_OK;
    LVS_REQUIRE(d_in && d_out && d_work, LVS_E_INVAL, "lvs_pbs_batch: NULL buffer");
    if (lut_ids) {
        for (size_t k = 0; k < B; ++k)
            LVS_REQUIRE(lut_ids[k] < LVS_LUT_SLOTS, LVS_E_INVAL, "lvs_pbs_batch: bad lut id");
    } else {
        LVS_REQUIRE(lut_id >= 0 && lut_id < LVS_LUT_SLOTS, LVS_E_INVAL, "lvs_pbs_batch: bad lut id");
    }
    LVS_REQUIRE(work_bytes >= lvs_pbs_workspace_bytes(B), LVS_E_NOMEM_DEVICE, "lvs_pbs_batch: workspace too small");
    LVS_REQUIRE(d_out + B * W <= d_in || d_in + B * W <= d_out, LVS_E_INVAL, "lvs_pbs_batch: in and out overlap");
    LVS_HIP(hipSetDevice(C->device));
    Plan P;
    build_pbs_plan(d_in, lut_ids, lut_id, B, d_out, P);
    return execute(C, P, reinterpret_cast<uint8_t*>(d_work));
}

extern "C++" {
namespace {
QuerySpec pair_query(const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, int encoding, uint64_t* h) {
    QuerySpec q;
    q.encoding = encoding;
    q.A = d_a;
    q.m = m;
    q.B = d_b;
    q.n = n;
    q.h_last = h;
    return q;
}

// Fills h[0..n) with Enc(1): the result for an empty first string.
int empty_first(Context* C, size_t n, uint64_t* d_h_last) {
    LVS_HIP(launch_trivial(d_h_last, int(n), 1, C->stream));
    return LVS_OK;
}
}  // namespace
}  // extern "C++"

size_t lvs_equality_workspace_bytes(size_t m, size_t n, int encoding) {
    const size_t eq1 = encoding == LVS_ENC_ASCII7 ? align256(sizeof(uint64_t) * m * n * W) : 0;
    return eq1 + plan_bytes(m * n * (encoding == LVS_ENC_ASCII7 ? 2 : 1), m * n);
}

int lvs_equality(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, int encoding,
                 uint64_t* d_eq9, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_equality: bad context");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    if (m == 0 || n == 0) return LVS_OK;
    LVS_REQUIRE(d_a && d_b && d_eq9 && d_work, LVS_E_INVAL, "lvs_equality: NULL buffer");
    LVS_REQUIRE(work_bytes >= lvs_equality_workspace_bytes(m, n, encoding), LVS_E_NOMEM_DEVICE,
                "lvs_equality: workspace too small");
    LVS_HIP(hipSetDevice(C->device));
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    std::vector<QuerySpec> qs{pair_query(d_a, m, d_b, n, encoding, nullptr)};
    qs[0].eq9 = d_eq9;
    if (encoding == LVS_ENC_ASCII7) {
        qs[0].eq1 = reinterpret_cast<uint64_t*>(ws);
        ws += align256(sizeof(uint64_t) * m * n * W);
    }
    Plan P;
    build_edit_distance_plan(qs, P, /*with_dp=*/false);
    return execute(C, P, ws);
}

size_t lvs_edit_distance_eq9_workspace_bytes(size_t m, size_t n) {
    std::vector<QuerySpec> qs(1);
    qs[0].m = m;
    qs[0].n = n;
    qs[0].eq9_in = reinterpret_cast<const uint64_t*>(16);
    qs[0].refresh = LVS_REFRESH_MIN;
    return plan_ws(qs);
}

int lvs_edit_distance_eq9(lvs_context* ctx, const uint64_t* d_eq9, size_t m, size_t n, uint64_t* d_h_last,
                          uint64_t* d_trace, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_edit_distance_eq9: bad context");
    LVS_REQUIRE((d_eq9 || m * n == 0) && (d_h_last || n == 0), LVS_E_INVAL, "lvs_edit_distance_eq9: NULL buffer");
    LVS_CHECK_LENGTHS(C, m, n, "lvs_edit_distance_eq9");
    LVS_HIP(hipSetDevice(C->device));
    if (n == 0) return LVS_OK;
    if (m == 0) return empty_first(C, n, d_h_last);
    LVS_REQUIRE(d_work && work_bytes >= lvs_edit_distance_eq9_workspace_bytes(m, n), LVS_E_NOMEM_DEVICE,
                "lvs_edit_distance_eq9: workspace too small");
    std::vector<QuerySpec> qs(1);
    qs[0].m = m;
    qs[0].n = n;
    qs[0].eq9_in = d_eq9;
    qs[0].h_last = d_h_last;
    qs[0].trace = d_trace;
    qs[0].refresh = C->refresh_every;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    Plan P;
    build_edit_distance_plan(qs, P);
    return execute(C, P, ws);
}

size_t lvs_edit_distance_workspace_bytes(size_t m, size_t n, int encoding) {
    std::vector<QuerySpec> qs{pair_query(nullptr, m, reinterpret_cast<const uint64_t*>(16), n, encoding, nullptr)};
    qs[0].refresh = LVS_REFRESH_MIN;
    return plan_ws(qs);
}

int lvs_edit_distance(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, int encoding,
                      uint64_t* d_h_last, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_edit_distance: bad context");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    LVS_REQUIRE((d_a || m == 0) && (d_b || n == 0) && (d_h_last || n == 0), LVS_E_INVAL,
                "lvs_edit_distance: NULL buffer");
    LVS_CHECK_LENGTHS(C, m, n, "lvs_edit_distance");
    LVS_HIP(hipSetDevice(C->device));
    if (n == 0) return LVS_OK;
    if (m == 0) return empty_first(C, n, d_h_last);
    LVS_REQUIRE(d_work && work_bytes >= lvs_edit_distance_workspace_bytes(m, n, encoding), LVS_E_NOMEM_DEVICE,
                "lvs_edit_distance: workspace too small");
    std::vector<QuerySpec> qs{pair_query(d_a, m, d_b, n, encoding, d_h_last)};
    qs[0].refresh = C->refresh_every;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    Plan P;
    const size_t cap = max_step_of(qs);
    build_edit_distance_plan(qs, P, true, round_of(C, cap), cap);
    return execute(C, P, ws);
}

size_t lvs_band_exact(size_t m, size_t n) { return std::max(m, n) - std::min(m, n) / 2; }

size_t lvs_band_cells(size_t m, size_t n, size_t ell) { return band_cells(m, n, long(std::min<size_t>(ell, m + n))); }

size_t lvs_edit_distance_band_workspace_bytes(size_t m, size_t n, int encoding, size_t ell) {
    std::vector<QuerySpec> qs{pair_query(nullptr, m, reinterpret_cast<const uint64_t*>(16), n, encoding, nullptr)};
    qs[0].band = long(std::min<size_t>(ell, m + n));
    qs[0].refresh = LVS_REFRESH_MIN;
    return plan_ws(qs);
}

int lvs_edit_distance_band(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n,
                           int encoding, size_t ell, uint64_t* d_path, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_edit_distance_band: bad context");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    LVS_REQUIRE((d_a || m == 0) && (d_b || n == 0) && (d_path || m + n == 0), LVS_E_INVAL,
                "lvs_edit_distance_band: NULL buffer");
    LVS_CHECK_LENGTHS(C, m, n, "lvs_edit_distance_band");
    if (m + n == 0) return LVS_OK;
    LVS_REQUIRE(d_work && work_bytes >= lvs_edit_distance_band_workspace_bytes(m, n, encoding, ell),
                LVS_E_NOMEM_DEVICE, "lvs_edit_distance_band: workspace too small");
    LVS_HIP(hipSetDevice(C->device));
    std::vector<QuerySpec> qs{pair_query(d_a, m, d_b, n, encoding, nullptr)};
    qs[0].band = long(std::min<size_t>(ell, m + n));
    qs[0].path = d_path;
    qs[0].refresh = C->refresh_every;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    Plan P;
    const size_t cap = max_step_of(qs);
    build_edit_distance_plan(qs, P, true, round_of(C, cap), cap);
    return execute(C, P, ws);
}

size_t lvs_edit_distance_clear_band_workspace_bytes(size_t m, size_t n, size_t ell) {
    std::vector<QuerySpec> qs(1);
    qs[0].m = m;
    qs[0].n = n;
    qs[0].band = long(std::min<size_t>(ell, m + n));
    qs[0].refresh = LVS_REFRESH_MIN;
    return plan_ws(qs);
}

int lvs_edit_distance_clear_band(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint8_t* alphabet,
                                 size_t alen, const uint8_t* b, size_t n, size_t ell, uint64_t* d_path, void* d_work,
                                 size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_edit_distance_clear_band: bad context");
    LVS_REQUIRE((d_table || m == 0) && (alphabet || alen == 0) && (b || n == 0) && (d_path || m + n == 0),
                LVS_E_INVAL, "lvs_edit_distance_clear_band: NULL buffer");
    LVS_CHECK_LENGTHS(C, m, n, "lvs_edit_distance_clear_band");
    std::vector<QuerySpec> qs(1);
    qs[0].cols.resize(n);
    for (size_t j = 0; j < n; ++j) {
        const uint8_t* hit = std::find(alphabet, alphabet + alen, b[j]);
        LVS_REQUIRE(hit != alphabet + alen, LVS_E_ALPHABET, "lvs_edit_distance_clear_band: symbol not in the table");
        qs[0].cols[j] = int32_t(hit - alphabet);
    }
    if (m + n == 0) return LVS_OK;
    LVS_REQUIRE(d_work && work_bytes >= lvs_edit_distance_clear_band_workspace_bytes(m, n, ell), LVS_E_NOMEM_DEVICE,
                "lvs_edit_distance_clear_band: workspace too small");
    LVS_HIP(hipSetDevice(C->device));
    qs[0].m = m;
    qs[0].n = n;
    qs[0].table = d_table;
    qs[0].band = long(std::min<size_t>(ell, m + n));
    qs[0].path = d_path;
    qs[0].refresh = C->refresh_every;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    Plan P;
    build_edit_distance_plan(qs, P);
    return execute(C, P, ws);
}

size_t lvs_preprocess_workspace_bytes(size_t m, size_t alphabet_len, int encoding) {
    const size_t cells = m * alphabet_len;
    const bool ascii = encoding == LVS_ENC_ASCII7;
    return (ascii ? align256(sizeof(uint64_t) * cells * W) : 0) + plan_bytes(cells * (ascii ? 2 : 1), cells);
}

int lvs_preprocess(lvs_context* ctx, const uint64_t* d_a, size_t m, int encoding, const uint8_t* alphabet,
                   size_t alen, uint64_t* d_table, void* d_work, size_t work_bytes) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_preprocess: bad context");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    if (m == 0 || alen == 0) return LVS_OK;
    LVS_REQUIRE(d_a && alphabet && d_table && d_work, LVS_E_INVAL, "lvs_preprocess: NULL buffer");
    LVS_REQUIRE(work_bytes >= lvs_preprocess_workspace_bytes(m, alen, encoding), LVS_E_NOMEM_DEVICE,
                "lvs_preprocess: workspace too small");
    std::vector<uint8_t> lo(alen), hi(alen);
    for (size_t c = 0; c < alen; ++c) {
        LVS_REQUIRE(encoding == LVS_ENC_ASCII7 ? alphabet[c] < 128 : alphabet[c] < 4, LVS_E_ALPHABET,
                    "lvs_preprocess: alphabet symbol outside the encoding");
        lo[c] = encoding == LVS_ENC_ASCII7 ? (alphabet[c] & 15) : alphabet[c];
        hi[c] = encoding == LVS_ENC_ASCII7 ? (alphabet[c] >> 4) : 0;
    }
    LVS_HIP(hipSetDevice(C->device));
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    uint64_t* eq1 = nullptr;
    if (encoding == LVS_ENC_ASCII7) {
        eq1 = reinterpret_cast<uint64_t*>(ws);
        ws += align256(sizeof(uint64_t) * m * alen * W);
    }
    Plan P;
    build_preprocess_plan(d_a, m, encoding, lo, hi, d_table, eq1, P);
    return execute(C, P, ws);
}

size_t lvs_edit_distance_clear_workspace_bytes(size_t m, size_t n) {
    std::vector<QuerySpec> qs(1);
    qs[0].m = m;
    qs[0].n = n;
    qs[0].refresh = LVS_REFRESH_MIN;
    return plan_ws(qs);
}

extern "C++" {
namespace {
// The cleartext main pass over table rows cols[j] of the b_j (both symbol kinds).
template <typename Sym>
int clear_pass(lvs_context* ctx, const uint64_t* d_table, size_t m, const Sym* alphabet, size_t alen, const Sym* b,
               size_t n, uint64_t* d_h_last, void* d_work, size_t work_bytes, const char* fn) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, std::string(fn) + ": bad context");
    LVS_REQUIRE((d_table || m == 0) && (alphabet || alen == 0) && (b || n == 0) && (d_h_last || n == 0),
                LVS_E_INVAL, std::string(fn) + ": NULL buffer");
    LVS_CHECK_LENGTHS(C, m, n, fn);
    std::vector<QuerySpec> qs(1);
    qs[0].cols.resize(n);
    for (size_t j = 0; j < n; ++j) {
        const Sym* hit = std::find(alphabet, alphabet + alen, b[j]);
        LVS_REQUIRE(hit != alphabet + alen, LVS_E_ALPHABET, std::string(fn) + ": symbol not in the table");
        qs[0].cols[j] = int32_t(hit - alphabet);
    }
    LVS_HIP(hipSetDevice(C->device));
    if (n == 0) return LVS_OK;
    if (m == 0) return empty_first(C, n, d_h_last);
    LVS_REQUIRE(d_work && work_bytes >= lvs_edit_distance_clear_workspace_bytes(m, n), LVS_E_NOMEM_DEVICE,
                std::string(fn) + ": workspace too small");
    qs[0].m = m;
    qs[0].n = n;
    qs[0].table = d_table;
    qs[0].h_last = d_h_last;
    qs[0].refresh = C->refresh_every;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    Plan P;
    build_edit_distance_plan(qs, P);
    return execute(C, P, ws);
}
}  // namespace
}  // extern "C++"

int lvs_edit_distance_clear(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint8_t* alphabet, size_t alen,
                            const uint8_t* b, size_t n, uint64_t* d_h_last, void* d_work, size_t work_bytes) {
    return clear_pass(ctx, d_table, m, alphabet, alen, b, n, d_h_last, d_work, work_bytes, "lvs_edit_distance_clear");
}

int lvs_edit_distance_clear_wide(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint64_t* alphabet,
                                 size_t alen, const uint64_t* b, size_t n, uint64_t* d_h_last, void* d_work,
                                 size_t work_bytes) {
    return clear_pass(ctx, d_table, m, alphabet, alen, b, n, d_h_last, d_work, work_bytes,
                      "lvs_edit_distance_clear_wide");
}

// ------------------------------------------------------------ batch plans

extern "C++" {
namespace lvs {
// Queries of a plan; refresh is the interval the plan uses (the workspace
// bound takes the shortest one).
int make_query_specs(const lvs_query* q, size_t nq, int encoding, size_t refresh, std::vector<QuerySpec>& qs) {
    qs.resize(nq);
    for (size_t k = 0; k < nq; ++k) {
        const lvs_query& x = q[k];
        QuerySpec& s = qs[k];
        s.encoding = encoding;
        s.m = x.m;
        s.n = x.n;
        s.A = x.d_a;
        s.refresh = refresh;
        s.trace = x.d_trace;
        LVS_REQUIRE(std::max(x.m, x.n) <= kMaxLen, LVS_E_INVAL, "lvs_plan: string longer than LVS_MAX_LEN");
        const bool banded = x.banded != 0;
        if (banded) {
            s.band = long(std::min<size_t>(x.ell, x.m + x.n));
            s.path = x.d_path;
            LVS_REQUIRE(x.d_path || x.m + x.n == 0, LVS_E_INVAL, "lvs_plan: NULL band path");
        } else {
            s.h_last = x.d_h_last;
            LVS_REQUIRE(x.d_h_last || x.n == 0, LVS_E_INVAL, "lvs_plan: NULL result buffer");
        }
        if (x.d_b) {
            s.B = x.d_b;
            LVS_REQUIRE(x.d_a || x.m == 0, LVS_E_INVAL, "lvs_plan: NULL buffer");
            s.eq9_out = x.d_eq9;
            s.eq1_out = encoding == LVS_ENC_ASCII7 ? x.d_eq1 : nullptr;
        } else {
            LVS_REQUIRE(!x.d_eq1 && !x.d_eq9, LVS_E_INVAL, "lvs_plan: d_eq1 / d_eq9 given for a cleartext query");
            LVS_REQUIRE((x.d_table || x.m == 0) && (x.b_clear || x.n == 0) && (x.alphabet || x.alen == 0),
                        LVS_E_INVAL, "lvs_plan: NULL buffer (cleartext query)");
            s.table = x.d_table;
            s.cols.resize(x.n);
            for (size_t j = 0; j < x.n; ++j) {
                const uint8_t* hit = std::find(x.alphabet, x.alphabet + x.alen, x.b_clear[j]);
                LVS_REQUIRE(hit != x.alphabet + x.alen, LVS_E_ALPHABET, "lvs_plan: symbol not in the table");
                s.cols[j] = int32_t(hit - x.alphabet);
            }
        }
    }
    return LVS_OK;
}
}  // namespace lvs
}  // extern "C++"

int lvs_plan_workspace_bytes(const lvs_query* queries, size_t nq, int encoding, size_t* bytes) {
    LVS_REQUIRE(bytes && (queries || nq == 0), LVS_E_INVAL, "lvs_plan_workspace_bytes: NULL argument");
    std::vector<QuerySpec> qs;
    int rc = make_query_specs(queries, nq, encoding, LVS_REFRESH_MIN, qs);
    if (rc) return rc;
    *bytes = plan_ws(qs);
    return LVS_OK;
}

int lvs_plan_create(lvs_context* ctx, const lvs_query* queries, size_t nq, int encoding, int flags, void* d_work,
                    size_t work_bytes, lvs_plan** out) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C && out && (queries || nq == 0), LVS_E_INVAL, "lvs_plan_create: bad argument");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    std::vector<QuerySpec> qs;
    int rc = make_query_specs(queries, nq, encoding, C->refresh_every, qs);
    if (rc) return rc;
    for (const auto& q : qs) LVS_CHECK_LENGTHS(C, q.m, q.n, "lvs_plan_create");
    LVS_REQUIRE(d_work && work_bytes >= plan_ws(qs), LVS_E_NOMEM_DEVICE, "lvs_plan_create: workspace too small");
    LVS_HIP(hipSetDevice(C->device));
    PlanHandle* H = new (std::nothrow) PlanHandle();
    LVS_REQUIRE(H, LVS_E_NOMEM_HOST, "lvs_plan_create: out of host memory");
    H->kind = kPlan;
    H->C = C;
    uint8_t* ws = reinterpret_cast<uint8_t*>(d_work);
    assign_buffers(qs, ws);
    const size_t cap = max_step_of(qs);
    build_edit_distance_plan(qs, H->P, true, round_of(C, cap), cap);
    hipError_t e = upload_plan(H->P, ws, C->stream);
    if (e == hipSuccess && (flags & LVS_PLAN_GRAPH)) e = capture_plan(C, H->P);
    if (e != hipSuccess) {
        delete H;
        set_error(std::string("lvs_plan_create: ") + hipGetErrorString(e));
        return LVS_E_DEVICE;
    }
    *out = reinterpret_cast<lvs_plan*>(H);
    return LVS_OK;
}

int lvs_plan_verify(const lvs_query* queries, size_t nq, int encoding, size_t round, int fill, size_t refresh,
                    size_t* steps, size_t* jobs, size_t* rounds, size_t* violations) {
    LVS_REQUIRE(queries || nq == 0, LVS_E_INVAL, "lvs_plan_verify: NULL queries");
    LVS_REQUIRE(valid_encoding(encoding), LVS_E_INVAL, "unknown encoding");
    LVS_REQUIRE(refresh == 0 || (refresh >= LVS_REFRESH_MIN && refresh <= LVS_REFRESH_MAX), LVS_E_INVAL,
                "lvs_plan_verify: bad refresh interval");
    std::vector<QuerySpec> qs;
    int rc = make_query_specs(queries, nq, encoding, refresh, qs);
    if (rc) return rc;
    // workspace buffers at addresses above every caller address; nothing is dereferenced
    uintptr_t top = 0;
    for (size_t k = 0; k < nq; ++k)
        for (uintptr_t a : {uintptr_t(queries[k].d_a), uintptr_t(queries[k].d_b), uintptr_t(queries[k].d_table),
                            uintptr_t(queries[k].d_h_last), uintptr_t(queries[k].d_path),
                            uintptr_t(queries[k].d_trace), uintptr_t(queries[k].d_eq1), uintptr_t(queries[k].d_eq9)})
            top = std::max(top, a);
    uint8_t* ws = reinterpret_cast<uint8_t*>((top + (uintptr_t(1) << 40)) & ~uintptr_t(255));
    assign_buffers(qs, ws);
    Plan P;
    const size_t cap = max_step_of(qs);
    build_edit_distance_plan(qs, P, true, fill ? round : 0, cap);
    size_t nrounds = 0;
    const size_t bad = verify_plan(P, round, cap, &nrounds);
    if (steps) *steps = P.steps.size();
    if (jobs) *jobs = P.jobs.size();
    if (rounds) *rounds = nrounds;
    if (violations) *violations = bad;
    return LVS_OK;
}

int lvs_plan_run(lvs_plan* plan) {
    auto* H = reinterpret_cast<PlanHandle*>(plan);
    LVS_REQUIRE(H && H->kind == kPlan, LVS_E_INVAL, "lvs_plan_run: bad plan");
    LVS_HIP(hipSetDevice(H->C->device));
    LVS_HIP(run_plan(H->C, H->P));
    return LVS_OK;
}

int lvs_plan_run_steps(lvs_plan* plan, size_t first, size_t count) {
    auto* H = reinterpret_cast<PlanHandle*>(plan);
    LVS_REQUIRE(H && H->kind == kPlan, LVS_E_INVAL, "lvs_plan_run_steps: bad plan");
    LVS_REQUIRE(first <= H->P.steps.size() && count <= H->P.steps.size() - first, LVS_E_INVAL,
                "lvs_plan_run_steps: steps past the end of the plan");
    LVS_HIP(hipSetDevice(H->C->device));
    LVS_HIP(run_plan_steps(H->C, H->P, first, count));
    return LVS_OK;
}

int lvs_plan_step_bootstraps(const lvs_plan* plan, size_t* counts, size_t n) {
    auto* H = reinterpret_cast<const PlanHandle*>(plan);
    LVS_REQUIRE(H && H->kind == kPlan, LVS_E_INVAL, "lvs_plan_step_bootstraps: bad plan");
    LVS_REQUIRE(counts || n == 0, LVS_E_INVAL, "lvs_plan_step_bootstraps: NULL counts");
    for (size_t k = 0; k < n && k < H->P.steps.size(); ++k)
        counts[k] = H->P.steps[k].sum >= 0 ? 0 : H->P.steps[k].count;
    return LVS_OK;
}

int lvs_plan_info(const lvs_plan* plan, size_t* steps, size_t* bootstraps, size_t* max_step) {
    auto* H = reinterpret_cast<const PlanHandle*>(plan);
    LVS_REQUIRE(H && H->kind == kPlan, LVS_E_INVAL, "lvs_plan_info: bad plan");
    if (steps) *steps = H->P.steps.size();
    if (bootstraps) *bootstraps = H->P.pbs();
    if (max_step) *max_step = H->P.max_step;
    return LVS_OK;
}

int lvs_profile_enable(lvs_context* ctx, int enable) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C, LVS_E_INVAL, "lvs_profile_enable: bad context");
    LVS_HIP(hipSetDevice(C->device));
    LVS_HIP(hipStreamSynchronize(C->stream));
    for (auto& t : C->timed) {
        C->spare.push_back(t.start);
        C->spare.push_back(t.end);
    }
    C->timed.clear();
    C->profiling = enable != 0;
    return LVS_OK;
}

int lvs_profile_read(lvs_context* ctx, int kernel, double* total_ms, uint64_t* launches, uint64_t* units) {
    Context* C = as_ctx(ctx);
    LVS_REQUIRE(C && total_ms && launches && units, LVS_E_INVAL, "lvs_profile_read: bad argument");
    LVS_HIP(hipSetDevice(C->device));
    double ms = 0;
    uint64_t n = 0, u = 0;
    for (auto& t : C->timed) {
        const bool br = t.kernel == kProfBrLatency || t.kernel == kProfBrThroughput || t.kernel == kProfBrW16 ||
                        t.kernel == kProfBrPair;
        if (t.kernel != kernel && !(kernel == kProfBlindRotate && br)) continue;
        LVS_HIP(hipEventSynchronize(t.end));
        float dt = 0;
        LVS_HIP(hipEventElapsedTime(&dt, t.start, t.end));
        ms += dt;
        ++n;
        u += t.units;
    }
    *total_ms = ms;
    *launches = n;
    *units = u;
    return LVS_OK;
}

void lvs_server_free_impl(void* h);
void lvs_engine_free_impl(void* h);

void lvs_free(void* handle) {
    if (!handle) return;
    switch (reinterpret_cast<Handle*>(handle)->kind) {
        case kClientKey: delete reinterpret_cast<ClientKey*>(handle); break;
        case kServerKey: delete reinterpret_cast<ServerKey*>(handle); break;
        case kServer: lvs_server_free_impl(handle); break;
        case kEngine: lvs_engine_free_impl(handle); break;
        case kPlan: {
            auto* H = reinterpret_cast<PlanHandle*>(handle);
            if (H->P.graph) (void)hipGraphExecDestroy(H->P.graph);   // teardown: nothing to report to
            delete H;
            break;
        }
        case kContext: {
            Context* C = reinterpret_cast<Context*>(handle);
            for (auto& t : C->timed) {
                (void)hipEventDestroy(t.start);
                (void)hipEventDestroy(t.end);
            }
            for (auto e : C->spare) (void)hipEventDestroy(e);
            if (C->capture_stream) (void)hipStreamDestroy(C->capture_stream);
            delete C;
            break;
        }
        default: break;
    }
}

}  // extern "C"
