// Wire format of keys and ciphertexts (the outsourcing setting of the
// paper's introduction: the client encrypts and keeps the secret key, the
// server computes on ciphertexts with the public server key and returns
// encrypted results).
//
// Every object is one record, all integers little-endian:
//   magic "LVS1" | u32 kind | u32 n_lwe, glwe_k, poly_N, pbs_base_log,
//   pbs_level, ks_base_log, ks_level | u64 lwe_noise_q64, glwe_noise_q64 |
//   u64 count | u64 payload bytes | payload | u64 FNV-1a of the payload
// count is the number of ciphertexts for LVS_WIRE_CIPHERTEXTS and 0 for keys.
// Payloads: client key = the small key's n bits then the GLWE key's N bits,
// one byte each; server key = the bootstrapping key's words then the key
// switching key's words; ciphertexts = count x (N+1) words.
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lvs_internal.h"

namespace lvs {
namespace {

constexpr size_t kHeader = 4 + 4 + 7 * 4 + 2 * 8 + 8 + 8;
constexpr size_t kTrailer = 8;

uint64_t fnv1a(const uint8_t* p, size_t n) {
    uint64_t h = 1469598103934665603ULL;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}

struct Writer {
    uint8_t* p;
    void u32(uint32_t v) {
        for (int k = 0; k < 4; ++k) *p++ = uint8_t(v >> (8 * k));
    }
    void u64(uint64_t v) {
        for (int k = 0; k < 8; ++k) *p++ = uint8_t(v >> (8 * k));
    }
    void bytes(const void* src, size_t n) {
        std::memcpy(p, src, n);
        p += n;
    }
    void words(const uint64_t* w, size_t n) {
        for (size_t i = 0; i < n; ++i) u64(w[i]);
    }
};

struct Reader {
    const uint8_t* p;
    const uint8_t* end;
    bool ok = true;
    bool need(size_t n) {
        if (size_t(end - p) < n) ok = false;
        return ok;
    }
    uint32_t u32() {
        if (!need(4)) return 0;
        uint32_t v = 0;
        for (int k = 0; k < 4; ++k) v |= uint32_t(*p++) << (8 * k);
        return v;
    }
    uint64_t u64() {
        if (!need(8)) return 0;
        uint64_t v = 0;
        for (int k = 0; k < 8; ++k) v |= uint64_t(*p++) << (8 * k);
        return v;
    }
};

struct Record {
    uint32_t kind;
    lvs_params params;
    uint64_t count;
    const uint8_t* payload;
    uint64_t payload_bytes;
};

size_t record_bytes(size_t payload) { return kHeader + payload + kTrailer; }

void write_record(uint8_t* buf, uint32_t kind, const lvs_params& p, uint64_t count, size_t payload_bytes,
                  void (*fill)(Writer&, const void*), const void* obj) {
    Writer w{buf};
    w.bytes("LVS1", 4);
    w.u32(kind);
    for (uint32_t v : {p.n_lwe, p.glwe_k, p.poly_N, p.pbs_base_log, p.pbs_level, p.ks_base_log, p.ks_level}) w.u32(v);
    w.u64(p.lwe_noise_q64);
    w.u64(p.glwe_noise_q64);
    w.u64(count);
    w.u64(payload_bytes);
    uint8_t* start = w.p;
    fill(w, obj);
    w.u64(fnv1a(start, payload_bytes));
}

// Parses and checks a record (magic, sizes, checksum, parameter set).
int read_record(const uint8_t* buf, size_t len, Record& r) {
    if (!buf || len < kHeader + kTrailer) {
        set_error("lvs_import: record too short");
        return LVS_E_INVAL;
    }
    if (std::memcmp(buf, "LVS1", 4) != 0) {
        set_error("lvs_import: not an lvs record");
        return LVS_E_INVAL;
    }
    Reader rd{buf + 4, buf + len};
    r.kind = rd.u32();
    lvs_params& p = r.params;
    p.n_lwe = rd.u32();
    p.glwe_k = rd.u32();
    p.poly_N = rd.u32();
    p.pbs_base_log = rd.u32();
    p.pbs_level = rd.u32();
    p.ks_base_log = rd.u32();
    p.ks_level = rd.u32();
    p.lwe_noise_q64 = rd.u64();
    p.glwe_noise_q64 = rd.u64();
    r.count = rd.u64();
    r.payload_bytes = rd.u64();
    if (!rd.ok || r.payload_bytes > len - kHeader - kTrailer || record_bytes(r.payload_bytes) != len) {
        set_error("lvs_import: record length does not match its header");
        return LVS_E_INVAL;
    }
    r.payload = rd.p;
    Reader tail{r.payload + r.payload_bytes, buf + len};
    if (tail.u64() != fnv1a(r.payload, r.payload_bytes)) {
        set_error("lvs_import: checksum mismatch");
        return LVS_E_INVAL;
    }
    if (!params_supported(p)) {
        set_error("lvs_import: parameter set not supported by the kernels");
        return LVS_E_PARAMS;
    }
    return LVS_OK;
}

void fill_client(Writer& w, const void* obj) {
    const auto* k = static_cast<const ClientKey*>(obj);
    w.bytes(k->s.data(), k->s.size());
    w.bytes(k->S.data(), k->S.size());
}

void fill_server(Writer& w, const void* obj) {
    const auto* k = static_cast<const ServerKey*>(obj);
    w.words(k->bsk.data(), k->bsk.size());
    w.words(k->ksk.data(), k->ksk.size());
}

struct CtSpan {
    const uint64_t* cts;
    size_t words;
};

void fill_cts(Writer& w, const void* obj) {
    const auto* s = static_cast<const CtSpan*>(obj);
    w.words(s->cts, s->words);
}

size_t bsk_words(const lvs_params& p) { return size_t(p.n_lwe) * 2 * 2 * p.poly_N; }
size_t ksk_words(const lvs_params& p) { return size_t(p.poly_N) * p.ks_level * (p.n_lwe + 1); }

}  // namespace
}  // namespace lvs

using namespace lvs;

extern "C" {

int lvs_export(int kind, const void* obj, size_t count, uint8_t* buf, size_t* len) {
    if (!obj || !len) {
        set_error("lvs_export: NULL argument");
        return LVS_E_INVAL;
    }
    const auto* h = static_cast<const Handle*>(obj);
    size_t payload = 0;
    lvs_params p{};
    void (*fill)(Writer&, const void*) = nullptr;
    CtSpan span{};
    const void* src = obj;
    if (kind == LVS_WIRE_CLIENT_KEY) {
        if (h->kind != kClientKey) {
            set_error("lvs_export: not a client key");
            return LVS_E_INVAL;
        }
        const auto* k = static_cast<const ClientKey*>(obj);
        p = k->p;
        payload = k->s.size() + k->S.size();
        fill = fill_client;
        count = 0;
    } else if (kind == LVS_WIRE_SERVER_KEY) {
        if (h->kind != kServerKey) {
            set_error("lvs_export: not a server key");
            return LVS_E_INVAL;
        }
        const auto* k = static_cast<const ServerKey*>(obj);
        p = k->p;
        payload = 8 * (k->bsk.size() + k->ksk.size());
        fill = fill_server;
        count = 0;
    } else if (kind == LVS_WIRE_CIPHERTEXTS) {
        if (count > (SIZE_MAX - kHeader - kTrailer) / (8 * size_t(kCtWords))) {
            set_error("lvs_export: too many ciphertexts for one record");
            return LVS_E_INVAL;
        }
        lvs_params_default(&p);
        span = CtSpan{static_cast<const uint64_t*>(obj), count * size_t(kCtWords)};
        payload = 8 * span.words;
        fill = fill_cts;
        src = &span;
    } else {
        set_error("lvs_export: unknown kind");
        return LVS_E_INVAL;
    }
    const size_t need = record_bytes(payload);
    if (!buf) {
        *len = need;
        return LVS_OK;
    }
    if (*len < need) {
        *len = need;
        set_error("lvs_export: buffer too small");
        return LVS_E_INVAL;
    }
    write_record(buf, uint32_t(kind), p, count, payload, fill, src);
    *len = need;
    return LVS_OK;
}

int lvs_import_key(const uint8_t* buf, size_t len, int* kind, void** out) {
    if (!kind || !out) {
        set_error("lvs_import_key: NULL argument");
        return LVS_E_INVAL;
    }
    Record r{};
    int rc = read_record(buf, len, r);
    if (rc) return rc;
    const lvs_params& p = r.params;
    if (r.kind == LVS_WIRE_CLIENT_KEY) {
        if (r.payload_bytes != size_t(p.n_lwe) + p.poly_N) {
            set_error("lvs_import_key: client key payload of the wrong size");
            return LVS_E_INVAL;
        }
        for (size_t i = 0; i < r.payload_bytes; ++i)
            if (r.payload[i] > 1) {
                set_error("lvs_import_key: key bit outside {0, 1}");
                return LVS_E_INVAL;
            }
        auto* k = new (std::nothrow) ClientKey();
        if (!k) {
            set_error("lvs_import_key: out of host memory");
            return LVS_E_NOMEM_HOST;
        }
        k->kind = kClientKey;
        k->p = p;
        try {
            k->s.assign(r.payload, r.payload + p.n_lwe);
            k->S.assign(r.payload + p.n_lwe, r.payload + p.n_lwe + p.poly_N);
        } catch (const std::bad_alloc&) {
            delete k;
            set_error("lvs_import_key: out of host memory");
            return LVS_E_NOMEM_HOST;
        }
        *kind = LVS_WIRE_CLIENT_KEY;
        *out = k;
        return LVS_OK;
    }
    if (r.kind == LVS_WIRE_SERVER_KEY) {
        if (r.payload_bytes != 8 * (bsk_words(p) + ksk_words(p))) {
            set_error("lvs_import_key: server key payload of the wrong size");
            return LVS_E_INVAL;
        }
        auto* k = new (std::nothrow) ServerKey();
        if (!k) {
            set_error("lvs_import_key: out of host memory");
            return LVS_E_NOMEM_HOST;
        }
        k->kind = kServerKey;
        k->p = p;
        try {
            k->bsk.resize(bsk_words(p));
            k->ksk.resize(ksk_words(p));
        } catch (const std::bad_alloc&) {
            delete k;
            set_error("lvs_import_key: out of host memory");
            return LVS_E_NOMEM_HOST;
        }
        Reader rd{r.payload, r.payload + r.payload_bytes};
        for (auto& v : k->bsk) v = rd.u64();
        for (auto& v : k->ksk) v = rd.u64();
        *kind = LVS_WIRE_SERVER_KEY;
        *out = k;
        return LVS_OK;
    }
    set_error("lvs_import_key: the record holds no key");
    return LVS_E_INVAL;
}

int lvs_import_ciphertexts(const uint8_t* buf, size_t len, uint64_t* out, size_t* count) {
    if (!count) {
        set_error("lvs_import_ciphertexts: NULL argument");
        return LVS_E_INVAL;
    }
    Record r{};
    int rc = read_record(buf, len, r);
    if (rc) return rc;
    if (r.kind != LVS_WIRE_CIPHERTEXTS || r.count > r.payload_bytes / (8 * uint64_t(kCtWords)) ||
        r.payload_bytes != 8 * r.count * uint64_t(kCtWords)) {
        set_error("lvs_import_ciphertexts: the record holds no ciphertexts");
        return LVS_E_INVAL;
    }
    if (!out) {
        *count = size_t(r.count);
        return LVS_OK;
    }
    if (*count < r.count) {
        *count = size_t(r.count);
        set_error("lvs_import_ciphertexts: output too small");
        return LVS_E_INVAL;
    }
    Reader rd{r.payload, r.payload + r.payload_bytes};
    for (size_t i = 0; i < r.count * kCtWords; ++i) out[i] = rd.u64();
    *count = size_t(r.count);
    return LVS_OK;
}

}  // extern "C"
