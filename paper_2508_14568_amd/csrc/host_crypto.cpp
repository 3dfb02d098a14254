// Host-side TFHE key generation, encryption and decryption for liblvs.
//
// Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used counter-style: the stream
// of object `tag` under `seed` starts at state mix(mix(seed) ^ tag), and draw
// i is the generator's output number i + 1 from that state.  Noise is the
// 12-term Irwin-Hall approximation of a Gaussian: (sum of 12 uniform 32-bit
// words - 6 * 2^32), whose standard deviation is 2^32, times sigma * 2^64,
// divided by 2^32 with rounding toward minus infinity.  This is a test-grade
// sampler chosen so that keys and ciphertexts are reproducible bit for bit.
#include <algorithm>
#include <thread>

#include "lvs_internal.h"

namespace lvs {

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

inline uint64_t splitmix_out(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Object kinds of the key and encryption streams.
constexpr uint64_t kTagSmallKey = 1, kTagGlweKey = 2, kTagBskMask = 3, kTagBskNoise = 4, kTagKskMask = 5,
                   kTagKskNoise = 6, kTagEncMask = 7, kTagEncNoise = 8;

inline uint64_t tag(uint64_t kind, uint64_t index) { return (kind << 48) | index; }

// acc += X^shift * poly in Z_{2^64}[X]/(X^N + 1), shift in [0, N).
void add_rotated(uint64_t* acc, const uint64_t* poly, int shift) {
    for (int t = 0; t < kN - shift; ++t) acc[t + shift] += poly[t];
    for (int t = kN - shift; t < kN; ++t) acc[t + shift - kN] -= poly[t];
}

}  // namespace

uint64_t rng_key(uint64_t seed, uint64_t t) { return splitmix_out(splitmix_out(seed) ^ t); }

uint64_t rng_draw(uint64_t key, uint64_t i) { return splitmix_out(key + kGolden * (i + 1)); }

uint64_t rng_noise(uint64_t key, uint64_t idx, uint64_t sigma_q64) {
    int64_t sum = -(int64_t(6) << 32);
    for (uint64_t u = 0; u < 12; ++u) sum += int64_t(rng_draw(key, 12 * idx + u) >> 32);
    const __int128 scaled = __int128(sum) * __int128(sigma_q64);
    return uint64_t(int64_t(scaled >> 32));
}

void keygen(const lvs_params& p, uint64_t seed, ClientKey& ck, ServerKey& sk) {
    const int n = int(p.n_lwe);
    ck.p = p;
    sk.p = p;
    ck.s.resize(n);
    ck.S.resize(kN);
    const uint64_t k_small = rng_key(seed, tag(kTagSmallKey, 0));
    const uint64_t k_glwe = rng_key(seed, tag(kTagGlweKey, 0));
    for (int i = 0; i < n; ++i) ck.s[i] = uint8_t(rng_draw(k_small, i) & 1);
    for (int j = 0; j < kN; ++j) ck.S[j] = uint8_t(rng_draw(k_glwe, j) & 1);

    // Bootstrapping key: GGSW(s_i) with one gadget level g = 2^(64 - 23).
    // Row 0 carries s_i * g on the mask, row 1 on the body; each row is a
    // GLWE encryption of zero (A uniform, B = A * S + E).
    sk.bsk.assign(size_t(n) * 2 * 2 * kN, 0);
    std::vector<int> ones;
    for (int j = 0; j < kN; ++j)
        if (ck.S[j]) ones.push_back(j);
    const uint64_t g = uint64_t(1) << (64 - kPbsBaseLog);
    auto build_rows = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i)
            for (int row = 0; row < 2; ++row) {
                uint64_t* A = &sk.bsk[((size_t(i) * 2 + row) * 2 + 0) * kN];
                uint64_t* B = &sk.bsk[((size_t(i) * 2 + row) * 2 + 1) * kN];
                const uint64_t km = rng_key(seed, tag(kTagBskMask, uint64_t(i) * 2 + row));
                const uint64_t ke = rng_key(seed, tag(kTagBskNoise, uint64_t(i) * 2 + row));
                for (int t = 0; t < kN; ++t) A[t] = rng_draw(km, t);
                for (int t = 0; t < kN; ++t) B[t] = rng_noise(ke, t, p.glwe_noise_q64);
                for (int j : ones) add_rotated(B, A, j);   // B += A * X^j for every S_j = 1
                if (ck.s[i]) (row == 0 ? A[0] : B[0]) += g;
            }
    };
    const int nthreads = std::max(1, std::min(16, int(std::thread::hardware_concurrency())));
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
        pool.emplace_back(build_rows, n * t / nthreads, n * (t + 1) / nthreads);
    for (auto& th : pool) th.join();

    // Key-switching key: row j*5 + (t-1) encrypts S_j * 2^(64 - 3t) under s.
    sk.ksk.assign(size_t(kKsRows) * (n + 1), 0);
    const uint64_t k_kn = rng_key(seed, tag(kTagKskNoise, 0));
    for (uint64_t r = 0; r < uint64_t(kKsRows); ++r) {
        const int j = int(r / kKsLevel), level = int(r % kKsLevel) + 1;
        uint64_t* row = &sk.ksk[r * (n + 1)];
        const uint64_t km = rng_key(seed, tag(kTagKskMask, r));
        uint64_t body = rng_noise(k_kn, r, p.lwe_noise_q64);
        for (int c = 0; c < n; ++c) {
            row[c] = rng_draw(km, c);
            if (ck.s[c]) body += row[c];
        }
        if (ck.S[j]) body += uint64_t(1) << (64 - kKsBaseLog * level);
        row[n] = body;
    }
}

void encrypt(const ClientKey& ck, uint32_t mu, uint64_t seed, uint64_t index, uint64_t* ct) {
    const uint64_t km = rng_key(seed, tag(kTagEncMask, index));
    const uint64_t ke = rng_key(seed, tag(kTagEncNoise, index));
    uint64_t body = (uint64_t(mu & 31u) << kDeltaLog) + rng_noise(ke, 0, ck.p.glwe_noise_q64);
    for (int j = 0; j < kN; ++j) {
        ct[j] = rng_draw(km, j);
        if (ck.S[j]) body += ct[j];
    }
    ct[kN] = body;
}

uint64_t phase(const ClientKey& ck, const uint64_t* ct) {
    uint64_t acc = ct[kN];
    for (int j = 0; j < kN; ++j)
        if (ck.S[j]) acc -= ct[j];
    return acc;
}

void trivial_ct(uint32_t mu, uint64_t* ct) {
    std::fill(ct, ct + kN, uint64_t(0));
    ct[kN] = uint64_t(mu & 31u) << kDeltaLog;
}

}  // namespace lvs
