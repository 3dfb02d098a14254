// Constants of the exact negacyclic products: four NTT primes, twiddle
// tables, Montgomery and explicit-CRT constants.
//
// A product of a decomposed polynomial (23-bit signed digits) with a GGSW row
// (64-bit coefficients read as signed) has integer coefficients bounded by
// 2 * N * 2^22 * 2^63 = 2^97 for the two rows of one external product.  With
// four primes p_r < 2^26, p_r = 1 mod 2N, Q = prod p_r ~ 2^104 > 2^98, so the
// residues determine the signed integer exactly (CRT with a signed lift) and
// its value mod 2^64 is the torus result.  Primes below 2^26 leave 6 bits of
// headroom in 32-bit words, so the transforms can skip most reductions.
#include <mutex>

#include "lvs_internal.h"

namespace lvs {

namespace {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return uint64_t((unsigned __int128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

bool is_prime(uint64_t n) {
    if (n < 2) return false;
    for (uint64_t q : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

uint32_t bitrev(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (bits - 1 - b);
    return r;
}

uint32_t shoup(uint32_t w, uint32_t p) { return uint32_t((uint64_t(w) << 32) / p); }

PrimeTables build() {
    PrimeTables t{};
    // The four largest primes below 2^26 that are 1 mod 2N = 4096.
    int found = 0;
    for (uint64_t k = ((uint64_t(1) << kPrimeBits) - 1) / (2 * kN); found < kPrimes; --k) {
        const uint64_t p = k * 2 * kN + 1;
        if (p < (uint64_t(1) << kPrimeBits) && is_prime(p)) t.p[found++] = uint32_t(p);
    }
    t.fwd.resize(size_t(kPrimes) * kN);
    t.fwd_shoup.resize(size_t(kPrimes) * kN);
    t.inv.resize(size_t(kPrimes) * kN);
    t.inv_shoup.resize(size_t(kPrimes) * kN);
    for (int r = 0; r < kPrimes; ++r) {
        const uint64_t p = t.p[r];
        // psi: a primitive 2N-th root of unity (psi^N = -1).
        uint64_t psi = 0;
        for (uint64_t x = 2;; ++x) {
            psi = powmod(x, (p - 1) / (2 * kN), p);
            if (powmod(psi, kN, p) == p - 1) break;
        }
        const uint64_t psi_inv = powmod(psi, p - 2, p);
        for (int k = 0; k < kN; ++k) {
            const uint32_t e = bitrev(uint32_t(k), kLogN);
            const uint32_t wf = uint32_t(powmod(psi, e, p)), wi = uint32_t(powmod(psi_inv, e, p));
            t.fwd[size_t(r) * kN + k] = wf;
            t.fwd_shoup[size_t(r) * kN + k] = shoup(wf, uint32_t(p));
            t.inv[size_t(r) * kN + k] = wi;
            t.inv_shoup[size_t(r) * kN + k] = shoup(wi, uint32_t(p));
        }
        // Montgomery: -p^{-1} mod 2^32 by Newton iteration.
        uint32_t inv = uint32_t(p);
        for (int it = 0; it < 5; ++it) inv *= 2u - uint32_t(p) * inv;
        t.mont_neg_inv[r] = 0u - inv;
        t.reduce_q[r] = uint32_t((uint64_t(1) << 32) / p);
    }
    // Explicit CRT: the residues reaching the CRT are y_i = X (Q/p_i)^{-1} mod
    // p_i because the transforms are linear and the weight (Q/p_i)^{-1} is
    // folded into the key together with 1/N; then X = sum y_i M_i - K Q.
    uint64_t Q = 1;
    for (int i = 0; i < kPrimes; ++i) Q *= t.p[i];
    t.Q_mod64 = Q;
    for (int r = 0; r < kPrimes; ++r) {
        const uint64_t p = t.p[r];
        uint64_t m64 = 1, mp = 1;
        for (int j = 0; j < kPrimes; ++j)
            if (j != r) {
                m64 *= t.p[j];
                mp = mulmod(mp, t.p[j], p);
            }
        t.crt_m[r] = m64;
        t.crt_g[r] = uint32_t((uint64_t(1) << 57) / p);
        const uint64_t c = powmod(mp, p - 2, p);            // (Q/p)^{-1} mod p
        const uint64_t ninv = powmod(kN, p - 2, p);
        t.bsk_scale[r] = uint32_t(mulmod(mulmod(ninv, c, p), (uint64_t(1) << 32) % p, p));
    }
    return t;
}

}  // namespace

const PrimeTables& prime_tables() {
    static PrimeTables tables = build();
    return tables;
}

}  // namespace lvs
