// Internal declarations shared by the host and device halves of liblvs.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lvs.h"

namespace lvs {

// Parameter set the kernels are written for.
constexpr int kN = 2048;           // GLWE polynomial size (k = 1)
constexpr int kLogN = 11;
constexpr int kCtWords = kN + 1;   // big-key LWE ciphertext
constexpr int kSmallN = 742;       // small LWE dimension
constexpr int kSmallWords = kSmallN + 1;
constexpr int kPbsBaseLog = 23;    // gadget base of the bootstrapping key, one level
constexpr int kKsBaseLog = 3;      // key switching: base 2^3, 5 levels
constexpr int kKsLevel = 5;
constexpr int kKsRows = kN * kKsLevel;
constexpr int kDeltaLog = 59;      // x in Z_32 encodes as x << 59
constexpr int kPrimes = 4;         // NTT primes of the exact negacyclic products
constexpr int kPrimeBits = 26;     // every prime is below 2^26

// Every handle starts with a tag so lvs_free can dispatch.
enum HandleKind : uint32_t { kClientKey = 0x4C565301, kServerKey = 0x4C565302, kContext = 0x4C565303, kPlan = 0x4C565304,
                             kServer = 0x4C565305, kEngine = 0x4C565306 };

struct Handle {
    uint32_t kind;
};

struct ClientKey : Handle {
    lvs_params p;
    std::vector<uint8_t> s;   // small key, n bits
    std::vector<uint8_t> S;   // GLWE key (= big LWE key), N bits
};

struct ServerKey : Handle {
    lvs_params p;
    std::vector<uint64_t> bsk;  // [n][2][2][N]: GGSW(s_i) rows (mask row, body row) x (mask, body)
    std::vector<uint64_t> ksk;  // [N * 5][n + 1]: LWE_s(S_j * 2^(64 - 3t))
};

void set_error(const std::string& msg);
bool params_supported(const lvs_params& p);

// Host crypto (host_crypto.cpp).
uint64_t rng_key(uint64_t seed, uint64_t tag);
uint64_t rng_draw(uint64_t key, uint64_t i);
uint64_t rng_noise(uint64_t key, uint64_t idx, uint64_t sigma_q64);
void keygen(const lvs_params& p, uint64_t seed, ClientKey& ck, ServerKey& sk);
void encrypt(const ClientKey& ck, uint32_t mu, uint64_t seed, uint64_t index, uint64_t* ct);
uint64_t phase(const ClientKey& ck, const uint64_t* ct);
void trivial_ct(uint32_t mu, uint64_t* ct);

// NTT constants (ntt_consts.cpp).
struct PrimeTables {
    uint32_t p[kPrimes];
    uint32_t mont_neg_inv[kPrimes];          // -p^{-1} mod 2^32
    // forward / inverse twiddles psi^{+-brv(k)} in [0, p) with Shoup companions floor(w 2^32 / p)
    std::vector<uint32_t> fwd, fwd_shoup, inv, inv_shoup;   // [kPrimes][kN]
    // N^{-1} (Q/p)^{-1} 2^32 mod p: the bootstrapping key's scale (Montgomery
    // form of the 1/N of the inverse transform and of the CRT weight)
    uint32_t bsk_scale[kPrimes];
    uint32_t reduce_q[kPrimes];              // floor(2^32 / p): reduction of a word to [0, 2p)
    // explicit CRT: X = sum_i y_i M_i - K Q with y_i = X (Q/p_i)^{-1} mod p_i
    uint64_t crt_m[kPrimes];                 // M_i = Q / p_i mod 2^64
    uint32_t crt_g[kPrimes];                 // floor(2^57 / p_i): fixed-point 1/p_i for K
    uint64_t Q_mod64;                        // p_0 p_1 p_2 p_3 mod 2^64
};
const PrimeTables& prime_tables();

}  // namespace lvs
