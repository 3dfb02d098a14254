/*
 * oracle/tfhe_ref.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-purpose CPU reference of the TFHE arithmetic that the
 * Leuvenshtein method runs on (the paper uses TFHE programmable bootstrapping,
 * Section 2.2, and refers to the TFHE literature for the scheme itself).  Only
 * the tests, the package smoke check and the benchmark's CPU baseline may load
 * this file's library.  It shares no code with the HIP library.
 *
 * Everything is integer arithmetic in Z/2^64 (unsigned wrap-around).  The
 * negacyclic polynomial products are written out as the schoolbook sum that
 * defines them: (a*d)[k] = sum_{i+j=k} a_i d_j - sum_{i+j=k+N} a_i d_j.
 * A key set may instead select Karatsuba's recursion for the blind rotation's
 * products (orc_keys_set_karatsuba): exact in Z/2^64 as well, pinned against
 * the schoolbook sum, about three times faster, for the full-size workloads.
 *
 * Conventions the paper leaves open (each is listed with its reading in the
 * design notes and pinned by tests):
 *   - plaintext space of 5 bits: value x in Z_32 is encoded as x * 2^59
 *     (Section 2.2: 4 free bits plus a padding bit);
 *   - ciphertexts between operations are LWE under the big key S (the
 *     coefficients of the GLWE key, dimension N); a bootstrap runs
 *     key switch -> modulus switch -> blind rotation -> sample extraction;
 *   - rounding: round-half-up everywhere ((x >> (s-1)) + 1) >> 1;
 *   - gadget digits are balanced, produced from the least significant level
 *     up with a carry, the carry out of the top level is dropped;
 *   - randomness: SplitMix64 (Steele, Lea, Flood 2014) used as a
 *     counter-based generator, keyed per object; Gaussian noise is the
 *     12-term Irwin-Hall approximation scaled by an integer sigma*2^64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;

typedef struct {
    int n;            /* small LWE dimension (bootstrapping key length)      */
    int N;            /* GLWE polynomial size, GLWE dimension k = 1          */
    int pbs_base_log; /* gadget base log of the bootstrapping key            */
    int pbs_level;    /* gadget levels of the bootstrapping key              */
    int ks_base_log;  /* key-switching base log                              */
    int ks_level;     /* key-switching levels                                */
    u64 lwe_sigma_q64;  /* noise std of small-key LWE, times 2^64            */
    u64 glwe_sigma_q64; /* noise std of GLWE / big-key LWE, times 2^64       */
} orc_params;

typedef struct {
    orc_params p;
    uint8_t* s;   /* small key, n bits                                       */
    uint8_t* S;   /* GLWE key polynomial, N bits (also the big LWE key)      */
    u64* bsk;     /* [n][2*pbs_level][2][N]: GGSW(s_i) rows, (mask, body)    */
    u64* ksk;     /* [N*ks_level][n+1]: LWE_s(S_j * 2^(64 - B*t))            */
    int karatsuba; /* blind rotation's products: 0 schoolbook, 1 Karatsuba   */
} orc_keys;

/* ---------------------------------------------------------------- PRNG */

#define ORC_PHI 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function. */
static u64 sm_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Stream key for object `tag` under `seed`; draw i is the (i+1)-th output of
 * a SplitMix64 generator whose state starts at that key. */
u64 orc_stream_key(u64 seed, u64 tag) { return sm_mix(sm_mix(seed) ^ tag); }
u64 orc_draw(u64 key, u64 i) { return sm_mix(key + (i + 1) * ORC_PHI); }

#define ORC_TAG(kind, idx) (((u64)(kind) << 48) | (u64)(idx))
enum { K_LWE_KEY = 1, K_GLWE_KEY = 2, K_BSK_MASK = 3, K_BSK_NOISE = 4,
       K_KSK_MASK = 5, K_KSK_NOISE = 6, K_ENC_MASK = 7, K_ENC_NOISE = 8 };

/* Noise sample idx of a stream: (sum of 12 uniform 32-bit draws - 6*2^32)
 * has mean 0 and standard deviation 2^32; scale by sigma*2^64 and divide by
 * 2^32 rounding toward minus infinity. */
u64 orc_gaussian(u64 key, u64 idx, u64 sigma_q64) {
    i64 acc = 0;
    for (int t = 0; t < 12; ++t) acc += (i64)(orc_draw(key, 12 * idx + (u64)t) >> 32);
    acc -= (i64)6 << 32;
    __int128 prod = (__int128)acc * (__int128)sigma_q64;
    return (u64)(i64)(prod >> 32);
}

/* ------------------------------------------------ polynomial arithmetic */

/* out += a * d in Z_{2^64}[X]/(X^N + 1), schoolbook, one output coefficient
 * at a time: out[k] += sum_i a[i] * dd[k - i], where dd extends d
 * negacyclically (dd[t] = d[t] for t >= 0 and dd[t] = -d[t + N] for t < 0,
 * because X^N = -1).  a holds torus coefficients, d small signed integers.
 * The loop is compiled twice so that hosts with 64-bit vector multiplies use
 * them; the arithmetic is identical. */
#define ORC_NEGACYCLIC_MAC_BODY                                                   \
    u64* r = (u64*)malloc(sizeof(u64) * (size_t)(2 * N));   /* r[x] = dd[N-1-x] */ \
    for (int x = 0; x < 2 * N - 1; ++x) {                                         \
        const int t = N - 1 - x;                                                  \
        r[x] = (t >= 0) ? (u64)d[t] : (u64)0 - (u64)d[t + N];                     \
    }                                                                             \
    for (int k = 0; k < N; ++k) {                                                 \
        const u64* rk = r + (N - 1 - k);               /* rk[i] = dd[k - i] */    \
        u64 acc = 0;                                                              \
        for (int i = 0; i < N; ++i) acc += a[i] * rk[i];                          \
        out[k] += acc;                                                            \
    }                                                                             \
    free(r);

__attribute__((target("avx512f,avx512dq,avx512vl")))
static void negacyclic_mac_avx512(u64* restrict out, const u64* restrict a, const i64* restrict d, int N) { ORC_NEGACYCLIC_MAC_BODY }
__attribute__((target("avx2")))
static void negacyclic_mac_avx2(u64* restrict out, const u64* restrict a, const i64* restrict d, int N) { ORC_NEGACYCLIC_MAC_BODY }
static void negacyclic_mac_plain(u64* restrict out, const u64* restrict a, const i64* restrict d, int N) { ORC_NEGACYCLIC_MAC_BODY }

void orc_negacyclic_mac(u64* out, const u64* a, const i64* d, int N) {
    static int isa = -1;
    if (isa < 0) {
        __builtin_cpu_init();
        isa = __builtin_cpu_supports("avx512dq") && __builtin_cpu_supports("avx512vl") ? 2
            : __builtin_cpu_supports("avx2") ? 1 : 0;
    }
    if (isa == 2) negacyclic_mac_avx512(out, a, d, N);
    else if (isa == 1) negacyclic_mac_avx2(out, a, d, N);
    else negacyclic_mac_plain(out, a, d, N);
}

/* Karatsuba's product of two polynomials of n coefficients (n a power of
 * two), without reduction: c[0 .. 2n) = a * b over Z/2^64 (c[2n-1] = 0).
 * Writing a = a0 + X^h a1 and b = b0 + X^h b1 (h = n/2),
 *   a*b = a0 b0 + X^h ((a0 + a1)(b0 + b1) - a0 b0 - a1 b1) + X^n a1 b1,
 * which uses only the ring's additions, subtractions and products, so the
 * result is exact in Z/2^64.  Products of ORC_KARA_BASE coefficients (or of
 * fewer, for a shorter polynomial) are the schoolbook double sum.  work holds
 * at least 4n words. */
#define ORC_KARA_BASE 8
static void kara_full(u64* restrict c, const u64* restrict a, const u64* restrict b, int n, u64* restrict work) {
    if (n == ORC_KARA_BASE) {          /* the base case with constant bounds */
        u64 acc[2 * ORC_KARA_BASE] = {0};
        for (int i = 0; i < ORC_KARA_BASE; ++i)
            for (int j = 0; j < ORC_KARA_BASE; ++j) acc[i + j] += a[i] * b[j];
        for (int t = 0; t < 2 * ORC_KARA_BASE; ++t) c[t] = acc[t];
        return;
    }
    if (n < ORC_KARA_BASE) {
        for (int t = 0; t < 2 * n; ++t) c[t] = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) c[i + j] += a[i] * b[j];
        return;
    }
    const int h = n / 2;
    u64* sa = work;              /* a0 + a1                         */
    u64* sb = work + h;          /* b0 + b1                         */
    u64* mid = work + n;         /* (a0 + a1)(b0 + b1), n words     */
    kara_full(c, a, b, h, work + 2 * n);             /* a0 b0 -> c[0 .. n)   */
    kara_full(c + n, a + h, b + h, h, work + 2 * n); /* a1 b1 -> c[n .. 2n)  */
    for (int t = 0; t < h; ++t) { sa[t] = a[t] + a[h + t]; sb[t] = b[t] + b[h + t]; }
    kara_full(mid, sa, sb, h, work + 2 * n);
    for (int t = 0; t < n; ++t) mid[t] -= c[t] + c[n + t];
    for (int t = 0; t < n; ++t) c[h + t] += mid[t];
}

/* out += a * d in Z_{2^64}[X]/(X^N + 1) through Karatsuba's full product,
 * then the reduction X^N = -1: out[k] += c[k] - c[k + N].  Same words as
 * orc_negacyclic_mac for every input (N a power of two).  buf holds 7N
 * words of scratch. */
static void negacyclic_mac_karatsuba_buf(u64* out, const u64* a, const i64* d, int N, u64* buf) {
    u64* du = buf;               /* d as words of Z/2^64 (two's complement)  */
    u64* c = buf + N;            /* the full product, 2N words               */
    u64* work = buf + 3 * N;     /* Karatsuba's scratch, 4N words            */
    for (int t = 0; t < N; ++t) du[t] = (u64)d[t];
    kara_full(c, a, du, N, work);
    for (int k = 0; k < N; ++k) out[k] += c[k] - c[k + N];
}

void orc_negacyclic_mac_karatsuba(u64* out, const u64* a, const i64* d, int N) {
    u64* buf = (u64*)malloc(sizeof(u64) * (size_t)(7 * N));
    negacyclic_mac_karatsuba_buf(out, a, d, N, buf);
    free(buf);
}

/* out = X^e * a for e in [0, 2N): coefficient t takes a[(t - e) mod 2N] when
 * that index is below N, else minus a[that index - N]. */
void orc_monomial_mul(u64* out, const u64* a, int e, int N) {
    for (int t = 0; t < N; ++t) {
        int src = ((t - e) % (2 * N) + 2 * N) % (2 * N);
        out[t] = (src < N) ? a[src] : (u64)0 - a[src - N];
    }
}

/* Balanced gadget decomposition of one torus value into `level` digits of
 * base 2^base_log; digit[lev] has weight 2^(64 - base_log*(lev+1)). */
void orc_decompose(u64 c, int base_log, int level, i64* digit) {
    const int prec = base_log * level;
    u64 r = ((c >> (63 - prec)) + 1) >> 1;          /* round(c / 2^(64-prec)) */
    if (prec < 64) r &= ((u64)1 << prec) - 1;
    const u64 mask = ((u64)1 << base_log) - 1;
    const i64 half = (i64)1 << (base_log - 1);
    for (int lev = level - 1; lev >= 0; --lev) {
        i64 dig = (i64)(r & mask);
        r >>= base_log;
        if (dig >= half) { dig -= (i64)1 << base_log; r += 1; }
        digit[lev] = dig;
    }
}

/* ------------------------------------------------------------- keygen */

typedef struct { orc_keys* k; u64 seed; int i0, i1; } bsk_job;

static void* bsk_worker(void* arg) {
    bsk_job* jb = (bsk_job*)arg;
    const orc_params* p = &jb->k->p;
    const int N = p->N, L = p->pbs_level, R = 2 * L;
    i64* Sd = (i64*)malloc(sizeof(i64) * N);
    for (int j = 0; j < N; ++j) Sd[j] = jb->k->S[j];
    for (int i = jb->i0; i < jb->i1; ++i) {
        for (int rho = 0; rho < R; ++rho) {
            u64* A = jb->k->bsk + (((size_t)i * R + rho) * 2 + 0) * N;
            u64* B = jb->k->bsk + (((size_t)i * R + rho) * 2 + 1) * N;
            const u64 km = orc_stream_key(jb->seed, ORC_TAG(K_BSK_MASK, (u64)i * R + rho));
            const u64 ke = orc_stream_key(jb->seed, ORC_TAG(K_BSK_NOISE, (u64)i * R + rho));
            for (int j = 0; j < N; ++j) A[j] = orc_draw(km, (u64)j);
            for (int j = 0; j < N; ++j) B[j] = orc_gaussian(ke, (u64)j, p->glwe_sigma_q64);
            orc_negacyclic_mac(B, A, Sd, N);              /* B = A*S + E */
            const int c = rho / L, lev = rho % L;
            const u64 g = (u64)1 << (64 - p->pbs_base_log * (lev + 1));
            if (jb->k->s[i]) { if (c == 0) A[0] += g; else B[0] += g; }
        }
    }
    free(Sd);
    return NULL;
}

orc_keys* orc_keygen(const orc_params* p, u64 seed, int nthreads) {
    orc_keys* k = (orc_keys*)calloc(1, sizeof(orc_keys));
    k->p = *p;
    const int n = p->n, N = p->N, R = 2 * p->pbs_level, L = p->ks_level;
    k->s = (uint8_t*)malloc((size_t)n);
    k->S = (uint8_t*)malloc((size_t)N);
    k->bsk = (u64*)malloc(sizeof(u64) * (size_t)n * R * 2 * N);
    k->ksk = (u64*)malloc(sizeof(u64) * (size_t)N * L * (n + 1));
    const u64 ks = orc_stream_key(seed, ORC_TAG(K_LWE_KEY, 0));
    for (int i = 0; i < n; ++i) k->s[i] = (uint8_t)(orc_draw(ks, (u64)i) & 1);
    const u64 kS = orc_stream_key(seed, ORC_TAG(K_GLWE_KEY, 0));
    for (int j = 0; j < N; ++j) k->S[j] = (uint8_t)(orc_draw(kS, (u64)j) & 1);

    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    bsk_job* jobs = (bsk_job*)malloc(sizeof(bsk_job) * nthreads);
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].k = k; jobs[t].seed = seed;
        jobs[t].i0 = (int)((long)n * t / nthreads);
        jobs[t].i1 = (int)((long)n * (t + 1) / nthreads);
        pthread_create(&th[t], NULL, bsk_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th); free(jobs);

    const u64 kn = orc_stream_key(seed, ORC_TAG(K_KSK_NOISE, 0));
    for (int j = 0; j < N; ++j) {
        for (int t = 1; t <= L; ++t) {
            const u64 r = (u64)j * L + (u64)(t - 1);
            u64* row = k->ksk + r * (u64)(n + 1);
            const u64 km = orc_stream_key(seed, ORC_TAG(K_KSK_MASK, r));
            u64 b = 0;
            for (int c = 0; c < n; ++c) { row[c] = orc_draw(km, (u64)c); b += row[c] * (u64)k->s[c]; }
            b += (u64)k->S[j] << (64 - p->ks_base_log * t);
            b += orc_gaussian(kn, r, p->lwe_sigma_q64);
            row[n] = b;
        }
    }
    return k;
}

/* Selects how the blind rotation multiplies polynomials: 0 the schoolbook
 * sum (the default), 1 Karatsuba's product.  Both give the same words. */
void orc_keys_set_karatsuba(orc_keys* k, int on) { k->karatsuba = on ? 1 : 0; }

void orc_keys_free(orc_keys* k) {
    if (!k) return;
    free(k->s); free(k->S); free(k->bsk); free(k->ksk); free(k);
}

const uint8_t* orc_keys_small(const orc_keys* k) { return k->s; }
const uint8_t* orc_keys_big(const orc_keys* k) { return k->S; }
const u64* orc_keys_bsk(const orc_keys* k) { return k->bsk; }
const u64* orc_keys_ksk(const orc_keys* k) { return k->ksk; }

/* --------------------------------------------------- encrypt / decrypt */

/* Big-key LWE encryption of mu in Z_32 as ciphertext number `index` drawn
 * under `seed`: a uniform, b = <a, S> + mu * 2^59 + e. */
void orc_encrypt(const orc_keys* k, u32 mu, u64 seed, u64 index, u64* ct) {
    const int N = k->p.N;
    const u64 km = orc_stream_key(seed, ORC_TAG(K_ENC_MASK, index));
    const u64 ke = orc_stream_key(seed, ORC_TAG(K_ENC_NOISE, index));
    u64 b = 0;
    for (int j = 0; j < N; ++j) { ct[j] = orc_draw(km, (u64)j); b += ct[j] * (u64)k->S[j]; }
    b += (u64)(mu & 31u) << 59;
    b += orc_gaussian(ke, 0, k->p.glwe_sigma_q64);
    ct[N] = b;
}

/* Phase b - <a, S> of a big-key LWE ciphertext. */
u64 orc_phase(const orc_keys* k, const u64* ct) {
    const int N = k->p.N;
    u64 ph = ct[N];
    for (int j = 0; j < N; ++j) ph -= ct[j] * (u64)k->S[j];
    return ph;
}

/* Phase of a small-key LWE ciphertext (dimension n). */
u64 orc_phase_small(const orc_keys* k, const u64* ct) {
    const int n = k->p.n;
    u64 ph = ct[n];
    for (int j = 0; j < n; ++j) ph -= ct[j] * (u64)k->s[j];
    return ph;
}

/* ------------------------------------------- bootstrap building blocks */

/* Key switch from the big key (dimension N) to the small key (dimension n):
 * out = (0, b) - sum_{j,t} d_{j,t} * KSK[j][t]. */
void orc_keyswitch(const orc_keys* k, const u64* in, u64* out) {
    const int n = k->p.n, N = k->p.N, L = k->p.ks_level;
    i64 dig[64];
    memset(out, 0, sizeof(u64) * (size_t)(n + 1));
    out[n] = in[N];
    for (int j = 0; j < N; ++j) {
        orc_decompose(in[j], k->p.ks_base_log, L, dig);
        for (int t = 0; t < L; ++t) {
            const u64 d = (u64)dig[t];
            const u64* row = k->ksk + ((u64)j * L + (u64)t) * (u64)(n + 1);
            for (int c = 0; c <= n; ++c) out[c] -= d * row[c];
        }
    }
}

/* Modulus switch of every word from 2^64 to 2N, rounding half up. */
void orc_modswitch(int n, int N, const u64* in, u32* out) {
    int log2n2 = 0;
    while ((1 << log2n2) < 2 * N) ++log2n2;
    for (int c = 0; c <= n; ++c)
        out[c] = (u32)((((in[c] >> (63 - log2n2)) + 1) >> 1) & (u64)(2 * N - 1));
}

/* Blind rotation: ACC = (0, X^{-b} * testpoly); then for each i
 * ACC += ExtProd(BSK_i, X^{a_i} * ACC - ACC).  acc is [2][N] (mask, body). */
void orc_blind_rotate(const orc_keys* k, const u64* testpoly, const u32* ms, u64* acc) {
    const int n = k->p.n, N = k->p.N, L = k->p.pbs_level, R = 2 * L;
    u64* A = acc;
    u64* B = acc + N;
    memset(A, 0, sizeof(u64) * (size_t)N);
    orc_monomial_mul(B, testpoly, (int)((2 * N - ms[n]) % (2 * N)), N);
    u64* rot = (u64*)malloc(sizeof(u64) * 2 * N);
    i64* D = (i64*)malloc(sizeof(i64) * (size_t)R * N);   /* [c*L + lev][N] */
    i64 dig[64];
    u64* kbuf = k->karatsuba ? (u64*)malloc(sizeof(u64) * 7 * (size_t)N) : NULL;
    for (int i = 0; i < n; ++i) {
        orc_monomial_mul(rot, A, (int)ms[i], N);
        orc_monomial_mul(rot + N, B, (int)ms[i], N);
        for (int t = 0; t < N; ++t) { rot[t] -= A[t]; rot[N + t] -= B[t]; }
        for (int c = 0; c < 2; ++c)
            for (int t = 0; t < N; ++t) {
                orc_decompose(rot[c * N + t], k->p.pbs_base_log, L, dig);
                for (int lev = 0; lev < L; ++lev) D[(size_t)(c * L + lev) * N + t] = dig[lev];
            }
        for (int rho = 0; rho < R; ++rho) {
            const u64* rowA = k->bsk + (((size_t)i * R + rho) * 2 + 0) * N;
            const u64* rowB = k->bsk + (((size_t)i * R + rho) * 2 + 1) * N;
            if (kbuf) {
                negacyclic_mac_karatsuba_buf(A, rowA, D + (size_t)rho * N, N, kbuf);
                negacyclic_mac_karatsuba_buf(B, rowB, D + (size_t)rho * N, N, kbuf);
            } else {
                orc_negacyclic_mac(A, rowA, D + (size_t)rho * N, N);
                orc_negacyclic_mac(B, rowB, D + (size_t)rho * N, N);
            }
        }
    }
    free(rot); free(D); free(kbuf);
}

/* Sample extraction of coefficient 0 into a big-key LWE ciphertext. */
void orc_sample_extract(int N, const u64* acc, u64* out) {
    out[0] = acc[0];
    for (int j = 1; j < N; ++j) out[j] = (u64)0 - acc[N - j];
    out[N] = acc[N];
}

/* Programmable bootstrap: sample_extract(blind_rotate(modswitch(keyswitch))). */
void orc_pbs(const orc_keys* k, const u64* testpoly, const u64* in, u64* out) {
    const int n = k->p.n, N = k->p.N;
    u64* small = (u64*)malloc(sizeof(u64) * (size_t)(n + 1));
    u32* ms = (u32*)malloc(sizeof(u32) * (size_t)(n + 1));
    u64* acc = (u64*)malloc(sizeof(u64) * 2 * (size_t)N);
    orc_keyswitch(k, in, small);
    orc_modswitch(n, N, small, ms);
    orc_blind_rotate(k, testpoly, ms, acc);
    orc_sample_extract(N, acc, out);
    free(small); free(ms); free(acc);
}

typedef struct {
    const orc_keys* k; const u64* polys; const int32_t* lut; const u64* in; u64* out;
    size_t B; size_t next; pthread_mutex_t* mu;
} pbs_job;

static void* pbs_worker(void* arg) {
    pbs_job* jb = (pbs_job*)arg;
    const size_t W = (size_t)jb->k->p.N + 1;
    for (;;) {
        pthread_mutex_lock(jb->mu);
        size_t b = jb->next++;
        pthread_mutex_unlock(jb->mu);
        if (b >= jb->B) break;
        orc_pbs(jb->k, jb->polys + (size_t)jb->lut[b] * jb->k->p.N, jb->in + b * W, jb->out + b * W);
    }
    return NULL;
}

/* B independent bootstraps, ciphertext b with test polynomial lut[b]; the
 * work is spread over nthreads threads (results do not depend on it). */
void orc_pbs_batch(const orc_keys* k, const u64* polys, const int32_t* lut, const u64* in,
                   size_t B, u64* out, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if ((size_t)nthreads > B) nthreads = (int)(B ? B : 1);
    pthread_mutex_t mu;
    pthread_mutex_init(&mu, NULL);
    pbs_job jb = {k, polys, lut, in, out, B, 0, &mu};
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, pbs_worker, &jb);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&mu);
}
