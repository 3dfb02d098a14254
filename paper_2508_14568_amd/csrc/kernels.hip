// gfx950 kernels of liblvs: key switching, blind rotation with exact
// multi-prime NTT products, bootstrapping-key conversion, and the linear
// ciphertext operations of the Leuvenshtein cell update.
//
// Integer arithmetic only.  A negacyclic product of the blind rotation is
// evaluated modulo four primes p_r < 2^26 (p_r = 1 mod 2N) by length-2048
// negacyclic NTTs and recombined with Garner's CRT and a signed lift; the
// integers involved are below 2^97 in magnitude while prod p_r ~ 2^104, so the
// torus result mod 2^64 is exact.
//
// Work mapping of the blind rotation: one workgroup per bootstrap; the
// wavefronts of prime p_r transform the decomposed mask polynomial in lanes
// 0-31 and the decomposed body polynomial in lanes 32-63, 64 (four-wave
// form) or 32 (eight-wave form, two waves per prime) coefficients per lane in
// registers: butterfly stages inside the lane, one LDS transpose, more stages
// inside the lane.  A lane-half swap (ds_bpermute) gives every lane both
// transformed digits of its positions for the products with the
// bootstrapping key; the inverse transform runs the same way back.  The 64-bit
// accumulator lives in registers, spread over the threads as the CRT
// reconstructs it; the decomposition digits are computed once per workgroup
// from an LDS copy of it, and after each external product the four residue
// sets meet in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "launch.h"
#include "lvs_internal.h"

namespace lvs {
namespace dev {

constexpr int kHalfLanes = 32;            // lanes per polynomial
constexpr int kEh = kN / kHalfLanes;       // 64 coefficients per lane
constexpr int kPoly = kN + kN / 64;        // LDS words of one padded polynomial

struct CrtConsts {
    uint32_t p[kPrimes];
    uint32_t mont[kPrimes];
    uint32_t red[kPrimes];                 // floor(2^32 / p)
    uint32_t g[kPrimes];                   // floor(2^57 / p)
    uint64_t m[kPrimes];                   // Q / p mod 2^64
    uint64_t Q;                            // Q mod 2^64
};

struct Tw {
    const uint2* fwd;       // [kPrimes][kN] (twiddle, Shoup companion)
    const uint2* inv;
};

// LDS word of coefficient j: one pad word per 64 keeps both transpose
// directions free of bank conflicts.
__device__ __forceinline__ uint32_t pad(uint32_t j) { return j + (j >> 6); }

// arr[w] for a wave-uniform w without dynamic indexing of kernel arguments.
__device__ __forceinline__ uint32_t pick(const uint32_t (&arr)[kPrimes], int w) {
    return w == 0 ? arr[0] : w == 1 ? arr[1] : w == 2 ? arr[2] : arr[3];
}

// a * w mod p in [0, 2p) for any a < 2^32 (Shoup, ws = floor(w 2^32 / p)).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t ws, uint32_t p) {
    const uint32_t q = __umulhi(a, ws);
    return a * w - q * p;
}

// x - c if x >= c else x (unsigned).
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t c) { return min(x, x - c); }

// Montgomery reduction: T * 2^-32 mod p in [0, 2p) for T < p 2^32.
__device__ __forceinline__ uint32_t redc(uint64_t T, uint32_t p, uint32_t mont) {
    const uint32_t m = uint32_t(T) * mont;
    return uint32_t((T + uint64_t(m) * p) >> 32);
}

// x mod p in [0, 2p) for any 32-bit x (Shoup reduction by 1, q = floor(2^32/p)).
__device__ __forceinline__ uint32_t reduce2p(uint32_t x, uint32_t q, uint32_t p) { return x - __umulhi(x, q) * p; }

// Value of the same register in lane ^ 32 (the other polynomial's lane).
__device__ __forceinline__ uint32_t swap_halves(uint32_t v, int lane) {
    return uint32_t(__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, int(v)));
}

// Forward negacyclic NTT of one polynomial held by a half wavefront
// (Cooley-Tukey, psi-merged twiddles, natural order in, bit-reversed order
// out).  In: lane lh holds coefficient lh + 32 e in x[e], each < 2p.  Out: x[e]
// holds transform position 64 lh + e, each < 24p.  No reduction is needed:
// a butterfly adds at most 2p to a value (x' = a + t, y' = a - t + 2p with
// t = w b mod p in [0, 2p)), and 2p + 11 * 2p < 2^31 for p < 2^26.
// Every stage is a template instance so that all register indices are
// compile-time constants.
//
// A lane may hold only NE of the 64 elements, elements e0 .. e0 + NE - 1 (the
// half-element forms below); stages whose partners lie within that range
// then run unchanged, with the twiddle of the element's global index.
template <int S, int NE = kEh>
__device__ __forceinline__ void fwd_stage(uint32_t (&x)[NE], const uint2* w, uint32_t p, int lh, int e0 = 0) {
    // S < 6: stride 1024 >> S, partners 32 >> S elements apart, uniform twiddles;
    // S >= 6: partners 1 << (10 - S) elements apart, one twiddle block per lane
    constexpr int half = (S < 6) ? (32 >> S) : (1 << (10 - S));
    static_assert(half < NE, "partners must lie in the lane's elements");
    // twiddle of element e = e0 + el: w[base + (e >> sh)]; e0 is 0 or 32, a
    // multiple of 2^sh whenever el < 32 can reach sh < 6, so the index splits
    // into a per-stage pointer and a compile-time offset
    constexpr int sh = (S < 6) ? (6 - S) : (11 - S);
    const int base = (S < 6) ? (1 << S) : (1 << S) + (lh << (S - 5));
    const uint2* wb = w + base + (e0 >> sh);
    const uint32_t two_p = 2 * p;
#pragma unroll
    for (int el = 0; el < NE; ++el) {
        if (el & half) continue;
        const uint2 tw = wb[el >> sh];
        // s = q p - w b = -t (mod 2^32) for the Shoup product t = w b mod p in
        // [0, 2p), so that a + t = a - s and a + 2p - t = a + 2p + s (v_add3)
        const uint32_t b = x[el + half];
        const uint32_t s = __umulhi(b, tw.y) * p - b * tw.x;
        const uint32_t a = x[el];
        x[el] = a - s;
        x[el + half] = a + two_p + s;
    }
}

// kSync: a workgroup barrier before the first write to scr (the caller's
// other waves may still be reading that memory).
template <bool kSync>
__device__ __forceinline__ void ntt_forward(uint32_t (&x)[kEh], uint32_t* scr, const uint2* w, uint32_t p, int lh) {
    fwd_stage<0>(x, w, p, lh);
    fwd_stage<1>(x, w, p, lh);
    fwd_stage<2>(x, w, p, lh);
    fwd_stage<3>(x, w, p, lh);
    fwd_stage<4>(x, w, p, lh);
    fwd_stage<5>(x, w, p, lh);
    if (kSync) __syncthreads();
    // transpose: coefficient lh + 32 e -> lane j >> 6, element j & 63
#pragma unroll
    for (int e = 0; e < kEh; ++e) scr[pad(lh + 32 * e)] = x[e];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < kEh; ++e) x[e] = scr[pad(64 * lh + e)];
    __builtin_amdgcn_wave_barrier();
    fwd_stage<6>(x, w, p, lh);
    fwd_stage<7>(x, w, p, lh);
    fwd_stage<8>(x, w, p, lh);
    fwd_stage<9>(x, w, p, lh);
    fwd_stage<10>(x, w, p, lh);
}

// Inverse negacyclic NTT without the 1/N factor (Gentleman-Sande, inverse
// psi twiddles, bit-reversed order in, natural order out).  In: x[e] holds
// position 64 lh + e, each < 2p.  Out: x[e] holds coefficient lh + 32 e as a
// residue below 16p (not reduced: the CRT accepts it).  A butterfly maps
// inputs below B to a sum below 2B and a product below 2p; the sums are
// brought back below 2p after stages 3 and 7, so B never exceeds 16p and
// a + B - b stays below 32p < 2^31.
template <int U, int NE = kEh>
__device__ __forceinline__ void inv_stage(uint32_t (&x)[NE], const uint2* w, uint32_t p, uint32_t q, int lh,
                                          int e0 = 0) {
    constexpr int half = (U < 5) ? (1 << U) : (1 << (U - 5));
    static_assert(half < NE, "partners must lie in the lane's elements");
    constexpr int since = (U <= 3) ? U : (U <= 7 ? U - 4 : U - 8);   // stages since the last reduction
    constexpr bool reduce = (U == 3 || U == 7);
    const uint32_t bound = (2 * p) << since;
    constexpr int sh = (U < 5) ? (U + 1) : (U - 4);
    const int base = (U < 5) ? (1 << (10 - U)) + (lh << (5 - U)) : (1 << (10 - U));
    const uint2* wb = w + base + (e0 >> sh);
#pragma unroll
    for (int el = 0; el < NE; ++el) {
        if (el & half) continue;
        const uint2 tw = wb[el >> sh];
        const uint32_t a = x[el], b = x[el + half];
        const uint32_t sum = a + b;
        x[el] = reduce ? reduce2p(sum, q, p) : sum;
        x[el + half] = mul_shoup(a + bound - b, tw.x, tw.y, p);
    }
}

// The per-lane stages (forward S >= 6, inverse U < 5) with their twiddles
// loaded ahead into registers: a lane holding elements e0 .. e0 + NE - 1 needs
// NE >> sh distinct twiddles per stage, so that the loads of a whole phase can
// be issued before the barrier that precedes it and wait there in the memory
// pipeline instead of stalling each stage.
template <int S, int NE>
struct FwdTw {
    uint2 v[NE >> (11 - S)];
};
template <int S, int NE>
__device__ __forceinline__ void load_fwd_tw(FwdTw<S, NE>& t, const uint2* w, int lh, int e0) {
    static_assert(S >= 6, "per-lane stages only");
    constexpr int sh = 11 - S;
    const uint2* wb = w + (1 << S) + (lh << (S - 5)) + (e0 >> sh);
#pragma unroll
    for (int k = 0; k < (NE >> sh); ++k) t.v[k] = wb[k];
}
template <int S, int NE>
__device__ __forceinline__ void fwd_stage_tw(uint32_t (&x)[NE], const FwdTw<S, NE>& t, uint32_t p) {
    constexpr int half = 1 << (10 - S);
    constexpr int sh = 11 - S;
    const uint32_t two_p = 2 * p;
#pragma unroll
    for (int el = 0; el < NE; ++el) {
        if (el & half) continue;
        const uint2 tw = t.v[el >> sh];
        const uint32_t b = x[el + half];
        const uint32_t s = __umulhi(b, tw.y) * p - b * tw.x;
        const uint32_t a = x[el];
        x[el] = a - s;
        x[el + half] = a + two_p + s;
    }
}
template <int U, int NE>
struct InvTw {
    uint2 v[NE >> (U + 1)];
};
template <int U, int NE>
__device__ __forceinline__ void load_inv_tw(InvTw<U, NE>& t, const uint2* w, int lh, int e0) {
    static_assert(U < 5, "per-lane stages only");
    constexpr int sh = U + 1;
    const uint2* wb = w + (1 << (10 - U)) + (lh << (5 - U)) + (e0 >> sh);
#pragma unroll
    for (int k = 0; k < (NE >> sh); ++k) t.v[k] = wb[k];
}
// Sign and offset plan of the in-lane inverse stages of the eight-wave forms.
// A butterfly needs one instruction for its sum and one for the input of its
// product when either its b element arrives negated (register -b: sum a - b,
// product input a + b + B) or its a element arrives with an offset B, a
// multiple of p no smaller than b's bound (product input a - b, sum
// a + b + c for any wanted offset c).  The plan arranges one of the two for
// every butterfly of the transform:
//  * row stages 0..4 (element bit j at stage j): the products enter stage 0
//    with the a elements offset by 2p (added to their Montgomery product's
//    high word); along the chain of sums of sums (elements whose low j bits
//    are zero, up to the reduction after stage 3) the sums add the next
//    stage's bound to their a elements in the same add3; every other output
//    is produced negated where the next stage takes it as b (products as
//    q p - x w instead of x w - q p, sums as b - a);
//  * stage 4 ends the row segment with the values of the wave holding the
//    positions with bit 5 set negated, so that column stage 5 (position bit
//    5, element bit 0 of the column layout) starts with its b elements
//    negated and every column stage keeps them so; stage 9 likewise negates
//    the half with position bit 10 set, which the CRT step's last stage takes
//    as b.
// The integers that reach the Shoup products, the reductions and the CRT are
// those of plain butterflies (a + b and a - b + B), so the bounds above hold
// unchanged.
template <int J, int RED, bool CHAIN>
struct InvPlan {
    static constexpr bool chain(int j, int el) { return CHAIN && j <= RED && (el & ((1 << j) - 1)) == 0; }
    // 1: b negated; 2: a offset by B
    static constexpr int mode(int el) { return chain(J, el) ? 2 : 1; }
    static constexpr bool next_b(int e) { return (e >> (J + 1)) & 1; }
};

// One butterfly of the plan: B and Bn are the bounds (multiples of p) of this
// stage and the next, q = floor(2^32 / p); NEG: the segment's last stage
// negates its outputs.
template <int J, int RED, bool CHAIN, bool NEG, int EL>
__device__ __forceinline__ void inv_bfly_plan(uint32_t& xa, uint32_t& xb, uint2 tw, uint32_t p, uint32_t q,
                                              uint32_t B, uint32_t Bn) {
    using Pl = InvPlan<J, RED, CHAIN>;
    constexpr int m = Pl::mode(EL);
    const uint32_t a = xa, b = xb;
    const uint32_t x = (m == 1) ? a + b + B : a - b;     // product input: the plain a - b + B
    if constexpr (J == RED) {
        // the plain sum, reduced below 2p
        const uint32_t sum = (m == 1) ? a - b : a + b - B;
        const uint32_t qq = __umulhi(sum, q) * p;
        xa = Pl::next_b(EL) ? qq - sum : sum - qq;
    } else if constexpr (J == 4) {
        static_assert(m == 1, "the last stage of a segment follows its reduction");
        xa = NEG ? b - a : a - b;
    } else if constexpr (Pl::chain(J + 1, EL)) {
        static_assert(m == 2, "chain sums come from chain pairs");
        const uint32_t c = Pl::next_b(EL) ? 0u : Bn;
        xa = a + b + (c - B);
    } else {
        static_assert(m == 1, "other sums come from pairs with b negated");
        xa = Pl::next_b(EL) ? b - a : a - b;
    }
    const uint32_t qd = __umulhi(x, tw.y);
    constexpr bool neg_d = (J == 4) ? NEG : Pl::next_b(EL + (1 << J));
    xb = neg_d ? qd * p - x * tw.x : x * tw.x - qd * p;
}

// The butterfly of element EL if EL is the a element of its pair (bit J clear);
// its twiddle is tws[EL >> sh].
template <int J, int RED, bool CHAIN, bool NEG, int EL, int NE>
__device__ __forceinline__ void inv_elem_plan(uint32_t (&x)[NE], const uint2* tws, int sh, uint32_t p, uint32_t q,
                                              uint32_t B, uint32_t Bn) {
    if constexpr (!((EL >> J) & 1))
        inv_bfly_plan<J, RED, CHAIN, NEG, EL>(x[EL], x[EL + (1 << J)], tws[EL >> sh], p, q, B, Bn);
}
template <int J, int RED, bool CHAIN, bool NEG, int NE, int... E>
__device__ __forceinline__ void inv_stage_plan(uint32_t (&x)[NE], const uint2* tws, int sh, uint32_t p, uint32_t q,
                                               uint32_t B, uint32_t Bn, std::integer_sequence<int, E...>) {
    (inv_elem_plan<J, RED, CHAIN, NEG, E>(x, tws, sh, p, q, B, Bn), ...);
}

// Row stages 0..4 of the plan (NEG: stage 4 of the wave whose positions have
// bit 5 set).
template <bool NEG = false, int U, int NE>
__device__ __forceinline__ void inv_stage_tw(uint32_t (&x)[NE], const InvTw<U, NE>& t, uint32_t p, uint32_t q) {
    static_assert(NE == 32, "the sign plan covers 32 elements per lane");
    static_assert(U == 4 || !NEG, "only the segment's last stage negates");
    constexpr int since = (U <= 3) ? U : U - 4;
    constexpr int since_next = (U + 1 <= 3) ? U + 1 : U - 3;
    inv_stage_plan<U, 3, true, NEG>(x, t.v, U + 1, p, q, (2 * p) << since, (2 * p) << since_next,
                                    std::make_integer_sequence<int, NE>{});
}

// The stages with wave-uniform twiddles (forward S < 6, inverse U >= 5) read
// from an LDS copy tl of entries 0 .. 63 of the prime's table: the waits for
// them then count on the LDS counter, not behind the key loads on the
// in-order vector memory counter.
template <int S, int NE>
__device__ __forceinline__ void fwd_stage_lds(uint32_t (&x)[NE], const uint2* tl, uint32_t p, int e0) {
    static_assert(S >= 1 && S < 6, "wave-uniform stages only");
    constexpr int half = 32 >> S;
    constexpr int sh = 6 - S;
    const uint2* wb = tl + (1 << S) + (e0 >> sh);
    const uint32_t two_p = 2 * p;
#pragma unroll
    for (int el = 0; el < NE; ++el) {
        if (el & half) continue;
        const uint2 tw = wb[el >> sh];
        const uint32_t b = x[el + half];
        const uint32_t s = __umulhi(b, tw.y) * p - b * tw.x;
        const uint32_t a = x[el];
        x[el] = a - s;
        x[el + half] = a + two_p + s;
    }
}
// Column stages 5..9 of the plan (NEG: stage 9 of the wave whose positions
// have bit 10 set).
template <int U, int NE, bool NEG = false>
__device__ __forceinline__ void inv_stage_lds(uint32_t (&x)[NE], const uint2* tl, uint32_t p, uint32_t q, int e0) {
    static_assert(U >= 5 && U < 10, "wave-uniform stages only");
    static_assert(NE == 32, "the sign plan covers 32 elements per lane");
    static_assert(U == 9 || !NEG, "only the segment's last stage negates");
    constexpr int since = (U <= 7) ? U - 4 : U - 8;
    constexpr int since_next = (U + 1 <= 7) ? U - 3 : U - 7;
    constexpr int sh = U - 4;
    inv_stage_plan<U - 5, 2, false, NEG>(x, tl + (1 << (10 - U)) + (e0 >> sh), sh, p, q, (2 * p) << since,
                                         (2 * p) << since_next, std::make_integer_sequence<int, NE>{});
}

__device__ __forceinline__ void ntt_inverse(uint32_t (&x)[kEh], uint32_t* scr, const uint2* w, uint32_t p, uint32_t q,
                                            int lh) {
    inv_stage<0>(x, w, p, q, lh);
    inv_stage<1>(x, w, p, q, lh);
    inv_stage<2>(x, w, p, q, lh);
    inv_stage<3>(x, w, p, q, lh);
    inv_stage<4>(x, w, p, q, lh);
    // transpose: position 64 lh + e -> lane j & 31, element j >> 5
#pragma unroll
    for (int e = 0; e < kEh; ++e) scr[pad(64 * lh + e)] = x[e];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < kEh; ++e) x[e] = scr[pad(lh + 32 * e)];
    __builtin_amdgcn_wave_barrier();
    inv_stage<5>(x, w, p, q, lh);
    inv_stage<6>(x, w, p, q, lh);
    inv_stage<7>(x, w, p, q, lh);
    inv_stage<8>(x, w, p, q, lh);
    inv_stage<9>(x, w, p, q, lh);
    inv_stage<10>(x, w, p, q, lh);
}

// Explicit CRT.  y_i (any representative below 2^30) of X (Q/p_i)^{-1} mod
// p_i for a signed integer |X| <= 2^97 < Q / 2^6.9 -> acc + X mod 2^64.  As
// integers sum_i y_i (Q/p_i) = X + K Q with K = sum_i y_i / p_i - X / Q, so K
// is the integer nearest sum y_i / p_i (within 2^-6.9 of it).
//
// K in 32-bit words: with G_i = floor(2^56 / p_i), floor(y_i G_i / 2^32) is
// y_i / p_i in units of 2^-24, low by less than 1 + y_i / 2^32 < 1.25 units,
// so the sum s of the four is below sum y_i / p_i by less than 5 units
// (2^-21.7) and (s + 2^23) >> 24 rounds to K; s < 2^30.1 (p_i > 2^25.9).
// X mod 2^64 = sum y_i (Q/p_i mod 2^64) - K Q: the 32x32-bit products with
// the low words are chained into acc by 64-bit multiply-adds, the products
// with the high words only add their low words at bit 32.
__device__ __forceinline__ uint64_t crt_add(uint64_t acc, const uint32_t (&y)[kPrimes], const CrtConsts& C) {
    uint32_t s = 1u << 23, h = 0;
    uint64_t r = acc;
#pragma unroll
    for (int i = 0; i < kPrimes; ++i) {
        s += __umulhi(y[i], C.g[i] >> 1);
        r += uint64_t(y[i]) * uint32_t(C.m[i]);
        h += y[i] * uint32_t(C.m[i] >> 32);
    }
    const uint32_t K = s >> 24;
    const uint64_t nQ = uint64_t(0) - C.Q;
    r += uint64_t(K) * uint32_t(nQ);
    h += K * uint32_t(nQ >> 32);
    return r + (uint64_t(h) << 32);
}

// ------------------------------------------------------------ key switch

constexpr int kKsSub = 128;                      // input coefficients per LDS round
constexpr int kKsCols = (kSmallWords + 255) / 256;

__global__ void __launch_bounds__(256) fill_u64_kernel(uint64_t* p, size_t count, uint64_t v) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Input word w of a job: sum_k coef[k] * src[k][w] (the body delta is added
// by the blind rotation, which reads the body itself).
__device__ __forceinline__ uint64_t job_word(const Job& J, int w) {
    uint64_t v = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (J.src[k]) v += uint64_t(int64_t(J.coef[k])) * J.src[k][w];
    return v;
}

// part[split][b][c] = - sum_{j in split, t} d_{j,t} KSK[j*5+t][c] for the
// input of job b (mask coefficients only; the body is added later).  Digits:
// round to 15 bits, then balanced base-8 digits from the least significant
// level with a carry (level t weight 2^(64-3t)); the top carry is dropped.
// One KSK row's words of a thread's columns; a column past the last reads
// the last column (its sums are never stored).
__device__ __forceinline__ void ks_load_row(uint64_t (&k)[kKsCols], const uint64_t* row, int tid) {
#pragma unroll
    for (int cs = 0; cs < kKsCols; ++cs) k[cs] = row[min(tid + 256 * cs, kSmallWords - 1)];
}

// The products of one row with the tile's biased digits (dp: one byte per
// ciphertext, T of them): sum (d + 4) k = sum (d + 4) k_lo + 2^32 sum (d + 4)
// k_hi (mod 2^64), the first sum kept in 64 bits (a 32 x 32 + 64
// multiply-add per product), the second in 32 bits; ksum collects the rows
// for the bias.
template <int T>
__device__ __forceinline__ void ks_row_products(const uint64_t* dp, const uint64_t (&k)[kKsCols],
                                                uint64_t (&acc_lo)[T][kKsCols], uint32_t (&acc_hi)[T][kKsCols],
                                                uint64_t (&ksum)[kKsCols]) {
#pragma unroll
    for (int cs = 0; cs < kKsCols; ++cs) ksum[cs] += k[cs];
    uint64_t w[(T + 7) / 8];
#pragma unroll
    for (int q = 0; q < (T + 7) / 8; ++q) w[q] = dp[q];
#pragma unroll
    for (int bb = 0; bb < T; ++bb) {
        const uint32_t d = uint32_t(w[bb >> 3] >> (8 * (bb & 7))) & 0xFFu;
#pragma unroll
        for (int cs = 0; cs < kKsCols; ++cs) {
            acc_lo[bb][cs] += uint64_t(d) * uint32_t(k[cs]);
            acc_hi[bb][cs] += d * uint32_t(k[cs] >> 32);
        }
    }
}

// Tiles of T job inputs x all n+1 output columns per workgroup: each KSK row
// is read once per tile and multiplied with the tile's T digits.
template <int T>
__global__ void __launch_bounds__(256) keyswitch_jobs_kernel(const Job* __restrict__ jobs, int B,
                                                             const uint64_t* __restrict__ ksk,
                                                             uint64_t* __restrict__ part, int chunk, int sub) {
    // one byte per row and tile ciphertext (rows padded to whole 8-byte
    // words): the balanced digit d in [-4, 4) stored as d + 4.  The products
    // then take unsigned 32 x 64-bit multiply-adds, and the bias comes off
    // once per split: sum (d + 4) k - 4 sum k = sum d k (mod 2^64).
    constexpr int kWords = (T + 7) / 8;
    __shared__ uint64_t digits[kKsSub * kKsLevel * kWords];
    const int tid = threadIdx.x;
    const int b0 = blockIdx.x * T;
    const int split = blockIdx.y;
    uint8_t* dig8 = reinterpret_cast<uint8_t*>(digits);
    uint64_t acc_lo[T][kKsCols];
    uint32_t acc_hi[T][kKsCols];
    uint64_t ksum[kKsCols];
#pragma unroll
    for (int cs = 0; cs < kKsCols; ++cs) ksum[cs] = 0;
#pragma unroll
    for (int bb = 0; bb < T; ++bb)
#pragma unroll
        for (int cs = 0; cs < kKsCols; ++cs) acc_lo[bb][cs] = acc_hi[bb][cs] = 0;
    for (int j0 = split * chunk; j0 < (split + 1) * chunk; j0 += sub) {
        __syncthreads();
        for (int idx = tid; idx < T * sub; idx += 256) {
            const int bb = idx / sub, jj = idx % sub;
            uint64_t c = 0;
            if (b0 + bb < B) c = job_word(jobs[b0 + bb], j0 + jj);
            uint64_t r = (((c >> 48) + 1) >> 1) & 0x7FFFu;     // round(c / 2^49) mod 2^15
#pragma unroll
            for (int lev = kKsLevel - 1; lev >= 0; --lev) {
                int d = int(r & 7u);
                r >>= 3;
                if (d >= 4) { d -= 8; r += 1; }
                dig8[(jj * kKsLevel + lev) * 8 * kWords + bb] = uint8_t(d + 4);
            }
        }
        __syncthreads();
        const uint64_t* rows = ksk + size_t(j0) * kKsLevel * kSmallWords;
        for (int rr = 0; rr < sub * kKsLevel; ++rr) {
            uint64_t k[kKsCols];
            ks_load_row(k, rows + size_t(rr) * kSmallWords, tid);
            ks_row_products<T>(digits + rr * kWords, k, acc_lo, acc_hi, ksum);
        }
    }
#pragma unroll
    for (int bb = 0; bb < T; ++bb) {
        if (b0 + bb >= B) break;
#pragma unroll
        for (int cs = 0; cs < kKsCols; ++cs) {
            const int col = tid + 256 * cs;
            // -sum d k over this split's rows
            const uint64_t acc = acc_lo[bb][cs] + (uint64_t(acc_hi[bb][cs]) << 32);
            if (col < kSmallWords) part[(size_t(split) * B + b0 + bb) * kSmallWords + col] = 4 * ksum[cs] - acc;
        }
    }
}

// ---------------------------------------------------------- blind rotation

struct BrArgs {
    const Job* jobs;           // [B]
    const uint64_t* part;      // [nsplit][B][n+1] key-switch partial sums (before modulus switching)
    int nsplit;
    const uint64_t* luts;      // [LVS_LUT_SLOTS][N] test polynomials
    const uint32_t* bsk;       // [n][kPrimes][2 rows][2 comps][N] NTT domain, Montgomery form, 1/N folded
    Tw tw;
    CrtConsts crt;
    int B;
};

constexpr int kBrThreads = 256;
constexpr int kAccPer = 2 * kN / kBrThreads;   // accumulator coefficients held by a thread
constexpr size_t kBrLds = sizeof(uint32_t) * kPrimes * 2 * kPoly                 // per-prime regions
                          + sizeof(uint32_t) * (kSmallWords + 1);                 // switched mask and body

// One workgroup of 4 wavefronts per bootstrap, two workgroups per CU.
//
// The 64-bit accumulator lives in registers: thread t owns coefficient
// c = t + 256 k' of polynomial k & 1 (k' = k >> 1), the same coefficients it
// reconstructs in the CRT step.  LDS holds four regions of 2 x kPoly words,
// one per prime; a CMux step uses them in turn as
//   (1) the accumulator's low and high words (regions 0 and 1), each thread
//       writing its own coefficients at the positions it alone reads in (5);
//   (2) the balanced digits of X^a ACC - ACC (region 2), every thread
//       forming its 16 digits from the rotated copy;
//   (3) per-wave transpose scratch of the forward transform (region of the
//       wave's prime), after a barrier that ends every read of the digits;
//   (4) the inverse transform's scratch, then its residues in natural order;
//   (5) the CRT of every owned coefficient from the four regions.
// Two workgroups fit on a CU; the bootstrapping-key values are loaded where
// the products need them.
__global__ void __launch_bounds__(kBrThreads, 2) blind_rotate_kernel(BrArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* region = reinterpret_cast<uint32_t*>(lds);   // [kPrimes][2][kPoly]
    uint32_t* abar = region + kPrimes * 2 * kPoly;          // [n+1]
    uint32_t* acc_lo = region;                             // [2][kPoly], step (1)
    uint32_t* acc_hi = region + 2 * kPoly;
    uint32_t* dig = region + 4 * kPoly;                    // [2][kPoly], step (2)

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int h = lane >> 5;          // 0: mask polynomial, 1: body polynomial
    const int lh = lane & 31;
    const uint32_t p = pick(A.crt.p, wave);
    const uint32_t mont = pick(A.crt.mont, wave);
    const uint32_t q = pick(A.crt.red, wave);
    const uint2* fw = A.tw.fwd + size_t(wave) * kN;
    const uint2* iw = A.tw.inv + size_t(wave) * kN;
    uint32_t* scr = region + (wave * 2 + h) * kPoly;
    // a digit d in [-2^22, 2^22) is stored as d + 2^22; adding p - 2^22 gives
    // a residue of d below 2p
    const uint32_t unbias = p - (1u << 22);

    for (int b = blockIdx.x; b < A.B; b += gridDim.x) {
        const Job& J = A.jobs[b];
        // finish the key switch (sum of the partial sums, plus the input body)
        // and switch the modulus to Z_{2N}: round(x / 2^52)
        for (int c = tid; c < kSmallWords; c += kBrThreads) {
            uint64_t v = 0;
            for (int sp = 0; sp < A.nsplit; ++sp) v += A.part[(size_t(sp) * A.B + b) * kSmallWords + c];
            if (c == kSmallN) v += job_word(J, kN) + J.delta;
            abar[c] = uint32_t((((v >> 51) + 1) >> 1) & (2 * kN - 1));
        }
        __syncthreads();
        const int lut = min(int(J.lut), LVS_LUT_SLOTS - 1);   // ids past the table clamp
        const uint64_t* tp = A.luts + size_t(lut) * kN;
        const uint32_t bbar = abar[kSmallN];
        // ACC = (0, X^{-bbar} * testpoly)
        uint64_t acc[kAccPer];
#pragma unroll
        for (int k = 0; k < kAccPer; ++k) {
            const uint32_t c = uint32_t(tid + kBrThreads * (k >> 1));
            const uint32_t src = (c + bbar) & (2 * kN - 1);
            const uint64_t v = tp[src & (kN - 1)];
            acc[k] = (k & 1) ? ((src < uint32_t(kN)) ? v : uint64_t(0) - v) : uint64_t(0);
        }

        for (int i = 0; i < kSmallN; ++i) {
            const uint32_t a = abar[i];
            // this step's bootstrapping-key values of the lane:
            // K[k * 32] = (K0[2k], K1[2k], K0[2k+1], K1[2k+1]) of positions 64 lh + 2k, + 1
            const uint4* K = reinterpret_cast<const uint4*>(A.bsk) + ((size_t(i) * kPrimes + wave) * 2 + h) * (kN / 2) + lh;
            // (1)
#pragma unroll
            for (int k = 0; k < kAccPer; ++k) {
                const int at = (k & 1) * kPoly + tid + kBrThreads * (k >> 1);
                acc_lo[at] = uint32_t(acc[k]);
                acc_hi[at] = uint32_t(acc[k] >> 32);
            }
            __syncthreads();
            // (2) digits of X^a ACC - ACC: round(t / 2^41) as a balanced 23-bit digit
#pragma unroll
            for (int k = 0; k < kAccPer; ++k) {
                const int qq = k & 1;
                const uint32_t c = uint32_t(tid + kBrThreads * (k >> 1));
                const uint32_t src = (c - a) & (2 * kN - 1);
                const int at = qq * kPoly + int(src & (kN - 1));
                uint64_t r = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
                if (src >= uint32_t(kN)) r = uint64_t(0) - r;
                const uint64_t t = r - acc[k];
                const uint32_t u = ((uint32_t(t >> 40) + 1) >> 1) & 0x7FFFFFu;   // round(t / 2^41) mod 2^23
                dig[qq * kPoly + c] = (u + 0x400000u) & 0x7FFFFFu;                // balanced digit + 2^22
            }
            __syncthreads();
            // (3)
            uint32_t x[kEh];
#pragma unroll
            for (int e = 0; e < kEh; ++e) x[e] = dig[h * kPoly + lh + 32 * e] + unbias;
            ntt_forward<true>(x, scr, fw, p, lh);
            // products with the GGSW rows: out_h = D_h K[h][h] + D_{1-h} K[1-h][h]
            // (the key holds the pair of a lane in that order)
#pragma unroll
            for (int e = 0; e < kEh; e += 2) {
                const uint4 kq = K[(e >> 1) * 32];
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const uint32_t own = x[e + o];
                    const uint32_t other = swap_halves(own, lane);
                    x[e + o] = redc(uint64_t(own) * (o ? kq.z : kq.x) + uint64_t(other) * (o ? kq.w : kq.y), p, mont);
                }
            }
            // (4)
            ntt_inverse(x, scr, iw, p, q, lh);
#pragma unroll
            for (int e = 0; e < kEh; ++e) scr[lh + 32 * e] = x[e];
            __syncthreads();
            // (5)
#pragma unroll
            for (int k = 0; k < kAccPer; ++k) {
                const int at = (k & 1) * kPoly + tid + kBrThreads * (k >> 1);
                uint32_t r[kPrimes];
#pragma unroll
                for (int w = 0; w < kPrimes; ++w) r[w] = region[w * 2 * kPoly + at];
                acc[k] = crt_add(acc[k], r, A.crt);
            }
        }
        // sample extraction of coefficient 0, then the job's output rule
#pragma unroll
        for (int k = 0; k < kAccPer; ++k) {
            const int at = (k & 1) * kPoly + tid + kBrThreads * (k >> 1);
            acc_lo[at] = uint32_t(acc[k]);
            acc_hi[at] = uint32_t(acc[k] >> 32);
        }
        __syncthreads();
        for (int t = tid; t < kCtWords; t += kBrThreads) {
            const int at = (t == 0) ? 0 : (t < kN) ? kN - t : kPoly;
            const uint64_t m = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
            const uint64_t v = (t > 0 && t < kN) ? uint64_t(0) - m : m;
            const uint64_t s0 = J.sub[0] ? J.sub[0][t] : 0;
            const uint64_t s1 = J.sub[1] ? J.sub[1][t] : 0;
            const uint64_t c0 = (t == kN) ? J.sub_delta[0] : 0;
            const uint64_t c1 = (t == kN) ? J.sub_delta[1] : 0;
            const uint64_t o0 = v - s0 - c0, o1 = v - s1 - c1;
            if (J.dst[0]) J.dst[0][t] = o0;
            if (J.dst[1]) J.dst[1][t] = o1;
            if (J.dst[2]) J.dst[2][t] = v;
            if (J.dst[3]) J.dst[3][t] = J.copy_of ? o1 : o0;
        }
        __syncthreads();
    }
}

// ------------------------------------------- blind rotation, latency form

// One workgroup of 8 wavefronts per bootstrap, one workgroup per CU: two
// waves per prime, wave part g holding the lane's elements 32 g .. 32 g + 31
// of both polynomials, so a bootstrap has twice the waves (and half the
// dependent work per wave) of the forms above.  Of the 11 forward stages only
// the first pairs the two halves (coefficients j and j + 1024), and of the 11
// inverse stages only the last: both run where one thread holds both
// coefficients of a pair, the first in the digit phase (for all four primes,
// straight from the digits, which never reach LDS), the last in the CRT step.
// Two LDS buffers alternate, F (first-stage outputs, inverse transposes) and
// I (accumulator copy, forward transposes, residues), so that five barriers
// per CMux order every access.  Positions after the forward
// transform are those of the forms above (lane lh, element e = 32 g + e'':
// position 64 lh + e), so the bootstrapping key is shared with them.
constexpr int kLatThreads = 512;
constexpr int kLatE = kEh / 2;                   // elements per lane and wave
constexpr int kLatAcc = 2 * kN / kLatThreads;    // accumulator coefficients per thread (8)
constexpr int kLatTwu = 64;                      // uniform-stage twiddles per prime and direction
constexpr size_t kLatLds = sizeof(uint32_t) * 2 * kPrimes * 2 * kPoly       // F and I
                           + sizeof(uint32_t) * (kSmallWords + 1)            // switched mask and body
                           + sizeof(uint2) * 2 * kPrimes * kLatTwu;          // uniform-stage twiddles

// Coefficient k of thread t: polynomial (k >> 1) & 1, index t + 512 (k >> 2)
// + 1024 (k & 1), so a thread holds both members (c, c + 1024) of each pair.
__device__ __forceinline__ int lat_poly(int k) { return (k >> 1) & 1; }
__device__ __forceinline__ int lat_coef(int tid, int k) { return tid + kLatThreads * (k >> 2) + (kN / 2) * (k & 1); }

__global__ void __launch_bounds__(kLatThreads, 1) blind_rotate_latency_kernel(BrArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* F = reinterpret_cast<uint32_t*>(lds);      // [kPrimes][2][kPoly]
    uint32_t* I = F + kPrimes * 2 * kPoly;               // [kPrimes][2][kPoly]
    uint32_t* abar = I + kPrimes * 2 * kPoly;            // [n+1]
    // entries 0 .. 63 of every prime's forward and inverse tables
    uint2* twu = reinterpret_cast<uint2*>(abar + kSmallWords + 1);   // [2][kPrimes][kLatTwu]
    // the accumulator copy sits at the residue slots of primes 0 and 1 that
    // the writing thread alone reads in the CRT step
    uint32_t* acc_lo = I;                                // [2][kPoly]
    uint32_t* acc_hi = I + 2 * kPoly;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = wave >> 1;          // prime
    const int g = wave & 1;           // element half
    const int e0 = kLatE * g;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int lh = lane & 31;
    const uint32_t p = pick(A.crt.p, r);
    const uint32_t mont = pick(A.crt.mont, r);
    const uint32_t q = pick(A.crt.red, r);
    const uint64_t off2p = uint64_t(2 * p) << 32;     // offset of the inverse transform's first a elements
    const uint2* fw = A.tw.fwd + size_t(r) * kN;
    const uint2* iw = A.tw.inv + size_t(r) * kN;
    uint32_t* scrF = F + (r * 2 + h) * kPoly;
    uint32_t* scrI = I + (r * 2 + h) * kPoly;
    uint2 wfirst[kPrimes], wlast[kPrimes];   // twiddles of forward stage 0 and inverse stage 10, every prime
#pragma unroll
    for (int w = 0; w < kPrimes; ++w) {
        wfirst[w] = A.tw.fwd[size_t(w) * kN + 1];
        wlast[w] = A.tw.inv[size_t(w) * kN + 1];
    }
    for (int t = tid; t < 2 * kPrimes * kLatTwu; t += kLatThreads) {
        const int dir = t / (kPrimes * kLatTwu), pr = (t / kLatTwu) % kPrimes, idx = t % kLatTwu;
        twu[t] = (dir ? A.tw.inv : A.tw.fwd)[size_t(pr) * kN + idx];
    }
    const uint2* const twf = twu + r * kLatTwu;                       // this wave's prime, forward
    const uint2* const twi = twu + (kPrimes + r) * kLatTwu;           // and inverse

    for (int b = blockIdx.x; b < A.B; b += gridDim.x) {
        const Job& J = A.jobs[b];
        for (int c = tid; c < kSmallWords; c += kLatThreads) {
            uint64_t v = 0;
            for (int sp = 0; sp < A.nsplit; ++sp) v += A.part[(size_t(sp) * A.B + b) * kSmallWords + c];
            if (c == kSmallN) v += job_word(J, kN) + J.delta;
            abar[c] = uint32_t((((v >> 51) + 1) >> 1) & (2 * kN - 1));
        }
        __syncthreads();
        const int lut = min(int(J.lut), LVS_LUT_SLOTS - 1);
        const uint64_t* tp = A.luts + size_t(lut) * kN;
        const uint32_t bbar = abar[kSmallN];
        uint64_t acc[kLatAcc];
#pragma unroll
        for (int k = 0; k < kLatAcc; ++k) {
            const uint32_t c = uint32_t(lat_coef(tid, k));
            const uint32_t src = (c + bbar) & (2 * kN - 1);
            const uint64_t v = tp[src & (kN - 1)];
            acc[k] = lat_poly(k) ? ((src < uint32_t(kN)) ? v : uint64_t(0) - v) : uint64_t(0);
        }

        // the lane's bootstrapping-key values of a CMux: the first half is
        // issued at the end of the previous CMux's inverse transform (it
        // arrives during the CRT), the second at the top of the CMux
        const uint4* const K0 = reinterpret_cast<const uint4*>(A.bsk) + (size_t(r) * 2 + h) * (kN / 2) + lh + 16 * e0;
        constexpr size_t kKeyStep = size_t(kPrimes) * 2 * (kN / 2);   // uint4 per CMux
        constexpr int kEarly = kLatE / 4;
        uint4 kpre[kLatE / 2];
#pragma unroll
        for (int k = 0; k < kEarly; ++k) kpre[k] = K0[k * 32];

        for (int i = 0; i < kSmallN; ++i) {
            const uint32_t a = abar[i];
            {
                const uint4* K = K0 + size_t(i) * kKeyStep;
#pragma unroll
                for (int k = kEarly; k < kLatE / 2; ++k) kpre[k] = K[k * 32];
            }
            asm volatile("" ::: "memory");
            // accumulator copy (low and high words)
#pragma unroll
            for (int k = 0; k < kLatAcc; ++k) {
                const int at = lat_poly(k) * kPoly + lat_coef(tid, k);
                acc_lo[at] = uint32_t(acc[k]);
                acc_hi[at] = uint32_t(acc[k] >> 32);
            }
            __syncthreads();
            // digits of X^a ACC - ACC for a pair (c, c + 1024), then the first
            // forward stage of every prime on the pair into F
#pragma unroll
            for (int k = 0; k < kLatAcc; k += 2) {
                const int qq = lat_poly(k);
                uint32_t u[2];
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const uint32_t c = uint32_t(lat_coef(tid, k + o));
                    const uint32_t src = (c - a) & (2 * kN - 1);
                    const int at = qq * kPoly + int(src & (kN - 1));
                    uint64_t rr = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
                    if (src >= uint32_t(kN)) rr = uint64_t(0) - rr;
                    const uint64_t t = rr - acc[k + o];
                    // round(t / 2^41) as a balanced 23-bit digit d, kept as d + 2^22
                    u[o] = ((((uint32_t(t >> 40) + 1) >> 1) & 0x7FFFFFu) + 0x400000u) & 0x7FFFFFu;
                }
                const int at = qq * kPoly + lat_coef(tid, k);
#pragma unroll
                for (int w = 0; w < kPrimes; ++w) {
                    // residues of the digits below 2p: d + 2^22 + (p - 2^22)
                    const uint32_t pw = A.crt.p[w];
                    const uint32_t lo = u[0] + (pw - (1u << 22)), hi = u[1] + (pw - (1u << 22));
                    const uint32_t s = __umulhi(hi, wfirst[w].y) * pw - hi * wfirst[w].x;
                    F[w * 2 * kPoly + at] = lo - s;
                    F[w * 2 * kPoly + at + kN / 2] = lo + 2 * pw + s;
                }
            }
            __syncthreads();
            // forward transform, stages 1..10, of this wave's half
            uint32_t x[kLatE];
            const uint32_t* const nat0 = scrF + lh + 32 * e0;
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = nat0[32 * el];
            fwd_stage_lds<1, kLatE>(x, twf, p, e0);
            fwd_stage_lds<2, kLatE>(x, twf, p, e0);
            fwd_stage_lds<3, kLatE>(x, twf, p, e0);
            fwd_stage_lds<4, kLatE>(x, twf, p, e0);
            fwd_stage_lds<5, kLatE>(x, twf, p, e0);
            // twiddles of stages 6..10, in flight across the transpose
            FwdTw<6, kLatE> t6;
            FwdTw<7, kLatE> t7;
            FwdTw<8, kLatE> t8;
            FwdTw<9, kLatE> t9;
            FwdTw<10, kLatE> t10;
            load_fwd_tw(t6, fw, lh, e0);
            load_fwd_tw(t7, fw, lh, e0);
            load_fwd_tw(t8, fw, lh, e0);
            load_fwd_tw(t9, fw, lh, e0);
            load_fwd_tw(t10, fw, lh, e0);
            asm volatile("" ::: "memory");
            // pad(lh + 32 e) = lh + 32 e + (e >> 1) and pad(64 lh + e) = 65 lh + e (lh < 32, e < 64)
            uint32_t* const col = scrI + lh + 32 * e0 + (e0 >> 1);
            uint32_t* const row = scrI + 65 * lh + e0;
#pragma unroll
            for (int el = 0; el < kLatE; ++el) col[32 * el + (el >> 1)] = x[el];
            __syncthreads();
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = row[el];
            fwd_stage_tw(x, t6, p);
            fwd_stage_tw(x, t7, p);
            fwd_stage_tw(x, t8, p);
            fwd_stage_tw(x, t9, p);
            fwd_stage_tw(x, t10, p);
            // products with the GGSW rows (own digit first, as in the key)
#pragma unroll
            for (int el = 0; el < kLatE; el += 2) {
                const uint4 kq = kpre[el >> 1];
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const uint32_t own = x[el + o];
                    const uint32_t other = swap_halves(own, lane);
                    // the a elements of inverse stage 0 (even) take the plan's offset 2p
                    const uint64_t t0 = (o ? uint64_t(0) : off2p) + uint64_t(own) * (o ? kq.z : kq.x);
                    x[el + o] = redc(t0 + uint64_t(other) * (o ? kq.w : kq.y), p, mont);
                }
            }
            // twiddles of inverse stages 0..4
            InvTw<0, kLatE> u0;
            InvTw<1, kLatE> u1;
            InvTw<2, kLatE> u2;
            InvTw<3, kLatE> u3;
            InvTw<4, kLatE> u4;
            load_inv_tw(u0, iw, lh, e0);
            load_inv_tw(u1, iw, lh, e0);
            load_inv_tw(u2, iw, lh, e0);
            load_inv_tw(u3, iw, lh, e0);
            load_inv_tw(u4, iw, lh, e0);
            asm volatile("" ::: "memory");
            // inverse transform, stages 0..9
            inv_stage_tw(x, u0, p, q);
            inv_stage_tw(x, u1, p, q);
            inv_stage_tw(x, u2, p, q);
            inv_stage_tw(x, u3, p, q);
            if (g) inv_stage_tw<true>(x, u4, p, q);
            else inv_stage_tw(x, u4, p, q);
            uint32_t* const rowI = scrF + 65 * lh + e0;
            uint32_t* const colI = scrF + lh + 32 * e0 + (e0 >> 1);
#pragma unroll
            for (int el = 0; el < kLatE; ++el) rowI[el] = x[el];
            __syncthreads();
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = colI[32 * el + (el >> 1)];
            inv_stage_lds<5, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<6, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<7, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<8, kLatE>(x, twi, p, q, e0);
            if (g) inv_stage_lds<9, kLatE, true>(x, twi, p, q, e0);
            else inv_stage_lds<9, kLatE>(x, twi, p, q, e0);
            uint32_t* const nat = scrI + lh + 32 * e0;
#pragma unroll
            for (int el = 0; el < kLatE; ++el) nat[32 * el] = x[el];
            {
                // the last CMux reloads its own key (in bounds, unused)
                const uint4* K = K0 + size_t(min(i + 1, kSmallN - 1)) * kKeyStep;
#pragma unroll
                for (int k = 0; k < kEarly; ++k) kpre[k] = K[k * 32];
            }
            asm volatile("" ::: "memory");
            __syncthreads();
            // last inverse stage (coefficients c and c + 1024), then the CRT
#pragma unroll
            for (int k = 0; k < kLatAcc; k += 2) {
                const int at = lat_poly(k) * kPoly + lat_coef(tid, k);
                uint32_t rlo[kPrimes], rhi[kPrimes];
#pragma unroll
                for (int w = 0; w < kPrimes; ++w) {
                    const uint32_t pw = A.crt.p[w];
                    const uint32_t u0 = I[w * 2 * kPoly + at];
                    const uint32_t u1 = I[w * 2 * kPoly + at + kN / 2];
                    // u1 arrives negated (the plan's stage 9)
                    rlo[w] = u0 - u1;                                        // below 16 p_w
                    rhi[w] = mul_shoup(u0 + u1 + 8 * pw, wlast[w].x, wlast[w].y, pw);
                }
                acc[k] = crt_add(acc[k], rlo, A.crt);
                acc[k + 1] = crt_add(acc[k + 1], rhi, A.crt);
            }
        }
        // sample extraction of coefficient 0, then the job's output rule
#pragma unroll
        for (int k = 0; k < kLatAcc; ++k) {
            const int at = lat_poly(k) * kPoly + lat_coef(tid, k);
            acc_lo[at] = uint32_t(acc[k]);
            acc_hi[at] = uint32_t(acc[k] >> 32);
        }
        __syncthreads();
        for (int t = tid; t < kCtWords; t += kLatThreads) {
            const int at = (t == 0) ? 0 : (t < kN) ? kN - t : kPoly;
            const uint64_t m = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
            const uint64_t v = (t > 0 && t < kN) ? uint64_t(0) - m : m;
            const uint64_t s0 = J.sub[0] ? J.sub[0][t] : 0;
            const uint64_t s1 = J.sub[1] ? J.sub[1][t] : 0;
            const uint64_t c0 = (t == kN) ? J.sub_delta[0] : 0;
            const uint64_t c1 = (t == kN) ? J.sub_delta[1] : 0;
            const uint64_t o0 = v - s0 - c0, o1 = v - s1 - c1;
            if (J.dst[0]) J.dst[0][t] = o0;
            if (J.dst[1]) J.dst[1][t] = o1;
            if (J.dst[2]) J.dst[2][t] = v;
            if (J.dst[3]) J.dst[3][t] = J.copy_of ? o1 : o0;
        }
        __syncthreads();
    }
}

// -------------------------------- blind rotation, two eight-wave groups per CU

// The eight-wave form with one LDS buffer instead of two, so that two
// workgroups (two bootstraps) share a CU: 16 waves per CU, 4 per SIMD, and
// one bootstrap's barrier and LDS waits are filled by the other's
// arithmetic.  Registers are held to 128 per thread (no key or twiddle
// prefetch across phases); every coefficient lives at its padded LDS
// position, so that each wave's transposes write exactly the words it has
// just read and one buffer serves every phase.  Six barriers per CMux:
// accumulator copy -> digits; digits read -> first stage written (the
// copy and the first-stage outputs share the buffer); first stage ->
// transform; the forward transpose; the inverse transpose; inverse outputs
// -> CRT.  Transform positions, key layout and results are those of the
// eight-wave form.
constexpr size_t kPairLds = sizeof(uint32_t) * kPrimes * 2 * kPoly              // X
                            + sizeof(uint32_t) * (kSmallWords + 1)              // switched mask and body
                            + sizeof(uint2) * 2 * kPrimes * kLatTwu;            // uniform-stage twiddles

__global__ void __launch_bounds__(kLatThreads, 4) blind_rotate_pair_kernel(BrArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* X = reinterpret_cast<uint32_t*>(lds);      // [kPrimes][2][kPoly], padded positions
    uint32_t* abar = X + kPrimes * 2 * kPoly;            // [n+1]
    uint2* twu = reinterpret_cast<uint2*>(abar + kSmallWords + 1);   // [2][kPrimes][kLatTwu]
    // the accumulator copy: low words in prime 0's regions, high words in
    // prime 1's, at the padded positions of the writing thread's coefficients
    uint32_t* acc_lo = X;
    uint32_t* acc_hi = X + 2 * kPoly;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = wave >> 1;          // prime
    const int g = wave & 1;           // element half
    const int e0 = kLatE * g;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int lh = lane & 31;
    const uint32_t p = pick(A.crt.p, r);
    const uint32_t mont = pick(A.crt.mont, r);
    const uint32_t q = pick(A.crt.red, r);
    const uint64_t off2p = uint64_t(2 * p) << 32;     // offset of the inverse transform's first a elements
    const uint2* fw = A.tw.fwd + size_t(r) * kN;
    const uint2* iw = A.tw.inv + size_t(r) * kN;
    uint32_t* const scr = X + (r * 2 + h) * kPoly;
    uint2 wfirst[kPrimes], wlast[kPrimes];
#pragma unroll
    for (int w = 0; w < kPrimes; ++w) {
        wfirst[w] = A.tw.fwd[size_t(w) * kN + 1];
        wlast[w] = A.tw.inv[size_t(w) * kN + 1];
    }
    for (int t = tid; t < 2 * kPrimes * kLatTwu; t += kLatThreads) {
        const int dir = t / (kPrimes * kLatTwu), pr = (t / kLatTwu) % kPrimes, idx = t % kLatTwu;
        twu[t] = (dir ? A.tw.inv : A.tw.fwd)[size_t(pr) * kN + idx];
    }
    const uint2* const twf = twu + r * kLatTwu;
    const uint2* const twi = twu + (kPrimes + r) * kLatTwu;
    // element el of the wave's half at pad(lh + 32 (e0 + el)) = lh + 32 e0 + e0 / 2 + 32 el + el / 2
    // (coefficient order) and at pad(64 lh + e0 + el) = 65 lh + e0 + el (transform order)
    uint32_t* const col = scr + lh + 32 * e0 + (e0 >> 1);
    uint32_t* const row = scr + 65 * lh + e0;

    for (int b = blockIdx.x; b < A.B; b += gridDim.x) {
        const Job& J = A.jobs[b];
        for (int c = tid; c < kSmallWords; c += kLatThreads) {
            uint64_t v = 0;
            for (int sp = 0; sp < A.nsplit; ++sp) v += A.part[(size_t(sp) * A.B + b) * kSmallWords + c];
            if (c == kSmallN) v += job_word(J, kN) + J.delta;
            abar[c] = uint32_t((((v >> 51) + 1) >> 1) & (2 * kN - 1));
        }
        __syncthreads();
        const int lut = min(int(J.lut), LVS_LUT_SLOTS - 1);
        const uint64_t* tp = A.luts + size_t(lut) * kN;
        const uint32_t bbar = abar[kSmallN];
        uint64_t acc[kLatAcc];
#pragma unroll
        for (int k = 0; k < kLatAcc; ++k) {
            const uint32_t c = uint32_t(lat_coef(tid, k));
            const uint32_t src = (c + bbar) & (2 * kN - 1);
            const uint64_t v = tp[src & (kN - 1)];
            acc[k] = lat_poly(k) ? ((src < uint32_t(kN)) ? v : uint64_t(0) - v) : uint64_t(0);
        }
        const uint4* const K0 = reinterpret_cast<const uint4*>(A.bsk) + (size_t(r) * 2 + h) * (kN / 2) + lh + 16 * e0;
        constexpr size_t kKeyStep = size_t(kPrimes) * 2 * (kN / 2);   // uint4 per CMux

        for (int i = 0; i < kSmallN; ++i) {
            const uint32_t a = abar[i];
#pragma unroll
            for (int k = 0; k < kLatAcc; ++k) {
                const int at = lat_poly(k) * kPoly + int(pad(uint32_t(lat_coef(tid, k))));
                acc_lo[at] = uint32_t(acc[k]);
                acc_hi[at] = uint32_t(acc[k] >> 32);
            }
            __syncthreads();
            // digits of X^a ACC - ACC, d + 2^22 for the balanced 23-bit digit d
            uint32_t u[kLatAcc];
#pragma unroll
            for (int k = 0; k < kLatAcc; ++k) {
                const uint32_t c = uint32_t(lat_coef(tid, k));
                const uint32_t src = (c - a) & (2 * kN - 1);
                const int at = lat_poly(k) * kPoly + int(pad(src & (kN - 1)));
                uint64_t rr = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
                if (src >= uint32_t(kN)) rr = uint64_t(0) - rr;
                const uint64_t t = rr - acc[k];
                u[k] = ((((uint32_t(t >> 40) + 1) >> 1) & 0x7FFFFFu) + 0x400000u) & 0x7FFFFFu;
            }
            __syncthreads();
            // the first forward stage of every prime on the pairs (c, c + 1024)
#pragma unroll
            for (int k = 0; k < kLatAcc; k += 2) {
                const int at = lat_poly(k) * kPoly + int(pad(uint32_t(lat_coef(tid, k))));
#pragma unroll
                for (int w = 0; w < kPrimes; ++w) {
                    const uint32_t pw = A.crt.p[w];
                    const uint32_t lo = u[k] + (pw - (1u << 22)), hi = u[k + 1] + (pw - (1u << 22));
                    const uint32_t s = __umulhi(hi, wfirst[w].y) * pw - hi * wfirst[w].x;
                    X[w * 2 * kPoly + at] = lo - s;
                    X[w * 2 * kPoly + at + kN / 2 + kN / 128] = lo + 2 * pw + s;   // pad(c + 1024)
                }
            }
            __syncthreads();
            uint32_t x[kLatE];
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = col[32 * el + (el >> 1)];
            fwd_stage_lds<1, kLatE>(x, twf, p, e0);
            fwd_stage_lds<2, kLatE>(x, twf, p, e0);
            fwd_stage_lds<3, kLatE>(x, twf, p, e0);
            fwd_stage_lds<4, kLatE>(x, twf, p, e0);
            fwd_stage_lds<5, kLatE>(x, twf, p, e0);
            // transpose through the words this wave has just read
#pragma unroll
            for (int el = 0; el < kLatE; ++el) col[32 * el + (el >> 1)] = x[el];
            __syncthreads();
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = row[el];
            asm volatile("" ::: "memory");   // keep each stage's twiddle loads in its stage
            {
                FwdTw<6, kLatE> t6;
                load_fwd_tw(t6, fw, lh, e0);
                fwd_stage_tw(x, t6, p);
            }
            asm volatile("" ::: "memory");   // keep each stage's twiddle loads in its stage
            {
                FwdTw<7, kLatE> t7;
                load_fwd_tw(t7, fw, lh, e0);
                fwd_stage_tw(x, t7, p);
            }
            asm volatile("" ::: "memory");   // keep each stage's twiddle loads in its stage
            {
                FwdTw<8, kLatE> t8;
                load_fwd_tw(t8, fw, lh, e0);
                fwd_stage_tw(x, t8, p);
            }
            asm volatile("" ::: "memory");   // keep each stage's twiddle loads in its stage
            {
                FwdTw<9, kLatE> t9;
                load_fwd_tw(t9, fw, lh, e0);
                fwd_stage_tw(x, t9, p);
            }
            asm volatile("" ::: "memory");   // keep each stage's twiddle loads in its stage
            {
                FwdTw<10, kLatE> t10;
                load_fwd_tw(t10, fw, lh, e0);
                fwd_stage_tw(x, t10, p);
            }
            // products with the GGSW rows (own digit first, as in the key), the
            // key loaded in four parts of 16 registers
            {
                const uint4* K = K0 + size_t(i) * kKeyStep;
#pragma unroll
                for (int part = 0; part < 4; ++part) {
                    asm volatile("" ::: "memory");
                    uint4 kq[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) kq[j] = K[(part * 4 + j) * 32];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int el = (part * 4 + j) * 2;
#pragma unroll
                        for (int o = 0; o < 2; ++o) {
                            const uint32_t own = x[el + o];
                            const uint32_t other = swap_halves(own, lane);
                            // the a elements of inverse stage 0 (even) take the plan's offset 2p
                            const uint64_t t0 = (o ? uint64_t(0) : off2p) + uint64_t(own) * (o ? kq[j].z : kq[j].x);
                            x[el + o] = redc(t0 + uint64_t(other) * (o ? kq[j].w : kq[j].y), p, mont);
                        }
                    }
                }
            }
            asm volatile("" ::: "memory");
            {
                InvTw<0, kLatE> u0;
                load_inv_tw(u0, iw, lh, e0);
                inv_stage_tw(x, u0, p, q);
            }
            asm volatile("" ::: "memory");
            {
                InvTw<1, kLatE> u1;
                load_inv_tw(u1, iw, lh, e0);
                inv_stage_tw(x, u1, p, q);
            }
            asm volatile("" ::: "memory");
            {
                InvTw<2, kLatE> u2;
                load_inv_tw(u2, iw, lh, e0);
                inv_stage_tw(x, u2, p, q);
            }
            asm volatile("" ::: "memory");
            {
                InvTw<3, kLatE> u3;
                load_inv_tw(u3, iw, lh, e0);
                inv_stage_tw(x, u3, p, q);
            }
            asm volatile("" ::: "memory");
            {
                InvTw<4, kLatE> u4;
                load_inv_tw(u4, iw, lh, e0);
                if (g) inv_stage_tw<true>(x, u4, p, q);
            else inv_stage_tw(x, u4, p, q);
            }
            // inverse transpose through the words this wave read after the forward one
#pragma unroll
            for (int el = 0; el < kLatE; ++el) row[el] = x[el];
            __syncthreads();
#pragma unroll
            for (int el = 0; el < kLatE; ++el) x[el] = col[32 * el + (el >> 1)];
            inv_stage_lds<5, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<6, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<7, kLatE>(x, twi, p, q, e0);
            inv_stage_lds<8, kLatE>(x, twi, p, q, e0);
            if (g) inv_stage_lds<9, kLatE, true>(x, twi, p, q, e0);
            else inv_stage_lds<9, kLatE>(x, twi, p, q, e0);
#pragma unroll
            for (int el = 0; el < kLatE; ++el) col[32 * el + (el >> 1)] = x[el];
            __syncthreads();
            // last inverse stage (coefficients c and c + 1024), then the CRT
#pragma unroll
            for (int k = 0; k < kLatAcc; k += 2) {
                const int at = lat_poly(k) * kPoly + int(pad(uint32_t(lat_coef(tid, k))));
                uint32_t rlo[kPrimes], rhi[kPrimes];
#pragma unroll
                for (int w = 0; w < kPrimes; ++w) {
                    const uint32_t pw = A.crt.p[w];
                    const uint32_t v0 = X[w * 2 * kPoly + at];
                    const uint32_t v1 = X[w * 2 * kPoly + at + kN / 2 + kN / 128];
                    // v1 arrives negated (the plan's stage 9)
                    rlo[w] = v0 - v1;                                        // below 16 p_w
                    rhi[w] = mul_shoup(v0 + v1 + 8 * pw, wlast[w].x, wlast[w].y, pw);
                }
                acc[k] = crt_add(acc[k], rlo, A.crt);
                acc[k + 1] = crt_add(acc[k + 1], rhi, A.crt);
            }
        }
        // sample extraction of coefficient 0, then the job's output rule (the
        // copy overwrites only words its own thread read in the CRT step)
#pragma unroll
        for (int k = 0; k < kLatAcc; ++k) {
            const int at = lat_poly(k) * kPoly + int(pad(uint32_t(lat_coef(tid, k))));
            acc_lo[at] = uint32_t(acc[k]);
            acc_hi[at] = uint32_t(acc[k] >> 32);
        }
        __syncthreads();
        for (int t = tid; t < kCtWords; t += kLatThreads) {
            const uint32_t c = (t == 0) ? 0u : (t < kN) ? uint32_t(kN - t) : 0u;
            const int at = (t == kN) ? kPoly + int(pad(0)) : int(pad(c));
            const uint64_t m = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
            const uint64_t v = (t > 0 && t < kN) ? uint64_t(0) - m : m;
            const uint64_t s0 = J.sub[0] ? J.sub[0][t] : 0;
            const uint64_t s1 = J.sub[1] ? J.sub[1][t] : 0;
            const uint64_t c0 = (t == kN) ? J.sub_delta[0] : 0;
            const uint64_t c1 = (t == kN) ? J.sub_delta[1] : 0;
            const uint64_t o0 = v - s0 - c0, o1 = v - s1 - c1;
            if (J.dst[0]) J.dst[0][t] = o0;
            if (J.dst[1]) J.dst[1][t] = o1;
            if (J.dst[2]) J.dst[2][t] = v;
            if (J.dst[3]) J.dst[3][t] = J.copy_of ? o1 : o0;
        }
        __syncthreads();
    }
}

// ------------------------------------------ blind rotation, sixteen-wave form

// One workgroup of 16 wavefronts per bootstrap (four per prime), one per CU,
// four waves per SIMD.  With position bits b10..b0 of a polynomial:
//  * the digit phase runs the first three forward stages (b10, b9, b8): a
//    pair of threads holds the eight positions c + 256 k (k = b10 b9 b8) of
//    a group, each thread the digits' residues for two primes;
//  * wave (prime r, quarter q = b10 b9) then holds, in element e of lane
//    (h, l), position q 512 + (l >> 4) 256 + 16 e + (l & 15) and runs the
//    stages of b7..b4 in the lane; a transpose local to the wave gives lane
//    l the positions q 512 + 16 l + e' for the stages of b3..b0 and for the
//    products, which are the key's order (position 64 lh + e with lh = 8 q +
//    (l >> 2), e = 16 (l & 3) + e');
//  * the inverse runs the same phases backwards and ends in the CRT step with
//    the last three stages; the two threads of a group exchange residues by
//    a lane permutation.
// Three workgroup barriers per CMux: accumulator copy -> digits, digits ->
// transform, transform -> CRT.
constexpr int kW16Threads = 1024;
constexpr int kW16E = 16;                                  // elements per lane and phase
constexpr int kW16Stride = kN + kN / 16 + 16;              // padded polynomial in LDS, 16 mod 32 words
constexpr int kW16Acc = kN + 32;                           // words of one padded accumulator polynomial
constexpr int kW16Twu = 128;                               // LDS twiddle entries per prime and direction
constexpr size_t kW16Lds = sizeof(uint32_t) * kPrimes * 2 * kW16Stride      // residues
                           + sizeof(uint32_t) * 2 * 2 * kW16Acc              // accumulator copy (lo, hi)
                           + sizeof(uint32_t) * (kSmallWords + 1)            // switched mask and body
                           + sizeof(uint2) * 2 * kPrimes * kW16Twu;          // twiddles 0..127
__device__ __forceinline__ int w16pad(int pos) { return pos + (pos >> 4); }
__device__ __forceinline__ int w16apad(int pos) { return pos + ((pos >> 10) << 4); }

// pick ? a : b for a per-lane pick, as arithmetic (no indexed array access)
__device__ __forceinline__ uint32_t sel(uint32_t pick_mask, uint32_t a, uint32_t b) {
    return (a & pick_mask) | (b & ~pick_mask);
}

// Value of v in lane ^ 1 (the other thread of a group).
__device__ __forceinline__ uint32_t lane_xor1(uint32_t v) {
    return uint32_t(__builtin_amdgcn_mov_dpp(int(v), 0xB1, 0xF, 0xF, false));   // quad_perm [1, 0, 3, 2]
}

__device__ __forceinline__ void fwd_bfly(uint32_t& a, uint32_t& b, uint2 tw, uint32_t p) {
    const uint32_t s = __umulhi(b, tw.y) * p - b * tw.x;
    const uint32_t x = a;
    a = x - s;
    b = x + 2 * p + s;
}

__device__ __forceinline__ void inv_bfly(uint32_t& a, uint32_t& b, uint2 tw, uint32_t p, uint32_t bound, bool reduce,
                                         uint32_t q) {
    const uint32_t x = a, y = b;
    const uint32_t sum = x + y;
    a = reduce ? reduce2p(sum, q, p) : sum;
    b = mul_shoup(x + bound - y, tw.x, tw.y, p);
}

__global__ void __launch_bounds__(kW16Threads, 1) blind_rotate_w16_kernel(BrArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* F = reinterpret_cast<uint32_t*>(lds);                  // [kPrimes][2][kW16Stride]
    uint32_t* acc_lo = F + kPrimes * 2 * kW16Stride;                 // [2][kW16Acc]
    uint32_t* acc_hi = acc_lo + 2 * kW16Acc;
    uint32_t* abar = acc_hi + 2 * kW16Acc;                           // [n+1]
    uint2* twl = reinterpret_cast<uint2*>(abar + kSmallWords + 1);   // [2][kPrimes][kW16Twu]

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = wave >> 2;          // prime of the transform phases
    const int q = wave & 3;           // position bits b10 b9 of the wave
    const int lane = tid & 63;
    const int h = lane >> 5;          // polynomial of the lane
    const int l = lane & 31;
    const int b8 = l >> 4;
    // digit and CRT phases: group (polynomial gh, c = gc), primes 2 pp and 2 pp + 1
    const int grp = tid >> 1, pp = tid & 1;
    const int gh = grp >> 8, gc = grp & 255;
    const uint32_t ppm = 0u - uint32_t(pp);     // all ones for the second thread of a group

    const uint32_t p = pick(A.crt.p, r);
    const uint32_t mont = pick(A.crt.mont, r);
    const uint32_t qr = pick(A.crt.red, r);
    const uint2* fw = A.tw.fwd + size_t(r) * kN;
    const uint2* iw = A.tw.inv + size_t(r) * kN;
    uint32_t* Fr = F + (r * 2 + h) * kW16Stride;
    const uint2* twf = twl + r * kW16Twu;
    const uint2* twi = twl + (kPrimes + r) * kW16Twu;
    for (int t = tid; t < 2 * kPrimes * kW16Twu; t += kW16Threads) {
        const int dir = t / (kPrimes * kW16Twu), pr = (t / kW16Twu) % kPrimes, idx = t % kW16Twu;
        twl[t] = (dir ? A.tw.inv : A.tw.fwd)[size_t(pr) * kN + idx];
    }
    // this thread's primes in the digit and CRT phases
    uint32_t pj[2], qj[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        pj[j] = pp ? A.crt.p[2 + j] : A.crt.p[j];
        qj[j] = pp ? A.crt.red[2 + j] : A.crt.red[j];
    }
    // B1: element e at position base1 + 16 e; B2: element e' at base2 + e'
    const int base1 = (q << 9) | (b8 << 8) | (l & 15);
    const int base2 = (q << 9) | (l << 4);
    uint32_t* const row1 = Fr + w16pad(base1);      // element e at row1[17 e]
    uint32_t* const row2 = Fr + w16pad(base2);      // element e' at row2[e']
    const int ql = (q << 5) | l;                    // position bits b10..b4 in the B2 layout
    const int qb = (q << 1) | b8;                   // position bits b10..b8 in the B1 layout

    for (int b = blockIdx.x; b < A.B; b += gridDim.x) {
        const Job& J = A.jobs[b];
        for (int c = tid; c < kSmallWords; c += kW16Threads) {
            uint64_t v = 0;
            for (int sp = 0; sp < A.nsplit; ++sp) v += A.part[(size_t(sp) * A.B + b) * kSmallWords + c];
            if (c == kSmallN) v += job_word(J, kN) + J.delta;
            abar[c] = uint32_t((((v >> 51) + 1) >> 1) & (2 * kN - 1));
        }
        __syncthreads();
        const int lut = min(int(J.lut), LVS_LUT_SLOTS - 1);
        const uint64_t* tp = A.luts + size_t(lut) * kN;
        const uint32_t bbar = abar[kSmallN];
        // the thread's accumulator coefficients: polynomial gh, positions gc + 256 (k + 4 pp)
        uint64_t acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t c = uint32_t(gc + 256 * (k + 4 * pp));
            const uint32_t src = (c + bbar) & (2 * kN - 1);
            const uint64_t v = tp[src & (kN - 1)];
            acc[k] = gh ? ((src < uint32_t(kN)) ? v : uint64_t(0) - v) : uint64_t(0);
        }

        for (int i = 0; i < kSmallN; ++i) {
            // the loop-invariant twiddle reads stay in the loop (registers are the limit here)
            asm volatile("" ::: "memory");
            const uint32_t a = abar[i];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int at = gh * kW16Acc + w16apad(gc + 256 * (k + 4 * pp));
                acc_lo[at] = uint32_t(acc[k]);
                acc_hi[at] = uint32_t(acc[k] >> 32);
            }
            __syncthreads();
            // digits of X^a ACC - ACC at the thread's four positions, then the
            // partner's four by a lane permutation
            uint32_t mine[4], d[8];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t c = uint32_t(gc + 256 * (k + 4 * pp));
                const uint32_t src = (c - a) & (2 * kN - 1);
                const int at = gh * kW16Acc + w16apad(int(src & (kN - 1)));
                uint64_t rr = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
                if (src >= uint32_t(kN)) rr = uint64_t(0) - rr;
                const uint64_t t = rr - acc[k];
                // round(t / 2^41) as a balanced 23-bit digit d, kept as d + 2^22
                mine[k] = ((((uint32_t(t >> 40) + 1) >> 1) & 0x7FFFFFu) + 0x400000u) & 0x7FFFFFu;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t other = lane_xor1(mine[k]);
                d[k] = sel(ppm, other, mine[k]);
                d[k + 4] = sel(ppm, mine[k], other);
            }
            // forward stages 0..2 (b10, b9, b8) of the thread's two primes
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t pw = pj[j];
                const uint2* tw = twl + (2 * pp + j) * kW16Twu;
                uint32_t y[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) y[k] = d[k] + (pw - (1u << 22));   // residue of d below 2p
                const uint2 t0 = tw[1];
#pragma unroll
                for (int k = 0; k < 4; ++k) fwd_bfly(y[k], y[k + 4], t0, pw);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (!(k & 2)) fwd_bfly(y[k], y[k + 2], tw[2 + (k >> 2)], pw);
#pragma unroll
                for (int k = 0; k < 8; k += 2) fwd_bfly(y[k], y[k + 1], tw[4 + (k >> 1)], pw);
                uint32_t* dst = F + ((2 * pp + j) * 2 + gh) * kW16Stride;
#pragma unroll
                for (int k = 0; k < 8; ++k) dst[w16pad(gc + 256 * k)] = y[k];
            }
            __syncthreads();
            // stages 3..6 (b7..b4): partners e and e + (8 >> (s - 3))
            uint32_t x[kW16E];
#pragma unroll
            for (int e = 0; e < kW16E; ++e) x[e] = row1[17 * e];
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 8)) fwd_bfly(x[e], x[e + 8], twf[8 + qb], p);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 4)) fwd_bfly(x[e], x[e + 4], twf[16 + (qb << 1) + (e >> 3)], p);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 2)) fwd_bfly(x[e], x[e + 2], twf[32 + (qb << 2) + (e >> 2)], p);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 1)) fwd_bfly(x[e], x[e + 1], twf[64 + (qb << 3) + (e >> 1)], p);
            // this CMux's key values of the lane (positions base2 + e', e' = 2 k, 2 k + 1)
            const uint4* K = reinterpret_cast<const uint4*>(A.bsk) + ((size_t(i) * kPrimes + r) * 2 + h) * (kN / 2) +
                             ((l & 3) << 3) * 32 + (q << 3) + (l >> 2);
            uint4 kpre[kW16E / 2];
#pragma unroll
            for (int k = 0; k < kW16E / 2; ++k) kpre[k] = K[k * 32];
            // transpose within the wave
#pragma unroll
            for (int e = 0; e < kW16E; ++e) row1[17 * e] = x[e];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int e = 0; e < kW16E; ++e) x[e] = row2[e];
            __builtin_amdgcn_wave_barrier();
            // stages 7..10 (b3..b0): partners e' and e' + (8 >> (s - 7))
            {
                const uint2 t7 = fw[128 + ql];
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 8)) fwd_bfly(x[e], x[e + 8], t7, p);
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 4)) fwd_bfly(x[e], x[e + 4], fw[256 + (ql << 1) + (e >> 3)], p);
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 2)) fwd_bfly(x[e], x[e + 2], fw[512 + (ql << 2) + (e >> 2)], p);
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 1)) fwd_bfly(x[e], x[e + 1], fw[1024 + (ql << 3) + (e >> 1)], p);
            }
            // products with the GGSW rows (own digit first, as in the key)
#pragma unroll
            for (int e = 0; e < kW16E; e += 2) {
                const uint4 kq = kpre[e >> 1];
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const uint32_t own = x[e + o];
                    const uint32_t other = swap_halves(own, lane);
                    x[e + o] = redc(uint64_t(own) * (o ? kq.z : kq.x) + uint64_t(other) * (o ? kq.w : kq.y), p, mont);
                }
            }
            // inverse stages 0..3 (b0..b3): partners e' and e' + (1 << u); reduce after 3
            {
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 1)) inv_bfly(x[e], x[e + 1], iw[1024 + (ql << 3) + (e >> 1)], p, 2 * p, false, qr);
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 2)) inv_bfly(x[e], x[e + 2], iw[512 + (ql << 2) + (e >> 2)], p, 4 * p, false, qr);
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 4)) inv_bfly(x[e], x[e + 4], iw[256 + (ql << 1) + (e >> 3)], p, 8 * p, false, qr);
                const uint2 u3 = iw[128 + ql];
#pragma unroll
                for (int e = 0; e < kW16E; ++e)
                    if (!(e & 8)) inv_bfly(x[e], x[e + 8], u3, p, 16 * p, true, qr);
            }
            // transpose back within the wave
#pragma unroll
            for (int e = 0; e < kW16E; ++e) row2[e] = x[e];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int e = 0; e < kW16E; ++e) x[e] = row1[17 * e];
            __builtin_amdgcn_wave_barrier();
            // inverse stages 4..7 (b4..b7): partners e and e + (1 << (u - 4)); reduce after 7
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 1)) inv_bfly(x[e], x[e + 1], twi[64 + (qb << 3) + (e >> 1)], p, 2 * p, false, qr);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 2)) inv_bfly(x[e], x[e + 2], twi[32 + (qb << 2) + (e >> 2)], p, 4 * p, false, qr);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 4)) inv_bfly(x[e], x[e + 4], twi[16 + (qb << 1) + (e >> 3)], p, 8 * p, false, qr);
#pragma unroll
            for (int e = 0; e < kW16E; ++e)
                if (!(e & 8)) inv_bfly(x[e], x[e + 8], twi[8 + qb], p, 16 * p, true, qr);
#pragma unroll
            for (int e = 0; e < kW16E; ++e) row1[17 * e] = x[e];
            __syncthreads();
            // inverse stages 8..10 (b8, b9, b10) of the thread's two primes, then
            // the four primes of four positions by a lane permutation, then the CRT
            uint32_t y[2][8];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t pw = pj[j];
                const uint2* tw = twl + (kPrimes + 2 * pp + j) * kW16Twu;
                const uint32_t* src = F + ((2 * pp + j) * 2 + gh) * kW16Stride;
#pragma unroll
                for (int k = 0; k < 8; ++k) y[j][k] = src[w16pad(gc + 256 * k)];
#pragma unroll
                for (int k = 0; k < 8; k += 2) inv_bfly(y[j][k], y[j][k + 1], tw[4 + (k >> 1)], pw, 2 * pw, false, qj[j]);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (!(k & 2)) inv_bfly(y[j][k], y[j][k + 2], tw[2 + (k >> 2)], pw, 4 * pw, false, qj[j]);
                const uint2 t1 = tw[1];
#pragma unroll
                for (int k = 0; k < 4; ++k) inv_bfly(y[j][k], y[j][k + 4], t1, pw, 8 * pw, false, qj[j]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                uint32_t recv[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) recv[j] = lane_xor1(sel(ppm, y[j][k], y[j][k + 4]));
                uint32_t res[kPrimes];
                res[0] = sel(ppm, recv[0], y[0][k]);
                res[1] = sel(ppm, recv[1], y[1][k]);
                res[2] = sel(ppm, y[0][k + 4], recv[0]);
                res[3] = sel(ppm, y[1][k + 4], recv[1]);
                acc[k] = crt_add(acc[k], res, A.crt);
            }
        }
        // sample extraction of coefficient 0, then the job's output rule
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int at = gh * kW16Acc + w16apad(gc + 256 * (k + 4 * pp));
            acc_lo[at] = uint32_t(acc[k]);
            acc_hi[at] = uint32_t(acc[k] >> 32);
        }
        __syncthreads();
        for (int t = tid; t < kCtWords; t += kW16Threads) {
            const int at = (t == 0) ? 0 : (t < kN) ? w16apad(kN - t) : kW16Acc;
            const uint64_t m = uint64_t(acc_lo[at]) | (uint64_t(acc_hi[at]) << 32);
            const uint64_t v = (t > 0 && t < kN) ? uint64_t(0) - m : m;
            const uint64_t s0 = J.sub[0] ? J.sub[0][t] : 0;
            const uint64_t s1 = J.sub[1] ? J.sub[1][t] : 0;
            const uint64_t c0 = (t == kN) ? J.sub_delta[0] : 0;
            const uint64_t c1 = (t == kN) ? J.sub_delta[1] : 0;
            const uint64_t o0 = v - s0 - c0, o1 = v - s1 - c1;
            if (J.dst[0]) J.dst[0][t] = o0;
            if (J.dst[1]) J.dst[1][t] = o1;
            if (J.dst[2]) J.dst[2][t] = v;
            if (J.dst[3]) J.dst[3][t] = J.copy_of ? o1 : o0;
        }
        __syncthreads();
    }
}

// ------------------------------------------------ bootstrapping-key conversion

// One wavefront per (GGSW row, prime): lanes 0-31 take the row's mask
// polynomial, lanes 32-63 its body polynomial; signed lift of the 64-bit
// coefficients, reduction mod p, forward NTT, scaling by (1/N) 2^32 mod p,
// and store in the order the blind rotation reads ([i][prime][row][h][e][lh]).
__global__ void __launch_bounds__(64) bsk_convert_kernel(const uint64_t* __restrict__ bsk, uint32_t* __restrict__ out,
                                                        Tw tw, CrtConsts C, const uint32_t* scale,
                                                        const uint32_t* scale_s) {
    // output order [i][prime][h][e / 2][lh][e % 2][rho ^ h]: one 16-byte load
    // gives both rows' values of two neighbouring positions, for lanes of the
    // body polynomial (h = 1) with the rows swapped, so that every lane
    // multiplies its own transformed digit by the first value of a pair
    // (D_h K[h][h]) and the other lane's by the second (D_{1-h} K[1-h][h])
    __shared__ uint32_t scratch[2 * kPoly];
    const int lane = threadIdx.x;
    const int h = lane >> 5, lh = lane & 31;
    const int row = blockIdx.x;             // i * 2 + rho
    const int r = blockIdx.y;               // prime
    const uint32_t p = pick(C.p, r);
    const uint64_t two64_mod_p = ((~uint64_t(0)) % p + 1) % p;
    uint32_t x[kEh];
#pragma unroll
    for (int e = 0; e < kEh; ++e) {
        const uint64_t c = bsk[(size_t(row) * 2 + h) * kN + lh + 32 * e];
        uint64_t m = c % p;
        if (c >> 63) m = (m + p - two64_mod_p) % p;     // c read as c - 2^64
        x[e] = uint32_t(m);
    }
    ntt_forward<false>(x, scratch + h * kPoly, tw.fwd + size_t(r) * kN, p, lh);
    const uint32_t sc = scale[r], scs = scale_s[r];
    const int i = row >> 1, rho = row & 1;
    uint32_t* dst = out + ((size_t(i) * kPrimes + r) * 2 + h) * (2 * kN) + lh * 4 + (rho ^ h);
#pragma unroll
    for (int e = 0; e < kEh; ++e) dst[(e >> 1) * 128 + (e & 1) * 2] = csub(mul_shoup(x[e], sc, scs, p), p);
}

// ----------------------------------------------------- linear operations

constexpr int kWordBlocks = (kCtWords + 255) / 256;   // 256-word slices of a ciphertext

// Noise-free encryptions of mu in rows [0, count).
__global__ void __launch_bounds__(256) trivial_kernel(uint64_t* out, uint32_t mu) {
    const int r = blockIdx.x / kWordBlocks;
    const int w = (blockIdx.x % kWordBlocks) * 256 + threadIdx.x;
    if (w >= kCtWords) return;
    out[size_t(r) * kCtWords + w] = (w == kN) ? (uint64_t(mu) << kDeltaLog) : 0;
}

// ---------------------------------------------------------- microbenchmarks

constexpr int kProbeChains = 16;

// The forward butterfly's instruction sequence on kProbeChains independent
// register pairs (the values wrap; only the instruction mix matters).
__global__ void __launch_bounds__(256) modmul_probe_kernel(uint32_t* out, uint32_t w, uint32_t ws, uint32_t p,
                                                           int iters) {
    const uint32_t g = blockIdx.x * 256 + threadIdx.x;
    uint32_t x[kProbeChains], y[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
        x[k] = g * 2654435761u + k;
        y[k] = g ^ (k * 40503u);
    }
    const uint32_t two_p = 2 * p;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) {
            const uint32_t s = __umulhi(y[k], ws) * p - y[k] * w;
            const uint32_t a = x[k];
            x[k] = a - s;
            y[k] = a + two_p + s;
        }
    }
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) c ^= x[k] + y[k];
    out[g] = c;
}

__global__ void __launch_bounds__(256) copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         size_t n) {
    for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) dst[i] = src[i];
}

// out[item][g] = sum of in[item][k] for k in [g * group, min(cnt, (g + 1) * group)),
// ciphertext by ciphertext (the merging sums of the wide-symbol equality).
__global__ void __launch_bounds__(256) group_sum_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                        size_t items, int cnt, int groups, int group) {
    const size_t total = items * size_t(groups) * kCtWords;
    for (size_t e = blockIdx.x * size_t(256) + threadIdx.x; e < total; e += size_t(gridDim.x) * 256) {
        const size_t w = e % kCtWords;
        const size_t ig = e / kCtWords;
        const size_t item = ig / size_t(groups);
        const int g = int(ig % size_t(groups));
        const int k0 = g * group, k1 = min(cnt, k0 + group);
        const uint64_t* src = in + (item * size_t(cnt) + size_t(k0)) * kCtWords + w;
        uint64_t acc = 0;
        for (int k = k0; k < k1; ++k, src += kCtWords) acc += *src;
        out[e] = acc;
    }
}

}  // namespace dev

// ------------------------------------------------------------- launchers

hipError_t launch_modmul_probe(uint32_t* out, int blocks, int iters, hipStream_t st) {
    const PrimeTables& T = prime_tables();
    const uint32_t p = T.p[0], w = T.fwd[5];
    const uint32_t ws = T.fwd_shoup[5];
    hipLaunchKernelGGL(dev::modmul_probe_kernel, dim3(blocks), dim3(256), 0, st, out, w, ws, p, iters);
    return hipGetLastError();
}

int modmul_probe_muls_per_thread_iter() { return 3 * dev::kProbeChains; }

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int cus, hipStream_t st) {
    const size_t n = bytes / 16;
    if (!n) return hipSuccess;
    const int blocks = int(std::min<size_t>((n + 255) / 256, size_t(cus) * 16));
    hipLaunchKernelGGL(dev::copy_probe_kernel, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const uint4*>(src),
                       reinterpret_cast<uint4*>(dst), n);
    return hipGetLastError();
}

namespace {
dev::CrtConsts make_crt() {
    const PrimeTables& T = prime_tables();
    dev::CrtConsts C{};
    for (int i = 0; i < kPrimes; ++i) {
        C.p[i] = T.p[i];
        C.mont[i] = T.mont_neg_inv[i];
        C.red[i] = T.reduce_q[i];
        C.g[i] = T.crt_g[i];
        C.m[i] = T.crt_m[i];
    }
    C.Q = T.Q_mod64;
    return C;
}
}  // namespace

hipError_t launch_fill_u64(uint64_t* p, size_t count, uint64_t v, hipStream_t st) {
    if (!count) return hipSuccess;
    const int blocks = int(std::min<size_t>((count + 255) / 256, 4096));
    hipLaunchKernelGGL(dev::fill_u64_kernel, dim3(blocks), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

int keyswitch_splits(int B, int tile) {
    // enough workgroups to fill the chip: tiles x splits >= 1024, at most 64
    // splits of 32 input coefficients, and at most kKsPartRows partial rows
    const int tiles = (B + tile - 1) / tile;
    int s = 1;
    while (s < 64 && tiles * s < 1024) s *= 2;
    while (s > 1 && size_t(s) * size_t(B) > kKsPartRows) s /= 2;
    return s;
}

size_t keyswitch_part_words(int B) {
    // A smaller batch can take more splits than a larger one, so the buffer
    // must hold the largest splits(b) * b over every b <= B and every tile;
    // past kKsPartRows ciphertexts a batch takes one split.
    size_t most = size_t(std::max(B, 1));
    const int top = std::min<int>(B, int(kKsPartRows));
    for (int tile : {4, 8, 16})
        for (int b = 1; b <= top; ++b) most = std::max(most, size_t(keyswitch_splits(b, tile)) * size_t(b));
    return most * kSmallWords;
}

hipError_t launch_keyswitch_jobs(const Job* jobs, int B, const uint64_t* ksk, uint64_t* part, hipStream_t st,
                                 int nsplit, int tile) {
    if (B <= 0) return hipSuccess;
    if (nsplit < 0 || nsplit > 64 || (nsplit & (nsplit - 1))) return hipErrorInvalidValue;
    if (tile != 4 && tile != 8 && tile != 16) return hipErrorInvalidValue;
    const int ns = nsplit ? nsplit : keyswitch_splits(B, tile);
    dim3 grid((B + tile - 1) / tile, ns);
    const int chunk = kN / ns;   // input coefficients per split, a power of two
    const int sub = std::min(chunk, dev::kKsSub);
    if (tile == 4)
        hipLaunchKernelGGL(dev::keyswitch_jobs_kernel<4>, grid, dim3(256), 0, st, jobs, B, ksk, part, chunk, sub);
    else if (tile == 8)
        hipLaunchKernelGGL(dev::keyswitch_jobs_kernel<8>, grid, dim3(256), 0, st, jobs, B, ksk, part, chunk, sub);
    else
        hipLaunchKernelGGL(dev::keyswitch_jobs_kernel<16>, grid, dim3(256), 0, st, jobs, B, ksk, part, chunk, sub);
    return hipGetLastError();
}

hipError_t prepare_kernels() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(dev::blind_rotate_latency_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(dev::kLatLds));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(dev::blind_rotate_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(dev::kBrLds));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(dev::blind_rotate_w16_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(dev::kW16Lds));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(dev::blind_rotate_pair_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(dev::kPairLds));
    return e;
}

hipError_t launch_blind_rotate_jobs(const Job* jobs, int B, const uint64_t* part, const uint64_t* luts,
                                    const uint32_t* bsk, const DevTables& t, int grid, int latency_form_max,
                                    int latency_waves, hipStream_t st, int nsplit, int throughput_waves) {
    if (B <= 0) return hipSuccess;
    if (nsplit < 0 || nsplit > 64 || (nsplit & (nsplit - 1))) return hipErrorInvalidValue;
    dev::BrArgs A{};
    A.jobs = jobs;
    A.part = part;
    A.nsplit = nsplit ? nsplit : keyswitch_splits(B);
    A.luts = luts;
    A.bsk = bsk;
    A.tw = dev::Tw{reinterpret_cast<const uint2*>(t.fwd), reinterpret_cast<const uint2*>(t.inv)};
    A.crt = make_crt();
    A.B = B;
    if (grid <= 0 || grid > B) grid = B;
    if (B <= latency_form_max && latency_waves == 16)
        hipLaunchKernelGGL(dev::blind_rotate_w16_kernel, dim3(grid), dim3(dev::kW16Threads), dev::kW16Lds, st, A);
    else if (B <= latency_form_max)
        hipLaunchKernelGGL(dev::blind_rotate_latency_kernel, dim3(grid), dim3(dev::kLatThreads), dev::kLatLds, st, A);
    else if (throughput_waves == 8)
        hipLaunchKernelGGL(dev::blind_rotate_pair_kernel, dim3(grid), dim3(dev::kLatThreads), dev::kPairLds, st, A);
    else
        hipLaunchKernelGGL(dev::blind_rotate_kernel, dim3(grid), dim3(dev::kBrThreads), dev::kBrLds, st, A);
    return hipGetLastError();
}

hipError_t launch_bsk_convert(const uint64_t* bsk_u64, uint32_t* out, const DevTables& t, hipStream_t st) {
    dim3 grid(kSmallN * 2, kPrimes);
    hipLaunchKernelGGL(dev::bsk_convert_kernel, grid, dim3(64), 0, st, bsk_u64, out,
                       dev::Tw{reinterpret_cast<const uint2*>(t.fwd), reinterpret_cast<const uint2*>(t.inv)}, make_crt(),
                       t.scale, t.scale_s);
    return hipGetLastError();
}

hipError_t launch_group_sum(const uint64_t* in, uint64_t* out, size_t items, int cnt, int groups, int group,
                            int cus, hipStream_t st) {
    const size_t total = items * size_t(groups) * kCtWords;
    if (!total) return hipSuccess;
    const int blocks = int(std::min<size_t>((total + 255) / 256, size_t(std::max(1, cus)) * 16));
    hipLaunchKernelGGL(dev::group_sum_kernel, dim3(blocks), dim3(256), 0, st, in, out, items, cnt, groups, group);
    return hipGetLastError();
}

hipError_t launch_trivial(uint64_t* out, int count, uint32_t mu, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::trivial_kernel, dim3(unsigned(count * dev::kWordBlocks)), dim3(256), 0, st, out, mu);
    return hipGetLastError();
}

}  // namespace lvs
