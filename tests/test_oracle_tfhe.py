"""Pins of the oracle's TFHE layer (schoolbook arithmetic in Z/2^64).

Each check is fixed by something outside the oracle: published generator
outputs, brute-force big-integer arithmetic, algebraic identities, decryption
with the secret key, and the paper's printed lookup tables (arXiv 2508.14568,
Section 2.2 Table table_lutrelu, Section 3.1 Table LUTmin).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import golden
from oracle import plaintext as P
from oracle import tfhe as T

M64 = 2**64


def brute_negacyclic(a, d, N):
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += int(a[i]) * int(d[j])
            else:
                out[k - N] -= int(a[i]) * int(d[j])
    return [x % M64 for x in out]


def test_splitmix64_published_sequence():
    """SplitMix64 seeded with 1234567 (reference outputs of the published
    generator); draw(key, i) is output i+1 of a generator whose state is key."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [T.draw(1234567, i) for i in range(5)] == want


def test_gaussian_moments_and_bounds():
    sigma = 130415703530680
    key = T.stream_key(3, 99)
    e = np.array([T.gaussian(key, i, sigma) for i in range(20000)], dtype=np.uint64).view(np.int64)
    x = e.astype(np.float64) / sigma
    assert abs(x.mean()) < 0.03
    assert abs(x.std() - 1.0) < 0.03
    assert np.abs(x).max() <= 6.0 + 1e-9


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_negacyclic_mul_brute_force(N):
    rng = np.random.default_rng(N)
    for _ in range(5):
        a = rng.integers(0, 2**63, size=N, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=N, dtype=np.uint64)
        d = rng.integers(-2**22, 2**22, size=N).astype(np.int64)
        assert T.negacyclic_mul(a, d).tolist() == brute_negacyclic(a, d, N)


def test_negacyclic_mul_full_size_against_convolution():
    """N = 2048: full integer convolution (Python ints) folded with X^N = -1."""
    N = 2048
    rng = np.random.default_rng(5)
    a = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
    d = rng.integers(-2**22, 2**22, size=N).astype(np.int64)
    full = np.convolve(np.array([int(x) for x in a], dtype=object), np.array([int(x) for x in d], dtype=object))
    folded = [(full[k] - (full[k + N] if k + N < len(full) else 0)) % M64 for k in range(N)]
    assert T.negacyclic_mul(a, d).tolist() == folded


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32, 64])
def test_negacyclic_mul_karatsuba_brute_force(N):
    """Karatsuba's product against the big-integer double sum: below, at and
    above its 8-coefficient schoolbook blocks (one to three recursion levels)."""
    rng = np.random.default_rng(100 + N)
    for _ in range(6):
        a = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
        d = rng.integers(-2**22, 2**22, size=N).astype(np.int64)
        assert T.negacyclic_mul_karatsuba(a, d).tolist() == brute_negacyclic(a, d, N)


def test_negacyclic_mul_karatsuba_full_size_against_convolution():
    """N = 2048 (eight recursion levels): the folded integer convolution, on
    random operands and on the extremes (every key word 2^64 - 1 or 2^63,
    every digit -2^22 or 2^22 - 1), where any carry or sign slip shows."""
    N = 2048
    rng = np.random.default_rng(6)
    cases = [(rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True),
              rng.integers(-2**22, 2**22, size=N).astype(np.int64)),
             (np.full(N, 2**64 - 1, dtype=np.uint64), np.full(N, -2**22, dtype=np.int64)),
             (np.full(N, 2**63, dtype=np.uint64), np.full(N, 2**22 - 1, dtype=np.int64))]
    for a, d in cases:
        full = np.convolve(np.array([int(x) for x in a], dtype=object), np.array([int(x) for x in d], dtype=object))
        folded = [(full[k] - (full[k + N] if k + N < len(full) else 0)) % M64 for k in range(N)]
        assert T.negacyclic_mul_karatsuba(a, d).tolist() == folded


def test_negacyclic_mul_karatsuba_equals_schoolbook():
    for N in (128, 512, 2048):
        rng = np.random.default_rng(N)
        for _ in range(3):
            a = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
            d = rng.integers(-2**22, 2**22, size=N).astype(np.int64)
            assert (T.negacyclic_mul_karatsuba(a, d) == T.negacyclic_mul(a, d)).all()


def test_pbs_karatsuba_equals_schoolbook(oracle_keys):
    """The blind rotation with Karatsuba's products gives the same words as
    with the schoolbook sums: three bootstraps at the benchmark parameters
    (one with a large input error) and all 32 inputs at toy parameters."""
    k = oracle_keys
    tp = np.stack([T.test_polynomial(P.lut_min_negated(), k.N), T.test_polynomial(P.LUT_EQ9, k.N)])
    cts = np.stack([k.encrypt(x, 31, x) for x in (0, 7, 19)])
    cts[2, k.N] = np.uint64((int(cts[2, k.N]) + 3 * 2**55) % M64)
    ids = [0, 1, 0]
    assert not k.karatsuba
    school = k.pbs_batch(cts, tp, ids)
    k.karatsuba = True
    try:
        kara = k.pbs_batch(cts, tp, ids)
    finally:
        k.karatsuba = False
    assert (school == kara).all()
    toy = T.Keys(T.toy_params(), seed=12)
    tpt = T.test_polynomial(P.LUT_X_MINUS_4, toy.N)
    cts = np.stack([toy.encrypt(x, 5, x) for x in range(32)])
    school = toy.pbs_batch(cts, tpt[None], 0)
    toy.karatsuba = True
    assert (toy.pbs_batch(cts, tpt[None], 0) == school).all()


def test_monomial_identities():
    N = 64
    rng = np.random.default_rng(2)
    a = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
    assert (T.monomial_mul(a, 0) == a).all()
    assert (T.monomial_mul(a, N) == (np.uint64(0) - a)).all()           # X^N = -1
    for e1, e2 in [(3, 5), (60, 70), (127, 1), (100, 100)]:
        lhs = T.monomial_mul(T.monomial_mul(a, e1), e2)
        assert (lhs == T.monomial_mul(a, (e1 + e2) % (2 * N))).all()
    # agrees with the schoolbook product by a monomial
    for e in (1, 17, 63):
        d = np.zeros(N, dtype=np.int64)
        d[e] = 1
        assert (T.negacyclic_mul(a, d) == T.monomial_mul(a, e)).all()


@pytest.mark.parametrize("base_log,level", [(23, 1), (3, 5), (4, 3), (10, 2)])
def test_decomposition_recomposes_within_half_step(base_log, level):
    rng = np.random.default_rng(base_log * 10 + level)
    prec = base_log * level
    vals = [0, M64 - 1, 2**63, 2**63 - 1, 1 << (63 - prec), (1 << (63 - prec)) - 1,
            (1 << (64 - prec)) * 5 + (1 << (63 - prec))] + [int(x) for x in rng.integers(0, 2**63, size=200)] \
        + [int(x) + 2**63 for x in rng.integers(0, 2**63, size=200)]
    for c in vals:
        dig = T.decompose(c, base_log, level)
        assert all(-(1 << (base_log - 1)) <= x < (1 << (base_log - 1)) for x in dig)
        rec = sum(x * (1 << (64 - base_log * (lev + 1))) for lev, x in enumerate(dig)) % M64
        err = (c - rec) % M64
        err = err - M64 if err >= 2**63 else err
        assert -(1 << (63 - prec)) <= err < (1 << (63 - prec))   # rounding half up


def test_encrypt_decrypt_roundtrip(oracle_keys):
    k = oracle_keys
    for mu in range(32):
        ct = k.encrypt(mu, 1000 + mu, 7)
        assert k.decrypt(ct) == mu
        assert abs(k.phase_error(ct)) <= 6 * 5424 + 1


def test_keys_binary_and_bsk_rows_decrypt(oracle_keys):
    """GGSW(s_i) rows: B - A*S is noise - s_i g S on the mask row and
    noise + s_i g on the body row (g = 2^41)."""
    k = oracle_keys
    s, S = k.small_key, k.big_key
    assert set(np.unique(s)) <= {0, 1} and set(np.unique(S)) <= {0, 1}
    assert 200 < s.sum() < 542 and 800 < S.sum() < 1248
    bsk = k.bsk()
    g = 1 << 41
    Sd = S.astype(np.int64)
    for i in (0, 1, 371, 741):
        for row in (0, 1):
            A, B = bsk[i, row, 0], bsk[i, row, 1]
            phase = (B - T.negacyclic_mul(A, Sd)).astype(np.uint64).view(np.int64).astype(object)
            if row == 1:
                expect = np.zeros(k.N, dtype=object)
                expect[0] = g * int(s[i])
            else:
                expect = np.array([-g * int(s[i]) * int(x) for x in S], dtype=object)
            noise = phase - expect
            assert max(abs(int(x)) for x in noise) <= 6 * 5424 + 1


def test_ksk_rows_decrypt(oracle_keys):
    k = oracle_keys
    ksk, S = k.ksk(), k.big_key
    for j in (0, 5, 2047):
        for t in range(1, 6):
            ph = k.phase_small(ksk[j * 5 + t - 1])
            want = (int(S[j]) << (64 - 3 * t)) % M64
            err = (ph - want) % M64
            err = err - M64 if err >= 2**63 else err
            assert abs(err) <= 6 * 130415703530680 + 1


def test_keyswitch_preserves_message(oracle_keys):
    k = oracle_keys
    for mu in (0, 1, 9, 15, 16, 31):
        ct = k.encrypt(mu, 55, mu)
        small = k.keyswitch(ct)
        ph = k.phase_small(small)
        assert (((ph >> 58) + 1) >> 1) % 32 == mu
        err = (ph - (mu << 59)) % M64
        err = err - M64 if err >= 2**63 else err
        assert abs(err) < 2**57


def test_modswitch_rounding():
    k = T.Keys(T.toy_params(), seed=3)          # only the sizes matter here
    N = k.N
    shift = 64 - (2 * N).bit_length() + 1       # 2^64 / 2N
    vals = np.array([0, 1 << (shift - 1), (1 << (shift - 1)) - 1, M64 - 1, 2**63, 5 << shift]
                    + [0] * (k.n + 1 - 6), dtype=np.uint64)
    out = k.modswitch(vals)
    # nearest integer to v * 2N / 2^64, ties rounded up, reduced mod 2N
    expect = [math.floor(Fraction(int(v) * 2 * N, M64) + Fraction(1, 2)) % (2 * N) for v in vals]
    assert out.tolist() == expect
    assert out[1] == 1 and out[2] == 0 and out[3] == 0 and out[4] == N


def test_sample_extract_phase():
    """The extracted LWE's phase is coefficient 0 of the GLWE phase."""
    k = T.Keys(T.toy_params(), seed=4)
    N = k.N
    rng = np.random.default_rng(0)
    A = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
    B = rng.integers(0, 2**64 - 1, size=N, dtype=np.uint64, endpoint=True)
    glwe_phase = (B - T.negacyclic_mul(A, k.big_key.astype(np.int64))).astype(np.uint64)
    lwe = k.sample_extract(np.concatenate([A, B]))
    assert k.phase(lwe) == int(glwe_phase[0])


def test_blind_rotate_trivial_input_is_rotation():
    """All-zero mask: every CMux adds ExtProd(BSK_i, 0) = 0, so the result is
    exactly (0, X^{-b} * testpoly)."""
    k = T.Keys(T.toy_params(), seed=5)
    tp = T.test_polynomial(P.LUT_X_MINUS_4, k.N)
    for b in (0, 1, 100, 2 * k.N - 1):
        ms = np.zeros(k.n + 1, dtype=np.uint32)
        ms[k.n] = b
        acc = k.blind_rotate(tp, ms)
        assert (acc[:k.N] == 0).all()
        assert (acc[k.N:] == T.monomial_mul(tp, (2 * k.N - b) % (2 * k.N))).all()


def _exhaustive(keys, lut16, seed):
    tp = T.test_polynomial(lut16, keys.N)
    cts = np.stack([keys.encrypt(x, seed, x) for x in range(32)])
    outs = keys.pbs_batch(cts, tp[None, :], 0)
    return [keys.decrypt(o) for o in outs]


@pytest.mark.parametrize("name", ["x-4", "lutmin_plain", "lutmin_negated", "eq", "eq9", "refresh"])
def test_pbs_exhaustive_toy(oracle_toy_keys, name):
    lut = {"x-4": P.LUT_X_MINUS_4, "lutmin_plain": P.lut_min_plain(), "lutmin_negated": P.lut_min_negated(),
           "eq": P.LUT_EQ, "eq9": P.LUT_EQ9, "refresh": P.LUT_REFRESH}[name]
    got = _exhaustive(oracle_toy_keys, lut, 77)
    assert got == [P.negacyclic_read(lut, x) for x in range(32)]


def test_pbs_table1_full_parameters(oracle_keys):
    """Table table_lutrelu, all 32 inputs, at the benchmark parameters."""
    got = _exhaustive(oracle_keys, P.LUT_X_MINUS_4, 2024)
    assert [g % 16 for g in got] == golden("table1_lut_x_minus_4.json")["outputs"]


def test_pbs_table2_full_parameters(oracle_keys):
    got = _exhaustive(oracle_keys, P.lut_min_plain(), 2025)
    assert [g % 16 for g in got] == golden("table2_lutmin.json")["outputs"]


def test_pbs_output_noise_is_fresh(oracle_keys):
    """A bootstrap's output noise does not depend on its input noise: inputs
    with large (but decodable) phase errors come out with small errors."""
    k = oracle_keys
    tp = T.test_polynomial(P.LUT_EQ9, k.N)
    cts = []
    for x, off in [(0, 2**56), (0, -(2**56)), (3, 3 * 2**55), (17, -(3 * 2**55))]:
        ct = k.encrypt(x, 9, x)
        ct[k.N] = np.uint64((int(ct[k.N]) + off) % M64)
        cts.append(ct)
    outs = k.pbs_batch(np.stack(cts), tp[None, :], 0)
    for (x, _), o in zip([(0, 0), (0, 0), (3, 0), (17, 0)], outs):
        assert k.decrypt(o) == P.negacyclic_read(P.LUT_EQ9, x)
        assert abs(k.phase_error(o)) < 2**52
