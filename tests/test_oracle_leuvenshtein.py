"""Pins of the encrypted Leuvenshtein oracle (Algorithms 3 and 4, Section 5
preprocessing of arXiv 2508.14568) against the plaintext definitions."""
import itertools

import pytest

import numpy as np

from conftest import golden
from oracle import leuvenshtein as L
from oracle import plaintext as P
from oracle import tfhe as T


def test_dna_equality_all_pairs(oracle_toy_keys):
    k = oracle_toy_keys
    A = L.encrypt_string(k, "ACGT", L.ENC_DNA2, 1)
    B = L.encrypt_string(k, "ACGT", L.ENC_DNA2, 2)
    _, eq9 = L.equality(k, A, B, L.ENC_DNA2)
    for i, j in itertools.product(range(4), range(4)):
        assert k.decrypt(eq9[i, j]) == (9 if i == j else 0)


def test_ascii_equality_algorithm3(oracle_toy_keys):
    """Pairs equal in both symbols, only the 4-bit one, only the 3-bit one, or
    neither (Section 4.3); eq1 decrypts to the 4-bit equality."""
    k = oracle_toy_keys
    xs = b"aAqQ0p~ "
    ys = b"aQqA1` ~"
    A = L.encrypt_string(k, xs, L.ENC_ASCII7, 3)
    B = L.encrypt_string(k, ys, L.ENC_ASCII7, 4)
    eq1, eq9 = L.equality(k, A, B, L.ENC_ASCII7)
    for i, j in itertools.product(range(len(xs)), range(len(ys))):
        assert k.decrypt(eq1[i, j]) == (1 if (xs[i] & 15) == (ys[j] & 15) else 0)
        assert k.decrypt(eq9[i, j]) == (9 if xs[i] == ys[j] else 0)


def test_fig3_encrypted(oracle_toy_keys):
    """KID / SIT: every M decrypts to the plaintext diagonal difference and the
    returned bottom row gives the distance 2 (Fig. fig_myers)."""
    k = oracle_toy_keys
    g = golden("fig3_kid_sit.json")
    A = L.encrypt_string(k, g["a"].encode(), L.ENC_ASCII7, 5)
    B = L.encrypt_string(k, g["b"].encode(), L.ENC_ASCII7, 6)
    h_last, rec = L.edit_distance(k, A, B, L.ENC_ASCII7, record=True)
    _, h, M = P.delta_dp(g["a"], g["b"])
    for (i, j), ct in rec["M"].items():
        assert k.decrypt_signed(ct) == M[i, j]
    assert [k.decrypt_signed(c) for c in h_last] == g["dh_rows"][3]
    assert L.decrypt_distance(k, 3, h_last) == g["distance"]


def test_alg4_order_equals_diagonal_order(oracle_toy_keys):
    """Section 6.2: cells of one anti-diagonal are independent, so evaluating
    them as a batch yields bit-identical ciphertexts."""
    k = oracle_toy_keys
    A = L.encrypt_string(k, b"ACGTTG", L.ENC_DNA2, 7)
    B = L.encrypt_string(k, b"CGTAA", L.ENC_DNA2, 8)
    _, eq9 = L.equality(k, A, B, L.ENC_DNA2)
    h1, r1 = L.dp(k, 6, 5, lambda i, j: eq9[i - 1, j - 1], order="alg4", record=True)
    h2, r2 = L.dp(k, 6, 5, lambda i, j: eq9[i - 1, j - 1], order="diagonal", record=True)
    assert (h1 == h2).all()
    for key in r1["M"]:
        assert (r1["M"][key] == r2["M"][key]).all()


def test_random_pairs_distance(oracle_toy_keys):
    k = oracle_toy_keys
    rng = np.random.default_rng(9)
    for t in range(4):
        a = bytes(int(c) for c in rng.choice(list(b"ACGT"), size=int(rng.integers(1, 7))))
        b = bytes(int(c) for c in rng.choice(list(b"ACGT"), size=int(rng.integers(1, 7))))
        A = L.encrypt_string(k, a, L.ENC_DNA2, 100 + t)
        B = L.encrypt_string(k, b, L.ENC_DNA2, 200 + t)
        h_last = L.edit_distance(k, A, B, L.ENC_DNA2)
        assert L.decrypt_distance(k, len(a), h_last) == P.edit_distance(a, b)


def test_empty_strings(oracle_toy_keys):
    k = oracle_toy_keys
    A = L.encrypt_string(k, b"ACG", L.ENC_DNA2, 1)
    E = L.encrypt_string(k, b"", L.ENC_DNA2, 2)
    assert L.decrypt_distance(k, 3, L.edit_distance(k, A, E, L.ENC_DNA2)) == 3
    assert L.decrypt_distance(k, 0, L.edit_distance(k, E, A, L.ENC_DNA2)) == 3
    assert L.decrypt_distance(k, 0, L.edit_distance(k, E, E, L.ENC_DNA2)) == 0


def test_preprocessing_table_abbey(oracle_toy_keys):
    """Table tab_pre: one enc(9) per column at the row of the character, zeros
    elsewhere (stored as eq9, as Section 5 allows)."""
    k = oracle_toy_keys
    g = golden("tab_pre_abbey.json")
    A = L.encrypt_string(k, g["word"].encode(), L.ENC_ASCII7, 12)
    alpha = g["alphabet"].encode()
    Tab = L.preprocess(k, A, alpha, L.ENC_ASCII7)
    dec = [[k.decrypt(Tab[c, i]) // 9 for i in range(5)] for c in range(len(alpha))]
    for ch, row in g["printed_rows"].items():
        assert dec[alpha.index(ch.encode())] == row
    assert all(sum(dec[c][i] for c in range(len(alpha))) == 1 for i in range(5))


def test_preprocessed_main_pass_matches(oracle_toy_keys):
    k = oracle_toy_keys
    a, b = b"kitten", b"sitting"
    alpha = bytes(sorted(set(b)))
    A = L.encrypt_string(k, a, L.ENC_ASCII7, 31)
    Tab = L.preprocess(k, A, alpha, L.ENC_ASCII7)
    h_last = L.edit_distance_clear(k, Tab, alpha, b, L.ENC_ASCII7)
    assert L.decrypt_distance(k, len(a), h_last) == P.edit_distance(a, b) == 3


def test_small_dna_full_parameters(oracle_keys):
    k = oracle_keys
    a, b = b"GAT", b"GT"
    A = L.encrypt_string(k, a, L.ENC_DNA2, 41)
    B = L.encrypt_string(k, b, L.ENC_DNA2, 42)
    h_last, rec = L.edit_distance(k, A, B, L.ENC_DNA2, record=True)
    assert L.decrypt_distance(k, 3, h_last) == P.edit_distance(a, b) == 1
    _, _, M = P.delta_dp(a, b)
    for (i, j), ct in rec["M"].items():
        assert k.decrypt_signed(ct) == M[i, j]


def test_band_encrypted_matches_plaintext(oracle_toy_keys):
    """Algorithm 1's band (Section 3.2) on encrypted DNA: every computed
    difference decrypts to the plaintext banded loop's value, cells outside
    the band are never bootstrapped, and the path decrypts to the banded
    distance (exact band: the Wagner-Fischer distance)."""
    k = oracle_toy_keys
    a, b = "ACGTTGCA", "CGTTAGCAT"
    A = L.encrypt_string(k, a.encode(), L.ENC_DNA2, 11)
    B = L.encrypt_string(k, b.encode(), L.ENC_DNA2, 12)
    for ell in (1, 3, P.exact_band(len(a), len(b))):
        path, rec = L.edit_distance_band(k, A, B, L.ENC_DNA2, ell, record=True)
        v, h = P.delta_dp_band(a, b, ell)
        assert set(rec["v"]) == {(i, j) for i in range(1, 9) for j in range(1, 10) if abs(i - j) <= ell}
        for (i, j), ct in rec["v"].items():
            assert k.decrypt_signed(ct) == v[i, j]
            assert k.decrypt_signed(rec["h"][(i, j)]) == h[i, j]
        assert len(path) == len(a) + len(b)
        assert L.decrypt_path(k, path) == P.band_distance(a, b, ell)
    assert L.decrypt_path(k, path) == P.edit_distance(a, b)


def test_band_cleartext_equals_encrypted(oracle_toy_keys):
    """The Section 5 table read by the banded loop gives the same path
    ciphertexts' values as the both-encrypted banded loop (ASCII)."""
    k = oracle_toy_keys
    a, b = b"kitten", b"sitting"
    A = L.encrypt_string(k, a, L.ENC_ASCII7, 13)
    alphabet = bytes(sorted(set(b)))
    table = L.preprocess(k, A, alphabet, L.ENC_ASCII7)
    ell = P.exact_band(len(a), len(b))
    path = L.edit_distance_clear_band(k, table, alphabet, b, ell)
    assert L.decrypt_path(k, path) == P.edit_distance(a, b) == 3
    B = L.encrypt_string(k, b, L.ENC_ASCII7, 14)
    path2 = L.edit_distance_band(k, A, B, L.ENC_ASCII7, 1)
    assert L.decrypt_path(k, path2) == P.band_distance(a, b, 1)


class _CountingKeys:
    """Keys whose bootstraps through the refresh table are logged."""

    def __init__(self, keys):
        self._k = keys
        self.refresh_calls = []

    def __getattr__(self, name):
        return getattr(self._k, name)

    def pbs_batch(self, cts, polys, lut_ids, nthreads=None):
        out = self._k.pbs_batch(cts, polys, lut_ids, nthreads)
        if np.isscalar(lut_ids) and lut_ids == L.LUT_IDS["refresh"]:
            self.refresh_calls.append((np.array(cts), out))
        return out


def test_refresh_table_is_identity_on_differences(oracle_toy_keys):
    """Section 3.1's refresh: a bootstrap through the refresh table returns
    -1, 0 and 1 unchanged, with the noise of a fresh bootstrap."""
    k = oracle_toy_keys
    tp = L.lut_polys(k.N)
    cts = []
    for x, off in [(0, 2**56), (1, -(2**56)), (31, 3 * 2**55), (1, 0)]:
        ct = k.encrypt(x, 19, x)
        ct[k.N] = np.uint64((int(ct[k.N]) + off) % 2**64)
        cts.append(ct)
    outs = k.pbs_batch(np.stack(cts), tp, L.LUT_IDS["refresh"])
    assert [k.decrypt_signed(o) for o in outs] == [0, 1, -1, 1]
    assert all(abs(k.phase_error(o)) < 2**52 for o in outs)


def test_refresh_schedule_keeps_distances(oracle_toy_keys):
    """Refreshing every R-th anti-diagonal changes no plaintext: distances
    stay the Wagner-Fischer ones; the refresh runs on exactly the diagonals
    s = R, 2R, ... below m + n, on the v and h of their cells, each output
    decrypting to its input."""
    rng = np.random.default_rng(23)
    for t, R in enumerate((2, 3, 5)):
        k = _CountingKeys(oracle_toy_keys)
        m, n = int(rng.integers(4, 9)), int(rng.integers(4, 9))
        a = bytes(int(c) for c in rng.choice(list(b"ACGT"), size=m))
        b = bytes(int(c) for c in rng.choice(list(b"ACGT"), size=n))
        A = L.encrypt_string(k, a, L.ENC_DNA2, 300 + t)
        B = L.encrypt_string(k, b, L.ENC_DNA2, 400 + t)
        h_last = L.edit_distance(k, A, B, L.ENC_DNA2, refresh_every=R)
        assert L.decrypt_distance(k, m, h_last) == P.edit_distance(a, b)
        diags = [s for s in range(2, m + n) if s % R == 0]
        assert len(k.refresh_calls) == len(diags)
        for s, (ins, outs) in zip(diags, k.refresh_calls):
            cells = min(m, s - 1) - max(1, s - n) + 1
            assert ins.shape[0] == 2 * cells
            assert [k.decrypt_signed(c) for c in ins] == [k.decrypt_signed(c) for c in outs]
            assert {k.decrypt_signed(c) for c in outs} <= {-1, 0, 1}


def test_refresh_band_and_cleartext(oracle_toy_keys):
    """The banded loop and the Section 5 cleartext loop with refresh give the
    same distances as without."""
    k = oracle_toy_keys
    a, b = "ACGTTGCA", "CGTTAGCAT"
    A = L.encrypt_string(k, a.encode(), L.ENC_DNA2, 15)
    B = L.encrypt_string(k, b.encode(), L.ENC_DNA2, 16)
    for ell in (1, P.exact_band(len(a), len(b))):
        path = L.edit_distance_band(k, A, B, L.ENC_DNA2, ell, refresh_every=3)
        assert L.decrypt_path(k, path) == P.band_distance(a, b, ell)
    a2, b2 = b"kitten", b"sitting"
    A2 = L.encrypt_string(k, a2, L.ENC_ASCII7, 17)
    alpha = bytes(sorted(set(b2)))
    Tab = L.preprocess(k, A2, alpha, L.ENC_ASCII7)
    h_last = L.edit_distance_clear(k, Tab, alpha, b2, L.ENC_ASCII7, refresh_every=4)
    assert L.decrypt_distance(k, len(a2), h_last) == 3


class _LutCountingKeys(_CountingKeys):
    """Keys that count bootstraps per table."""

    def __init__(self, keys):
        super().__init__(keys)
        self.count = {}

    def pbs_batch(self, cts, polys, lut_ids, nthreads=None):
        name = {v: k for k, v in L.LUT_IDS.items()}[int(lut_ids)]
        self.count[name] = self.count.get(name, 0) + np.asarray(cts).reshape(-1, self._k.N + 1).shape[0]
        return self._k.pbs_batch(cts, polys, lut_ids, nthreads)


@pytest.mark.parametrize("width", [4, 7, 21, 64])
def test_wide_equality_encrypted(oracle_toy_keys, width):
    """Section 4.2's hybrid on encrypted symbols: eq9 decrypts to 9 [x = y]
    for equal pairs, pairs differing in one chunk only, and random pairs; the
    bootstraps per pair match the count of the method (one per chunk, then
    the merging levels)."""
    k = _LutCountingKeys(oracle_toy_keys)
    rng = np.random.default_rng(width)
    base = [int(rng.integers(0, 2 ** min(width, 62))) % (2 ** width) for _ in range(3)]
    xs = base + [base[0]]
    ys = [base[1], base[0] ^ (1 << int(rng.integers(0, width))), int(rng.integers(0, 2 ** min(width, 62))),
          base[0]]
    A = L.encrypt_symbols(k, xs, width, 51)
    B = L.encrypt_symbols(k, ys, width, 52)
    assert A.shape == (4, P.wide_chunk_count(width), k.N + 1)
    eq9 = L.equality_wide(k, A, B, width)
    for i, x in enumerate(xs):
        for j, y in enumerate(ys):
            assert k.decrypt(eq9[i, j]) == (9 if x == y else 0), (i, j)
    assert sum(k.count.values()) == 16 * P.pbs_hybrid(width)
    c = P.wide_chunk_count(width)
    if c > 1:
        assert k.count["eq"] == 16 * c and k.count["max9"] == 16


def test_wide_edit_distance(oracle_toy_keys):
    """Edit distance over 21-bit symbols (Unicode code points) equals
    Wagner-Fischer on the symbol sequences, with and without refresh."""
    k = oracle_toy_keys
    rng = np.random.default_rng(77)
    alphabet = [int(v) for v in rng.integers(0, 2 ** 21, size=4)]
    a = [alphabet[int(t)] for t in rng.integers(0, 4, size=5)]
    b = [alphabet[int(t)] for t in rng.integers(0, 4, size=6)]
    A = L.encrypt_symbols(k, a, 21, 61)
    B = L.encrypt_symbols(k, b, 21, 62)
    for R in (0, 4):
        h_last = L.edit_distance_wide(k, A, B, 21, refresh_every=R)
        assert L.decrypt_distance(k, len(a), h_last) == P.edit_distance(a, b)


def test_wide_preprocessing_table(oracle_toy_keys):
    """Section 5's table over wide symbols: one Enc(9) per column at the
    row of the symbol; the cleartext main pass gives the Wagner-Fischer
    distance."""
    k = oracle_toy_keys
    a = [0x1F600, 0x41, 0x1F600, 0x3042, 0x41]
    b = [0x41, 0x1F600, 0x3042, 0x3042]
    alphabet = sorted(set(b)) + [0x10FFFF]
    A = L.encrypt_symbols(k, a, 21, 71)
    table = L.preprocess_wide(k, A, alphabet, 21)
    for s_, v in enumerate(alphabet):
        assert [k.decrypt(table[s_, i]) for i in range(len(a))] == [9 if x == v else 0 for x in a]
    h_last = L.edit_distance_clear(k, table, alphabet, b, None)
    assert L.decrypt_distance(k, len(a), h_last) == P.edit_distance(a, b)
