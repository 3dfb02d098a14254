"""Pins of the oracle's plaintext layer against the paper's printed values,
closed forms and brute force (arXiv 2508.14568)."""
import functools
import itertools

import numpy as np

from conftest import golden
from oracle import plaintext as P


def recursive_levenshtein(a, b):
    """The original recursive definition (Section 2.3), memoised; independent
    of the dynamic-programming oracle."""
    @functools.lru_cache(maxsize=None)
    def lev(i, j):
        if i == len(a):
            return len(b) - j
        if j == len(b):
            return len(a) - i
        if a[i] == b[j]:
            return lev(i + 1, j + 1)
        return 1 + min(lev(i + 1, j), lev(i, j + 1), lev(i + 1, j + 1))
    return lev(0, 0)


def test_fig1_dmatrices():
    for case in golden("fig1_dmatrix.json")["cases"]:
        D = P.wagner_fischer(case["a"], case["b"])
        assert D.tolist() == case["D"]
        assert P.edit_distance(case["a"], case["b"]) == case["distance"]


def test_fig3_delta_arrows():
    g = golden("fig3_kid_sit.json")
    D = P.wagner_fischer(g["a"], g["b"])
    assert D.tolist() == g["D"]
    v, h, M = P.delta_dp(g["a"], g["b"])
    for i, row in enumerate(g["dh_rows"]):
        assert [int(h[i, j]) for j in range(1, 4)] == row
    for j, col in enumerate(g["dv_cols"]):
        assert [int(v[i, j]) for i in range(1, 4)] == col
    assert P.distance_from_last_row(3, h[3, 1:]) == g["distance"]
    # M is the diagonal difference D[i,j] - D[i-1,j-1]
    assert (M[1:, 1:] == D[1:, 1:] - D[:-1, :-1]).all()


def test_section2_hamming_vs_edit():
    g = golden("section2_examples.json")
    assert sum(x != y for x, y in zip(g["a"], g["b"])) == g["hamming"]
    assert P.edit_distance(g["a"], g["b"]) == g["edit"]


def test_wf_and_delta_dp_exhaustive_small():
    """Every pair of strings of length <= 4 over a 3-letter alphabet: WF equals
    the recursive definition, and the difference DP reproduces WF's
    differences and distance."""
    alphabet = "abc"
    strings = [""] + ["".join(t) for L in range(1, 5) for t in itertools.product(alphabet, repeat=L)]
    rng = np.random.default_rng(0)
    sample = [strings[k] for k in rng.choice(len(strings), size=60, replace=False)] + ["", "a", "abc"]
    for a in sample:
        for b in sample:
            D = P.wagner_fischer(a, b)
            assert D[len(a), len(b)] == recursive_levenshtein(a, b)
            v, h, _ = P.delta_dp(a, b)
            dv, dh = P.deltas_from_matrix(D)
            if a and b:
                assert (v[1:, :] == dv[1:, :]).all() and (h[:, 1:] == dh[:, 1:]).all()
            assert P.distance_from_last_row(len(a), h[len(a), 1:]) == D[len(a), len(b)]


def test_random_longer_strings():
    rng = np.random.default_rng(1)
    for _ in range(30):
        a = "".join(rng.choice(list("ACGT"), size=rng.integers(0, 12)))
        b = "".join(rng.choice(list("ACGT"), size=rng.integers(0, 12)))
        assert P.edit_distance(a, b) == recursive_levenshtein(a, b)
        _, h, _ = P.delta_dp(a, b)
        assert P.distance_from_last_row(len(a), h[len(a), 1:]) == recursive_levenshtein(a, b)


def test_cell_identity_all_18_inputs():
    """Each (dv_in, dh_in, eq) against a Wagner-Fischer step on the 2x2 block
    with corner D[i-1,j-1] = 0 (Eq. mye_eq_2 against Eq. eq_wf)."""
    for dv_in, dh_in, eq in itertools.product((-1, 0, 1), (-1, 0, 1), (0, 1)):
        up = dh_in          # D[i-1, j]
        left = dv_in        # D[i, j-1]
        d = min(0 + (1 - eq), up + 1, left + 1)
        assert P.cell(eq, dv_in, dh_in) == (d - up, d - left)
        # and the two forms printed before the rewrite (Section 2.3)
        assert d - up == min(1, dv_in + 1 - dh_in, 1 - eq - dh_in)
        assert d - left == min(1, 1 + dh_in - dv_in, 1 - eq - dv_in)


def test_table2_lutmin():
    g = golden("table2_lutmin.json")
    lut = P.lut_min_plain()
    assert [P.negacyclic_read(lut, x, 16) for x in range(32)] == g["outputs"]


def test_lut_min_negated_key():
    """The key of Eq. (eq_keyeq2) that Algorithms 1 and 4 use: the table is
    derived by enumeration; it starts and ends with zeros so that keys 16 and
    17 fold onto -f(0) and -f(1) (Section 3.1)."""
    lut = P.lut_min_negated()
    assert lut == [0, 0, 0, 1, 1, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0]
    for dv, dh, eq in itertools.product((-1, 0, 1), (-1, 0, 1), (0, 1)):
        x = P.key_negated(dv, dh, eq)
        assert P.negacyclic_read(lut, x) == P.cell_M(eq, dv, dh) % 32
    # the plain-key table is the same function under the reflected dv index
    plain = P.lut_min_plain()
    for dv, dh, eq in itertools.product((-1, 0, 1), (-1, 0, 1), (0, 1)):
        assert P.negacyclic_read(plain, P.key_plain(dv, dh, eq)) == P.negacyclic_read(lut, P.key_negated(dv, dh, eq))


def test_table1_x_minus_4():
    g = golden("table1_lut_x_minus_4.json")
    assert [P.negacyclic_read(P.LUT_X_MINUS_4, x, 16) for x in range(32)] == g["outputs"]


def test_lut_eq_and_eq9_over_all_differences():
    """Eqs. (eq_eqlut), (eq_eqlut9): a difference z in [-15, 15] reads 1 (or
    9) exactly at z = 0 thanks to the negacyclic extension."""
    for z in range(-15, 16):
        assert P.negacyclic_read(P.LUT_EQ, z) == (1 if z == 0 else 0)
        assert P.negacyclic_read(P.LUT_EQ9, z) == (9 if z == 0 else 0)


def test_refresh_lut_identity_on_differences():
    """Section 3.1's refresh of a difference: -1, 0 and 1 read themselves."""
    for z in (-1, 0, 1):
        assert P.negacyclic_read(P.LUT_REFRESH, z) == z % 32


def test_algorithm3_plaintext_all_ascii_pairs():
    """Algorithm 3/4 equality in the clear over all 128 x 128 characters."""
    for x in range(128):
        x1, x2 = P.ascii_symbols(x)
        for y in range(128):
            y1, y2 = P.ascii_symbols(y)
            eq1 = P.negacyclic_read(P.LUT_EQ, x1 - y1)
            z2 = 2 * (x2 - y2) + (1 - eq1)
            assert -15 <= z2 <= 15
            assert P.negacyclic_read(P.LUT_EQ9, z2) == (9 if x == y else 0)


def test_key_range_fits_lookup():
    """key = (1 - dv) + 3 (1 + dh) + eq9 spans 0..17 (18 values, Section 3.1)."""
    keys = {P.key_negated(dv, dh, eq) for dv, dh, eq in itertools.product((-1, 0, 1), (-1, 0, 1), (0, 1))}
    assert keys == set(range(18))


def test_counts_fixture_consistency():
    g = golden("counts.json")
    assert g["exact_total_per_cell_ascii"] == g["equality_pbs_ascii"] + g["pbs_per_cell"]


# ---------------------------------------------------------------- band modes

def _random_pairs(seed, count, max_len, alphabets=("ab", "abcd", "ACGT")):
    rng = np.random.default_rng(seed)
    for t in range(count):
        alpha = alphabets[t % len(alphabets)]
        m, n = (int(x) for x in rng.integers(0, max_len + 1, size=2))
        a = "".join(alpha[k] for k in rng.integers(0, len(alpha), size=m))
        b = "".join(alpha[k] for k in rng.integers(0, len(alpha), size=n))
        yield a, b


def test_band_cell_count_eq_skip():
    """Eq. (eq_skip): cells with |i - j| <= ell of an m x m matrix, by brute
    force, for every ell < m up to m = 40."""
    for m in range(1, 41):
        for ell in range(0, m):
            count = sum(1 for i in range(1, m + 1) for j in range(1, m + 1) if P.band_contains(i, j, ell))
            assert count == P.band_cell_count_formula(m, ell), (m, ell)


def test_band_path_sums_wf_differences():
    """The diagonal path of Section 3.2 telescopes: the WF matrix's own
    differences along it sum to D[m, n] (independent of the banded loop)."""
    for a, b in _random_pairs(21, 300, 12):
        D = P.wagner_fischer(a, b)
        dv, dh = P.deltas_from_matrix(D)
        path = P.band_path(len(a), len(b))
        assert len(path) == len(a) + len(b)
        assert sum((dv if k == "v" else dh)[i, j] for k, i, j in path) == D[len(a), len(b)]


def test_exact_band_equals_wf():
    """Section 3.2: with ell = ceil(max(m, n) / 2) (m = n) the banded result is
    the exact distance; for m != n with ell = max(m, n) - floor(min / 2)."""
    for a, b in _random_pairs(22, 1500, 14):
        assert P.band_distance(a, b, P.exact_band(len(a), len(b))) == P.edit_distance(a, b), (a, b)
    assert P.exact_band(8, 8) == 4 and P.exact_band(7, 7) == 4 and P.exact_band(1, 5) == 5


def test_approximate_band_bounds():
    """m = n: the band of half-width w never returns less than the distance,
    and returns it exactly whenever D <= 2w + 1 (an optimal path with cost D
    stays within floor(D / 2) of the diagonal, Section 3.2)."""
    seen_over = 0
    for a, b in _random_pairs(23, 1500, 12):
        if len(a) != len(b):
            continue
        D = P.edit_distance(a, b)
        for w in range(0, len(a) + 1):
            r = P.band_distance(a, b, w)
            assert r >= D, (a, b, w)
            if D <= 2 * w + 1:
                assert r == D, (a, b, w)
            seen_over += r > D
    assert seen_over > 0        # the bound is not vacuous: small bands do overestimate


def test_full_band_equals_delta_dp():
    """A band covering the whole matrix computes every cell of Algorithm 1."""
    for a, b in _random_pairs(24, 200, 9):
        v, h = P.delta_dp_band(a, b, max(len(a), len(b)))
        v2, h2, _ = P.delta_dp(a, b)
        assert (v == v2).all() and (h == h2).all()


def test_equality_method_counts_section4():
    """Section 4's counts: an ASCII check costs 2 bootstraps with the
    Section 4.3 method, 5 with 2-bit chunks and 3 with 4-bit chunks merged;
    the Section 4.3 method is the cheapest up to 16-bit symbols and the
    hybrid beyond (Fig. fig_eq); the hybrid roughly halves the 2-bit cost."""
    assert (P.pbs_chain(7), P.pbs_two_bit(7), P.pbs_hybrid(7)) == (2, 5, 3)
    for w in range(5, 17):
        assert P.pbs_chain(w) <= P.pbs_hybrid(w) and P.pbs_chain(w) <= P.pbs_two_bit(w), w
    for w in range(17, 65):
        assert P.pbs_hybrid(w) <= P.pbs_chain(w), w
    assert all(P.pbs_hybrid(w) < P.pbs_chain(w) for w in range(26, 65))
    for w in range(8, 65):
        assert 3 * P.pbs_hybrid(w) <= 2 * P.pbs_two_bit(w), w
        assert w < 32 or P.pbs_hybrid(w) <= 0.55 * P.pbs_two_bit(w), w
    # the merge of c sub-equalities: groups of at most 15, level by level
    assert P.merge_levels(1) == [] and P.merge_levels(15) == [1]
    assert P.merge_levels(16) == [2, 1] and P.merge_levels(226) == [16, 2, 1]


def test_hybrid_equality_exhaustive_small_widths():
    """Every pair of symbols up to 8 bits: the hybrid returns 9 exactly on
    equal symbols."""
    for w in range(1, 9):
        for x in range(2 ** w):
            for y in range(2 ** w):
                assert P.hybrid_equal_plain(x, y, w) == (9 if x == y else 0), (w, x, y)


def test_hybrid_equality_all_chunk_patterns():
    """Every pattern of equal / unequal chunks for 2, 15, 16 and 17 chunks,
    and random patterns over 226 chunks (three merging levels): equal only
    when every chunk is."""
    rng = np.random.default_rng(41)
    for c in (2, 15, 16, 17):
        w = 4 * c
        for pattern in range(2 ** c):
            x = int(rng.integers(0, 2 ** 62)) % (2 ** w) if w <= 62 else \
                sum(int(rng.integers(0, 16)) << (4 * k) for k in range(c))
            y = x
            for k in range(c):
                if pattern >> k & 1:
                    y ^= (1 + int(rng.integers(0, 15))) << (4 * k)
            assert P.hybrid_equal_plain(x, y, w) == (9 if pattern == 0 else 0), (c, pattern)
    for _ in range(200):
        x = sum(int(rng.integers(0, 16)) << (4 * k) for k in range(226))
        k = int(rng.integers(0, 226))
        y = x ^ ((1 + int(rng.integers(0, 15))) << (4 * k)) if rng.random() < 0.7 else x
        assert P.hybrid_equal_plain(x, y, 904) == (9 if x == y else 0)
