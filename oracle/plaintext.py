"""Oracle, plaintext layer -- TEST INFRASTRUCTURE ONLY.

The cleartext definitions that the encrypted method must reproduce exactly
(arXiv 2508.14568):
  * Wagner-Fischer distance matrix, Eq. (eq_wf) in Section 2.3.
  * Difference encoding of the distance matrix, Eq. (eq:delta) (Myers).
  * The shared non-linearity M = 1 + min(-eq, dv_in, dh_in) with
    dv_out = M - dh_in and dh_out = M - dv_in, Eq. (mye_eq_2), Section 3.1.
  * The single-lookup cell tables: the key (dv+1) + 3(1+dh) + 9eq of
    Eq. (eq_keyeq) with Table LUTmin, and the noise-reduced key
    (1-dv) + 3(1+dh) + 9eq of Eq. (eq_keyeq2) that Algorithms 1 and 4 use.
  * Equality tables LUT_eq and LUT_eq9, Eqs. (eq_eqlut) and (eq_eqlut9).
  * The 7-bit character split into a 4-bit and a 3-bit symbol (Section 4.3).
  * Skipping irrelevant cells (Section 3.2, Algorithm 1's band |i - j| <= ell)
    with the result summed along the diagonal.
  * Equality of wide symbols (Section 4.2, the hybrid of the 4-bit
    subtraction check with Algorithm 2's merging) and the bootstrap counts
    of the three equality methods the section compares.
"""
import itertools

import numpy as np


def wagner_fischer(a, b) -> np.ndarray:
    """Full (m+1) x (n+1) distance matrix: D[i,0] = i, D[0,j] = j and
    D[i,j] = D[i-1,j-1] if a_i = b_j else 1 + min of the three neighbours."""
    m, n = len(a), len(b)
    D = np.zeros((m + 1, n + 1), dtype=np.int64)
    D[:, 0] = np.arange(m + 1)
    D[0, :] = np.arange(n + 1)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            if a[i - 1] == b[j - 1]:
                D[i, j] = D[i - 1, j - 1]
            else:
                D[i, j] = 1 + min(D[i - 1, j], D[i, j - 1], D[i - 1, j - 1])
    return D


def edit_distance(a, b) -> int:
    return int(wagner_fischer(a, b)[len(a), len(b)])


def deltas_from_matrix(D: np.ndarray):
    """dv[i,j] = D[i,j] - D[i-1,j] (i >= 1) and dh[i,j] = D[i,j] - D[i,j-1]
    (j >= 1); entries that the definition does not cover are left at 0."""
    dv = np.zeros_like(D)
    dh = np.zeros_like(D)
    dv[1:, :] = D[1:, :] - D[:-1, :]
    dh[:, 1:] = D[:, 1:] - D[:, :-1]
    return dv, dh


def cell_M(eq: int, dv_in: int, dh_in: int) -> int:
    """M = 1 + min(-eq, dv_in, dh_in), Eq. (mye_eq_2)."""
    return 1 + min(-eq, dv_in, dh_in)


def cell(eq: int, dv_in: int, dh_in: int):
    """(dv_out, dh_out) of one cell through the shared non-linearity."""
    M = cell_M(eq, dv_in, dh_in)
    return M - dh_in, M - dv_in


def delta_dp(a, b):
    """The difference-encoded dynamic programme with boundary v[i,0] = 1 and
    h[0,j] = 1 (Algorithms 1/4 set-up); returns (v, h, M) as (m+1)x(n+1)
    integer arrays in the loop order of the algorithms (j outer, i inner)."""
    m, n = len(a), len(b)
    v = np.ones((m + 1, n + 1), dtype=np.int64)
    h = np.ones((m + 1, n + 1), dtype=np.int64)
    M = np.zeros((m + 1, n + 1), dtype=np.int64)
    for j in range(1, n + 1):
        for i in range(1, m + 1):
            eq = 1 if a[i - 1] == b[j - 1] else 0
            M[i, j] = cell_M(eq, v[i, j - 1], h[i - 1, j])
            v[i, j] = M[i, j] - h[i - 1, j]
            h[i, j] = M[i, j] - v[i, j - 1]
    return v, h, M


def band_contains(i: int, j: int, ell: int) -> bool:
    """Algorithm 1 computes cell (i, j) only when |i - j| <= ell (Section 3.2,
    skipping irrelevant cells; Algorithm 4 prints '<', Algorithm 1 and the
    cell count of Eq. (eq_skip) use '<=')."""
    return abs(i - j) <= ell


def band_cell_count_formula(m: int, ell: int) -> int:
    """Eq. (eq_skip), m = n and ell < m: m (2 ell + 1) - ell^2 - ell."""
    return m * (2 * ell + 1) - ell * ell - ell


def exact_band(m: int, n: int) -> int:
    """Band half-width whose result is the exact distance.  Section 3.2 gives
    ceil(max(m, n) / 2) for m = n; for m != n the band must also reach the
    corner (m, n), and max(m, n) - floor(min(m, n) / 2) covers every cell of
    an optimal path (equal to ceil(m / 2) when m = n)."""
    return max(m, n) - min(m, n) // 2


def delta_dp_band(a, b, ell: int):
    """Algorithm 1's loop (j outer, i inner) over the cells with |i - j| <= ell;
    the differences of cells never computed keep the OneMatrix value 1.
    Returns (v, h) as (m+1) x (n+1) integer arrays."""
    m, n = len(a), len(b)
    v = np.ones((m + 1, n + 1), dtype=np.int64)
    h = np.ones((m + 1, n + 1), dtype=np.int64)
    for j in range(1, n + 1):
        for i in range(1, m + 1):
            if band_contains(i, j, ell):
                eq = 1 if a[i - 1] == b[j - 1] else 0
                M = cell_M(eq, v[i, j - 1], h[i - 1, j])
                v[i, j], h[i, j] = M - h[i - 1, j], M - v[i, j - 1]
    return v, h


def band_path(m: int, n: int):
    """The differences whose sum is the banded result (Section 3.2: the
    final row is no longer available, so the score is summed along the
    diagonal): D[k,k] - D[k-1,k-1] = v[k,k-1] + h[k,k] for k = 1..min(m, n),
    then the rest of the last row (h[m,j], j > m) or column (v[i,n], i > n).
    Entries are ('v' | 'h', i, j); there are m + n of them."""
    out = []
    for k in range(1, min(m, n) + 1):
        out += [("v", k, k - 1), ("h", k, k)]
    out += [("h", m, j) for j in range(m + 1, n + 1)]
    out += [("v", i, n) for i in range(n + 1, m + 1)]
    return out


def band_distance(a, b, ell: int) -> int:
    """Sum of the band path's differences after the banded loop."""
    v, h = delta_dp_band(a, b, ell)
    return int(sum((v if kind == "v" else h)[i, j] for kind, i, j in band_path(len(a), len(b))))


def distance_from_last_row(m: int, h_last) -> int:
    """D[m,n] = D[m,0] + sum_j dh[m,j] = m + sum_{j=1..n} h[m,j]."""
    return int(m + sum(int(x) for x in h_last))


# --------------------------------------------------------------- tables

def lut_from_function(f, key_of):
    """Build the 16-entry table of a function f over all inputs (dv, dh, eq)
    keyed by key_of(dv, dh, eq) in [0, 18).  Keys 16 and 17 land on the
    negated entries 0 and 1 (Section 2.2), so both must be 0 there; the
    assertion enforces it."""
    table = {}
    for dv, dh, eq in itertools.product((-1, 0, 1), (-1, 0, 1), (0, 1)):
        k = key_of(dv, dh, eq)
        val = f(eq, dv, dh)
        assert table.get(k, val) == val, "key collision with different values"
        table[k] = val
    assert set(table) == set(range(18))
    lut = [table[x] for x in range(16)]
    for x in (16, 17):
        assert (-lut[x - 16]) % 32 == table[x] % 32, "negacyclic extension violated"
    return lut


def key_plain(dv, dh, eq):
    """Eq. (eq_keyeq): (dv + 1) + 3 (1 + dh) + 9 eq."""
    return (dv + 1) + 3 * (1 + dh) + 9 * eq


def key_negated(dv, dh, eq):
    """Eq. (eq_keyeq2): (1 - dv) + 3 (1 + dh) + 9 eq."""
    return (1 - dv) + 3 * (1 + dh) + 9 * eq


def lut_min_plain():
    """Table LUTmin of Section 3.1 (key of Eq. eq_keyeq)."""
    return lut_from_function(cell_M, key_plain)


def lut_min_negated():
    """Table for the key of Eq. (eq_keyeq2), which Algorithms 1 and 4 use; the
    paper states that the table changes but does not print it."""
    return lut_from_function(cell_M, key_negated)


LUT_EQ = [1] + [0] * 15          # Eq. (eq_eqlut)
LUT_EQ9 = [9] + [0] * 15         # Eq. (eq_eqlut9)
LUT_X_MINUS_4 = [(x - 4) % 16 for x in range(16)]   # Table table_lutrelu
# Refresh of a difference (Section 3.1: the differences are bootstrapped
# again before their noise reaches the threshold, Fig. noise5): the identity
# on {-1, 0, 1}.  In the negacyclic layout an input of -1 (= 31) reads
# -f(15), so f(15) = 1.
LUT_REFRESH = [0, 1] + [0] * 13 + [1]


def negacyclic_read(lut16, x: int, modulus: int = 32) -> int:
    """Value a bootstrap returns for plaintext x in Z_32 (Section 2.2): the
    entry itself below 16, its negation for 16 <= x < 32."""
    x %= 32
    return lut16[x] % modulus if x < 16 else (-lut16[x - 16]) % modulus


# ------------------------------------------------------------- symbols

def ascii_symbols(c: int):
    """7-bit character -> (4-bit symbol, 3-bit symbol) = (c & 15, c >> 4)."""
    assert 0 <= c < 128
    return c & 15, c >> 4


def dna_code(base) -> int:
    return "ACGT".index(base) if isinstance(base, str) else int(base)


# ------------------------------------------------- wide symbols (Section 4.2)

# Merging (Algorithm 2): the sub-equalities are summed in groups of at most
# t - 1 = 15 (a lookup reads 16 values), and a bootstrap tests whether a
# group's sum reached the group size.  Here a group of g is offset by 15 - g
# so that one table serves every group size: the sum reads 15 exactly when
# all g sub-equalities are 1.
MERGE_GROUP = 15
LUT_MAX = [0] * 15 + [1]
LUT_MAX9 = [0] * 15 + [9]


def wide_chunk_count(width: int) -> int:
    """4-bit chunks of a width-bit symbol (the hybrid encoding, Section 4.2)."""
    assert width >= 1
    return (width + 3) // 4


def wide_chunks(v: int, width: int):
    """Chunk k holds bits 4k .. 4k + 3 of v (the last chunk may be narrower)."""
    assert 0 <= v < 2 ** width
    return [(v >> (4 * k)) & 15 for k in range(wide_chunk_count(width))]


def merge_levels(count: int):
    """Group counts of the successive merging levels for `count`
    sub-equalities (empty for one: its own bootstrap gives the result)."""
    levels = []
    while count > 1:
        count = (count + MERGE_GROUP - 1) // MERGE_GROUP
        levels.append(count)
    return levels


def hybrid_equal_plain(x: int, y: int, width: int) -> int:
    """The hybrid equality in the clear: sub-equality of every chunk pair
    (z = x_k - y_k read through LUT_eq), then the merging levels (a group of
    g reads LUT_max at sum + 15 - g; the last level reads LUT_max9).  Returns
    the final bootstrap's value, 9 [x = y]."""
    cx, cy = wide_chunks(x, width), wide_chunks(y, width)
    if len(cx) == 1:
        return negacyclic_read(LUT_EQ9, cx[0] - cy[0])
    sub = [negacyclic_read(LUT_EQ, a - b) for a, b in zip(cx, cy)]
    while len(sub) > 1:
        groups = [sub[k:k + MERGE_GROUP] for k in range(0, len(sub), MERGE_GROUP)]
        lut = LUT_MAX9 if len(groups) == 1 else LUT_MAX
        sub = [negacyclic_read(lut, sum(g) + MERGE_GROUP - len(g)) for g in groups]
    return sub[0]


def pbs_hybrid(width: int) -> int:
    """Bootstraps of the hybrid equality: one per 4-bit chunk plus the merges."""
    c = wide_chunk_count(width)
    return c + sum(merge_levels(c))


def pbs_two_bit(width: int) -> int:
    """Bootstraps of Algorithm 2 as TFHE-rs runs it: one per 2-bit chunk
    (key x + 4 y) plus the same merges."""
    c = (width + 1) // 2
    return c + sum(merge_levels(c))


def pbs_chain(width: int) -> int:
    """Bootstraps of the Section 4.3 method extended to any width: a 4-bit
    symbol, then 3-bit symbols, each folded with the previous result as in
    Algorithm 3 (2 (x - y) + (1 - eq) stays within [-15, 15])."""
    return 1 + (max(0, width - 4) + 2) // 3
