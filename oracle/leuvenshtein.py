"""Oracle, encrypted Leuvenshtein -- TEST INFRASTRUCTURE ONLY.

The encrypted algorithm of arXiv 2508.14568 written out step by step on top
of the schoolbook TFHE oracle (``tfhe.py``):
  * Algorithm 3 / Algorithm 4 equality: z1 = x1 - y1, eq1 = PBS(z1; LUT_eq),
    z2 = 2 (x2 - y2) + (1 - eq1), eq9 = PBS(z2; LUT_eq9) for 7-bit characters
    split into a 4-bit and a 3-bit symbol (Section 4.3); one PBS on x - y for
    2-bit DNA bases (Section 6.3 uses a single equality PBS for DNA).
  * Algorithm 4 main loop (j outer, i inner): key = (1 - v[i,j-1]) +
    3 (1 + h[i-1,j]) + eq9[i,j] (Eq. eq_keyeq2), M = PBS(key; LUT_min),
    v[i,j] = M - h[i-1,j], h[i,j] = M - v[i,j-1], boundary v[i,0] = h[0,j] = 1.
  * Result: D = m + sum_j h[m,j] (the return of Algorithm 4 with the boundary
    term h[m,0] left out; Fig. fig_myers shows the bold bottom-row arrows
    summing to the distance).
  * Section 5 preprocessing: T[c][i] = Enc(9 [a_i = c]) for c in an alphabet
    S; the main loop then reads eq9[i,j] = T[b_j][i] with no bootstrap.
  * Section 6.2 (parallelism over cells): cells on one anti-diagonal are
    independent; ``dp(..., order="diagonal")`` evaluates them as one batch.
  * Section 3.2 / Algorithm 1 band: only cells with |i - j| <= ell are
    bootstrapped (and only their equality pairs); the result is the sum of
    the differences along the diagonal path (``dp_band``).
  * Section 3.1 noise refresh: the differences written on every R-th
    anti-diagonal are bootstrapped again through the identity table
    (``refresh_every``), which restarts their noise growth.
  * Section 4.2 equality of wide symbols (the hybrid method): a symbol of
    w bits is encrypted as ceil(w / 4) 4-bit chunks; every chunk pair gives
    a sub-equality PBS(x_k - y_k; LUT_eq), and Algorithm 2's merging sums
    groups of at most 15 and bootstraps each sum (``equality_wide``).
"""
import numpy as np

from . import plaintext as P
from . import tfhe as T

ENC_ASCII7 = 0
ENC_DNA2 = 1

LUT_IDS = {"eq": 0, "eq9": 1, "min": 2, "refresh": 3, "max": 4, "max9": 5}


def lut_polys(N: int) -> np.ndarray:
    """Test polynomials in the order of LUT_IDS."""
    return np.stack([T.test_polynomial(P.LUT_EQ, N), T.test_polynomial(P.LUT_EQ9, N),
                     T.test_polynomial(P.lut_min_negated(), N), T.test_polynomial(P.LUT_REFRESH, N),
                     T.test_polynomial(P.LUT_MAX, N), T.test_polynomial(P.LUT_MAX9, N)])


def refresh_due(s: int, m: int, n: int, refresh_every: int) -> bool:
    """Whether the differences written on anti-diagonal s are bootstrapped
    again before diagonal s + 1 reads them (every refresh_every-th diagonal;
    0: never).  Reading of Section 3.1's refresh: every chain of differences
    passes through each anti-diagonal, so refreshing the outputs of one
    diagonal restarts the noise growth of all of them."""
    return refresh_every > 0 and s % refresh_every == 0 and s < m + n


def symbols(s, encoding):
    """Per-character symbol lists: ASCII -> (c & 15, c >> 4); DNA -> (code,)."""
    if encoding == ENC_ASCII7:
        return [P.ascii_symbols(c) for c in s]
    return [(P.dna_code(c),) for c in s]


def encrypt_string(keys: T.Keys, s, encoding: int, seed: int) -> np.ndarray:
    """Array (m, nsym, N+1): symbol r of character i is ciphertext number
    i * nsym + r under the encryption seed."""
    syms = symbols(s, encoding)
    nsym = 2 if encoding == ENC_ASCII7 else 1
    out = np.zeros((len(syms), nsym, keys.N + 1), dtype=T.U64)
    for i, sy in enumerate(syms):
        for r in range(nsym):
            out[i, r] = keys.encrypt(sy[r], seed, i * nsym + r)
    return out


def encrypt_symbols(keys: T.Keys, syms, width: int, seed: int) -> np.ndarray:
    """Array (len, c, N+1) of wide symbols, c = ceil(width / 4): chunk k of
    symbol i is ciphertext number i * c + k under the encryption seed."""
    c = P.wide_chunk_count(width)
    out = np.zeros((len(syms), c, keys.N + 1), dtype=T.U64)
    for i, v in enumerate(syms):
        for k, x in enumerate(P.wide_chunks(int(v), width)):
            out[i, k] = keys.encrypt(x, seed, i * c + k)
    return out


def _pbs(keys, cts, lut_name, nthreads):
    polys = lut_polys(keys.N)
    return keys.pbs_batch(cts, polys, LUT_IDS[lut_name], nthreads)


def equality(keys: T.Keys, A: np.ndarray, B: np.ndarray, encoding: int, nthreads=None):
    """eq9[i,j] for every pair (all m*n pairs are independent of the DP).
    Returns (eq1, eq9) with eq1 None for DNA; arrays are (m, n, N+1)."""
    m, n, W = A.shape[0], B.shape[0], keys.N + 1
    if encoding == ENC_DNA2:
        z = (A[:, None, 0, :] - B[None, :, 0, :]).astype(T.U64).reshape(m * n, W)
        return None, _pbs(keys, z, "eq9", nthreads).reshape(m, n, W)
    z1 = (A[:, None, 0, :] - B[None, :, 0, :]).astype(T.U64).reshape(m * n, W)
    eq1 = _pbs(keys, z1, "eq", nthreads)
    one = T.trivial(1, keys.N)
    z2 = (T.scale(A[:, None, 1, :], 2) - T.scale(B[None, :, 1, :], 2)).reshape(m * n, W)
    z2 = (z2 + one[None, :] - eq1).astype(T.U64)
    eq9 = _pbs(keys, z2, "eq9", nthreads)
    return eq1.reshape(m, n, W), eq9.reshape(m, n, W)


def merge_wide(keys: T.Keys, sub: np.ndarray, nthreads=None) -> np.ndarray:
    """Algorithm 2's merging over the last axis but one of sub (..., c, N+1)
    holding encryptions of 0/1: groups of at most 15 are summed, offset by
    15 - g (a noise-free constant) and bootstrapped through LUT_max (LUT_max9
    at the last level), until one ciphertext is left per leading index."""
    lead, W = sub.shape[:-2], sub.shape[-1]
    cur = sub.reshape(-1, sub.shape[-2], W)
    while cur.shape[1] > 1:
        c = cur.shape[1]
        groups = [(k, min(c, k + P.MERGE_GROUP)) for k in range(0, c, P.MERGE_GROUP)]
        lut = "max9" if len(groups) == 1 else "max"
        sums = np.stack([(cur[:, a:b].sum(axis=1, dtype=T.U64)
                          + T.trivial(P.MERGE_GROUP - (b - a), keys.N)[None, :]).astype(T.U64)
                         for a, b in groups], axis=1)
        cur = _pbs(keys, sums.reshape(-1, W), lut, nthreads).reshape(cur.shape[0], len(groups), W)
    return cur[:, 0].reshape(*lead, W)


def equality_wide(keys: T.Keys, A: np.ndarray, B: np.ndarray, width: int, nthreads=None) -> np.ndarray:
    """eq9[i,j] = Enc(9 [a_i = b_j]) for symbols of `width` bits encrypted
    by encrypt_symbols: one sub-equality PBS per 4-bit chunk pair, then the
    merging (a single chunk reads LUT_eq9 directly).  Shape (m, n, N+1)."""
    m, n, W = A.shape[0], B.shape[0], keys.N + 1
    c = P.wide_chunk_count(width)
    assert A.shape[1] == c and B.shape[1] == c
    z = (A[:, None, :, :] - B[None, :, :, :]).astype(T.U64).reshape(m * n * c, W)
    if c == 1:
        return _pbs(keys, z, "eq9", nthreads).reshape(m, n, W)
    sub = _pbs(keys, z, "eq", nthreads).reshape(m * n, c, W)
    return merge_wide(keys, sub, nthreads).reshape(m, n, W)


def preprocess_wide(keys: T.Keys, A: np.ndarray, alphabet, width: int, nthreads=None) -> np.ndarray:
    """Section 5's table for wide symbols: T[s][i] = Enc(9 [a_i = alphabet[s]])
    by the hybrid equality against the cleartext symbol (a noise-free
    chunk).  Shape (|alphabet|, m, N+1)."""
    m, W = A.shape[0], keys.N + 1
    c = P.wide_chunk_count(width)
    S = len(alphabet)
    clear = np.stack([np.stack([T.trivial(x, keys.N) for x in P.wide_chunks(int(v), width)]) for v in alphabet])
    z = (A[None, :, :, :] - clear[:, None, :, :]).astype(T.U64).reshape(S * m * c, W)
    if c == 1:
        return _pbs(keys, z, "eq9", nthreads).reshape(S, m, W)
    sub = _pbs(keys, z, "eq", nthreads).reshape(S * m, c, W)
    return merge_wide(keys, sub, nthreads).reshape(S, m, W)


def edit_distance_wide(keys: T.Keys, A: np.ndarray, B: np.ndarray, width: int, nthreads=None,
                       refresh_every: int = 0):
    """Wide-symbol equality of every pair, then the diagonal-order main loop."""
    m, n = A.shape[0], B.shape[0]
    if m == 0 or n == 0:
        return np.tile(T.trivial(1, keys.N), (n, 1))
    eq9 = equality_wide(keys, A, B, width, nthreads)
    return dp(keys, m, n, lambda i, j: eq9[i - 1, j - 1], "diagonal", nthreads, False, refresh_every)


def preprocess(keys: T.Keys, A: np.ndarray, alphabet, encoding: int, nthreads=None):
    """Section 5 table T[c][i] = Enc(9 [a_i = alphabet[c]]), shape (|S|, m, N+1):
    the equality pipeline with the cleartext symbol as a noise-free ciphertext."""
    m, W = A.shape[0], keys.N + 1
    Bc = np.stack([np.stack([T.trivial(s, keys.N) for s in sy]) for sy in symbols(alphabet, encoding)])
    _, eq9 = equality(keys, A, Bc, encoding, nthreads)        # (m, |S|, W)
    return np.ascontiguousarray(eq9.transpose(1, 0, 2))


def dp(keys: T.Keys, m: int, n: int, eq9_at, order: str = "alg4", nthreads=None, record: bool = False,
       refresh_every: int = 0):
    """Main loop of Algorithm 4 over an m x n grid; eq9_at(i, j) returns the
    ciphertext of 9 [a_i = b_j] (1-based indices).  Returns the last-row
    vector h[m, 1..n] (n ciphertexts) and, when record is set, a dict with
    every key and M ciphertext.  refresh_every > 0 (diagonal order only)
    bootstraps the v and h written on every refresh_every-th anti-diagonal
    through the identity table (refresh_due)."""
    assert refresh_every == 0 or order == "diagonal"
    N, W = keys.N, keys.N + 1
    polys = lut_polys(N)
    one = T.trivial(1, N)
    four = T.trivial(4, N)
    V = np.tile(one, (m + 1, 1))      # V[i] = v[i, last j]   (v[i,0] = 1)
    H = np.tile(one, (n + 1, 1))      # H[j] = h[last i, j]   (h[0,j] = 1)
    rec = {"key": {}, "M": {}} if record else None

    def key_of(i, j):
        return (four - V[i] + T.scale(H[j], 3) + eq9_at(i, j)).astype(T.U64)

    def update(i, j, M):
        v_new = (M - H[j]).astype(T.U64)
        h_new = (M - V[i]).astype(T.U64)
        V[i], H[j] = v_new, h_new

    if order == "alg4":
        for j in range(1, n + 1):
            for i in range(1, m + 1):
                key = key_of(i, j)
                M = keys.pbs(key, polys[LUT_IDS["min"]])
                if record:
                    rec["key"][(i, j)], rec["M"][(i, j)] = key, M
                update(i, j, M)
    elif order == "diagonal":
        for s in range(2, m + n + 1):
            cells = [(i, s - i) for i in range(max(1, s - n), min(m, s - 1) + 1)]
            keys_b = np.stack([key_of(i, j) for i, j in cells])
            Ms = keys.pbs_batch(keys_b, polys, LUT_IDS["min"], nthreads)
            for (i, j), key, M in zip(cells, keys_b, Ms):
                if record:
                    rec["key"][(i, j)], rec["M"][(i, j)] = key, M
                update(i, j, M)
            if refresh_due(s, m, n, refresh_every):
                fresh = keys.pbs_batch(np.stack([V[i] for i, _ in cells] + [H[j] for _, j in cells]), polys,
                                       LUT_IDS["refresh"], nthreads)
                for k, (i, j) in enumerate(cells):
                    V[i], H[j] = fresh[k], fresh[len(cells) + k]
    else:
        raise ValueError(order)
    h_last = H[1:].copy()
    return (h_last, rec) if record else h_last


def edit_distance(keys: T.Keys, A: np.ndarray, B: np.ndarray, encoding: int, order="diagonal",
                  nthreads=None, record=False, refresh_every: int = 0):
    """Algorithm 4 on two encrypted strings; returns h[m,1..n] (and records)."""
    m, n = A.shape[0], B.shape[0]
    if m == 0 or n == 0:
        h_last = np.tile(T.trivial(1, keys.N), (n, 1))
        return (h_last, {"eq9": None}) if record else h_last
    eq1, eq9 = equality(keys, A, B, encoding, nthreads)
    out = dp(keys, m, n, lambda i, j: eq9[i - 1, j - 1], order, nthreads, record, refresh_every)
    if record:
        out[1]["eq1"], out[1]["eq9"] = eq1, eq9
    return out


def edit_distance_clear(keys: T.Keys, table: np.ndarray, alphabet, b, encoding: int, order="diagonal",
                        nthreads=None, record=False, refresh_every: int = 0):
    """Main loop with eq9[i,j] = T[b_j][i] read from the preprocessing table."""
    m, n = table.shape[1], len(b)
    index = {c: k for k, c in enumerate(alphabet)}
    cols = [index[c] for c in b]
    if m == 0 or n == 0:
        return np.tile(T.trivial(1, keys.N), (n, 1))
    return dp(keys, m, n, lambda i, j: table[cols[j - 1], i - 1], order, nthreads, record, refresh_every)


def dp_band(keys: T.Keys, m: int, n: int, eq9_at, ell: int, nthreads=None, record: bool = False,
            refresh_every: int = 0):
    """Algorithm 1 restricted to the band |i - j| <= ell (Section 3.2), cells
    of one anti-diagonal as one batch; neighbours outside the band keep the
    OneMatrix value (a noise-free 1).  Returns the m + n ciphertexts of the
    band path (plaintext.band_path; v[1,0] is the noise-free boundary 1) and,
    when record is set, every computed (v, h) pair."""
    N = keys.N
    polys = lut_polys(N)
    one = T.trivial(1, N)
    four = T.trivial(4, N)
    v = {}
    h = {}
    path_vals = {}     # (v, h) of a refreshed cell as its bootstrap produced them

    def v_at(i, j):
        return v.get((i, j), one)

    def h_at(i, j):
        return h.get((i, j), one)

    for s in range(2, m + n + 1):
        cells = [(i, s - i) for i in range(max(1, s - n), min(m, s - 1) + 1) if P.band_contains(i, s - i, ell)]
        if not cells:
            continue
        keys_b = np.stack([(four - v_at(i, j - 1) + T.scale(h_at(i - 1, j), 3) + eq9_at(i, j)).astype(T.U64)
                           for i, j in cells])
        Ms = keys.pbs_batch(keys_b, polys, LUT_IDS["min"], nthreads)
        fresh_path = {}
        for (i, j), M in zip(cells, Ms):
            v[(i, j)] = (M - h_at(i - 1, j)).astype(T.U64)
            h[(i, j)] = (M - v_at(i, j - 1)).astype(T.U64)
        if refresh_due(s, m, n, refresh_every):
            # the path keeps the values as computed; the state is refreshed
            for i, j in cells:
                fresh_path[(i, j)] = (v[(i, j)], h[(i, j)])
            fresh = keys.pbs_batch(np.stack([v[c] for c in cells] + [h[c] for c in cells]), polys,
                                   LUT_IDS["refresh"], nthreads)
            for k, c in enumerate(cells):
                v[c], h[c] = fresh[k], fresh[len(cells) + k]
            path_vals.update(fresh_path)
    def path_at(kind, i, j):
        if (i, j) in path_vals:
            return path_vals[(i, j)][0 if kind == "v" else 1]
        return v_at(i, j) if kind == "v" else h_at(i, j)

    path = np.stack([path_at(kind, i, j) for kind, i, j in P.band_path(m, n)]) \
        if m + n else np.zeros((0, N + 1), dtype=T.U64)
    return (path, {"v": v, "h": h}) if record else path


def edit_distance_band(keys: T.Keys, A: np.ndarray, B: np.ndarray, encoding: int, ell: int, nthreads=None,
                       record=False, refresh_every: int = 0):
    """Equality for the pairs inside the band only, then the banded loop;
    returns the band path (and records)."""
    m, n, W = A.shape[0], B.shape[0], keys.N + 1
    cells = [(i, j) for i in range(1, m + 1) for j in range(1, n + 1) if P.band_contains(i, j, ell)]
    eq9 = {}
    if cells:
        Ai = np.stack([A[i - 1] for i, _ in cells])
        Bj = np.stack([B[j - 1] for _, j in cells])
        # equality() over aligned pairs: a (k x 1) grid per cell, batched
        if encoding == ENC_DNA2:
            z = (Ai[:, 0, :] - Bj[:, 0, :]).astype(T.U64)
            e9 = _pbs(keys, z, "eq9", nthreads)
        else:
            z1 = (Ai[:, 0, :] - Bj[:, 0, :]).astype(T.U64)
            e1 = _pbs(keys, z1, "eq", nthreads)
            z2 = (T.scale(Ai[:, 1, :], 2) - T.scale(Bj[:, 1, :], 2) + T.trivial(1, keys.N)[None, :] - e1)
            e9 = _pbs(keys, z2.astype(T.U64), "eq9", nthreads)
        eq9 = {c: e9[k] for k, c in enumerate(cells)}
    return dp_band(keys, m, n, lambda i, j: eq9[(i, j)], ell, nthreads, record, refresh_every)


def edit_distance_clear_band(keys: T.Keys, table: np.ndarray, alphabet, b, ell: int, nthreads=None, record=False,
                             refresh_every: int = 0):
    """Banded loop with eq9[i,j] = T[b_j][i] from the preprocessing table."""
    m, n = table.shape[1], len(b)
    index = {c: k for k, c in enumerate(alphabet)}
    cols = [index[c] for c in b]
    return dp_band(keys, m, n, lambda i, j: table[cols[j - 1], i - 1], ell, nthreads, record, refresh_every)


def decrypt_path(keys: T.Keys, path: np.ndarray) -> int:
    """Sum of the decrypted differences of a band path."""
    return int(sum(keys.decrypt_signed(ct) for ct in path))


def decrypt_distance(keys: T.Keys, m: int, h_last: np.ndarray) -> int:
    """D = m + sum_j dec(h[m,j]) with dec in {-1, 0, 1}; the sum is taken in
    the clear since D can exceed the 5-bit plaintext space."""
    return P.distance_from_last_row(m, [keys.decrypt_signed(ct) for ct in h_last])
