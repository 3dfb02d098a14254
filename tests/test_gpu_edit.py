"""GPU edit distance through the C ABI against the oracle (Algorithms 1, 3, 4
and the Section 5 preprocessing of arXiv 2508.14568).

Bar: every compared ciphertext bit-exact, every decrypted distance equal to
Wagner-Fischer.  Small cases are checked in full against a live oracle run;
the 32 x 32 ASCII pair and the 256 x 256 DNA pair (every ciphertext) against
oracle digests written by tests/golden/make_oracle_vectors.py, the former
also with live sampled checks."""
import hashlib
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN, oracle_vectors
from gpu_common import KEY_SEED, assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu

SEED_A, SEED_B = 1001, 1002


def digest(ct):
    return hashlib.sha256(np.ascontiguousarray(ct, dtype=np.uint64).tobytes()).hexdigest()


def gpu_run(g, sa, sb, enc, trace=True):
    """Equality matrix, M trace and bottom row from the GPU."""
    L, torch = g.L, g.torch
    m, n = len(sa), len(sb)
    A = L.lvs_encrypt_string(g.ck, sa, enc, SEED_A)
    B = L.lvs_encrypt_string(g.ck, sb, enc, SEED_B)
    dA, dB = L.to_device(A, g.dev), L.to_device(B, g.dev)
    d_eq9 = torch.zeros(max(1, m * n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    d_tr = torch.zeros_like(d_eq9) if trace else None
    d_h = torch.zeros(max(1, n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_equality(g.ctx, dA, m, dB, n, enc, d_eq9)
    L.lvs_edit_distance_eq9(g.ctx, d_eq9, m, n, d_h, d_trace=d_tr)
    torch.cuda.synchronize()
    eq9 = L.to_host(d_eq9)[:m * n * L.CT_WORDS].reshape(m, n, L.CT_WORDS)
    tr = L.to_host(d_tr)[:m * n * L.CT_WORDS].reshape(m, n, L.CT_WORDS) if trace else None
    h = L.to_host(d_h)[:n * L.CT_WORDS].reshape(n, L.CT_WORDS)
    return A, B, eq9, tr, h


def gpu_one_shot(g, A, m, B, n, enc):
    L, torch = g.L, g.torch
    d_h = torch.zeros(max(1, n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev) if m else None, m, L.to_device(B, g.dev) if n else None,
                        n, enc, d_h)
    torch.cuda.synchronize()
    return L.to_host(d_h)[:n * L.CT_WORDS].reshape(n, L.CT_WORDS)


def check_full(g, okeys, a, b, enc, sa, sb):
    """Every eq9, every M and the bottom row against a live oracle run."""
    A, B, eq9, tr, h = gpu_run(g, sa, sb, enc)
    m, n = len(a), len(b)
    oA = OL.encrypt_string(okeys, sa, enc, SEED_A)
    oB = OL.encrypt_string(okeys, sb, enc, SEED_B)
    assert (oA == A).all() and (oB == B).all()
    oh, rec = OL.edit_distance(okeys, oA, oB, enc, order="diagonal", record=True)
    for i in range(m):
        for j in range(n):
            assert_same_ct(eq9[i, j], rec["eq9"][i, j], f"eq9[{i},{j}]")
            assert_same_ct(tr[i, j], rec["M"][(i + 1, j + 1)], f"M[{i + 1},{j + 1}]")
    for j in range(n):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert g.L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b)
    # the one-shot entry point gives the same row
    assert (gpu_one_shot(g, A, m, B, n, enc) == h).all()
    return h


def test_tiny_dna_full(gpu, okeys):
    """Tiny DNA workload (2 x 6 bases): all 72 bootstraps bit-exact, and equal
    to the stored oracle digests."""
    say("tiny dna full")
    a, b = W.tiny_dna()
    h = check_full(gpu, okeys, a, b, OL.ENC_DNA2, W.dna_codes(a), W.dna_codes(b))
    meta = json.load(open(os.path.join(GOLDEN, "oracle_tiny_dna.json")))
    assert meta["a"] == a.decode() and meta["b"] == b.decode() and meta["key_seed"] == KEY_SEED
    assert [digest(c) for c in h] == meta["h_last_sha256"]
    assert (np.load(os.path.join(GOLDEN, "oracle_tiny_dna_h_last.npy")) == h).all()


@pytest.mark.parametrize("a,b", [(b"KID", b"SIT"), (b"abc", b"yabcxz"), (b"Q", b"Q"), (b"pq", b"Zz")])
def test_small_ascii_full(gpu, okeys, a, b):
    """ASCII pairs including Fig. fig_myers (KID/SIT) and ragged m != n."""
    say("small ascii", a, b)
    check_full(gpu, okeys, a, b, OL.ENC_ASCII7, a, b)


def test_empty_strings(gpu):
    say("empty strings")
    g = gpu
    L = g.L
    A = L.lvs_encrypt_string(g.ck, b"ACGT", L.LVS_ENC_ASCII7, 1)
    h = gpu_one_shot(g, A, 4, None, 0, L.LVS_ENC_ASCII7)
    assert h.shape[0] == 0 and L.lvs_decrypt_distance(g.ck, h, 4) == 4
    h = gpu_one_shot(g, None, 0, A, 4, L.LVS_ENC_ASCII7)
    assert L.lvs_decrypt_distance(g.ck, h, 0) == 4


def test_plain_ascii_32(gpu, okeys):
    """The 32-character ASCII workload: every eq9 and M against the oracle
    digests, the bottom row element by element against the stored oracle
    row, live oracle checks of sampled equalities and of the first cell."""
    say("plain ascii 32")
    g = gpu
    a, b = W.plain_ascii()
    A, B, eq9, tr, h = gpu_run(g, a, b, OL.ENC_ASCII7)
    meta = json.load(open(os.path.join(GOLDEN, "oracle_plain_ascii.json")))
    assert meta["a"] == a.decode() and meta["b"] == b.decode()
    m, n = len(a), len(b)
    bad_eq = [(i, j) for i in range(m) for j in range(n) if digest(eq9[i, j]) != meta["eq9_sha256"][i][j]]
    bad_m = [(i, j) for i in range(m) for j in range(n) if digest(tr[i, j]) != meta["M_sha256"][i][j]]
    assert not bad_eq and not bad_m, (bad_eq[:5], bad_m[:5])
    ref = np.load(os.path.join(GOLDEN, "oracle_plain_ascii_h_last.npy"))
    for j in range(n):
        assert_same_ct(h[j], ref[j], f"h[m,{j + 1}]")
    assert g.L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b) == meta["distance"]
    # live oracle: sampled equalities (2 bootstraps each) and the first cell
    oA = OL.encrypt_string(okeys, a, OL.ENC_ASCII7, SEED_A)
    oB = OL.encrypt_string(okeys, b, OL.ENC_ASCII7, SEED_B)
    pairs = [(0, 0), (5, 17), (31, 31), (12, 3)]
    for i, j in pairs:
        _, e9 = OL.equality(okeys, oA[i:i + 1], oB[j:j + 1], OL.ENC_ASCII7)
        assert_same_ct(eq9[i, j], e9[0, 0], f"eq9[{i},{j}]")
    _, rec = OL.dp(okeys, 1, 1, lambda i, j: eq9_oracle_00(okeys, oA, oB), order="alg4", record=True)
    assert_same_ct(tr[0, 0], rec["M"][(1, 1)], "M[1,1]")


def eq9_oracle_00(okeys, oA, oB):
    _, e9 = OL.equality(okeys, oA[0:1], oB[0:1], OL.ENC_ASCII7)
    return e9[0, 0]


def row_digest(cells):
    """SHA-256 over the SHA-256 digests of a row's ciphertexts (the form
    tests/golden/make_oracle_vectors.py stores for the full-size workloads)."""
    return hashlib.sha256(b"".join(hashlib.sha256(np.ascontiguousarray(c).tobytes()).digest()
                                   for c in cells)).hexdigest()


def test_dna_256_alignment(gpu):
    """DNA 256 x 256 (5% edits), the context's default refresh (anti-diagonal
    256 bootstrapped again): every one of the 65,536 eq9 and 65,536 M
    ciphertexts and the 256 result ciphertexts bit-exact with the oracle
    (digests written by tests/golden/make_oracle_vectors.py), and the exact
    distance."""
    say("dna 256")
    g = gpu
    a, b = W.dna_align()
    meta = oracle_vectors("dna_align")
    assert meta["a"] == a.decode() and meta["b"] == b.decode() and meta["key_seed"] == KEY_SEED
    assert (meta["seed_a"], meta["seed_b"]) == (SEED_A, SEED_B)
    refresh = g.L.lvs_context_get_refresh(g.ctx)
    assert refresh == meta["refresh_every"], refresh
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    L, torch = g.L, g.torch
    m, n = len(a), len(b)
    # the plain path's own plan (one query: the plan lvs_edit_distance builds,
    # equality inside the wavefront, refresh after anti-diagonal 256) keeping
    # every eq9 and M
    A = L.lvs_encrypt_string(g.ck, sa, L.LVS_ENC_DNA2, SEED_A)
    B = L.lvs_encrypt_string(g.ck, sb, L.LVS_ENC_DNA2, SEED_B)
    d_eq9 = torch.zeros(m * n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    d_tr = torch.zeros_like(d_eq9)
    item = {"d_a": L.to_device(A, g.dev), "m": m, "d_b": L.to_device(B, g.dev), "n": n,
            "d_h_last": torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev), "d_eq9": d_eq9, "d_trace": d_tr}
    plan = L.lvs_plan_create(g.ctx, [item], L.LVS_ENC_DNA2)
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    del plan
    eq9 = L.to_host(d_eq9).reshape(m, n, L.CT_WORDS)
    tr = L.to_host(d_tr).reshape(m, n, L.CT_WORDS)
    h = L.to_host(item["d_h_last"]).reshape(n, L.CT_WORDS)
    assert (gpu_one_shot(g, A, m, B, n, OL.ENC_DNA2) == h).all()      # bench.py's call
    assert g.L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b) == meta["distance"]
    bad_eq = [i for i in range(m) if row_digest(eq9[i]) != meta["eq9_row_sha256"][i]]
    bad_m = [i for i in range(m) if row_digest(tr[i]) != meta["M_row_sha256"][i]]
    bad_h = [j for j in range(n) if digest(h[j]) != meta["h_last_sha256"][j]]
    assert not bad_eq and not bad_m and not bad_h, (bad_eq[:5], bad_m[:5], bad_h[:5])


def test_preprocess_and_clear(gpu, okeys):
    """Section 5: the table T[c][i] and the main pass with a cleartext string,
    bit-exact with the oracle; the distance equals Wagner-Fischer."""
    say("preprocess + clear")
    g = gpu
    L, torch = g.L, g.torch
    a, b = b"kitten", b"sitting"
    alpha = bytes(sorted(set(b)))
    m, n, S = len(a), len(b), len(alpha)
    A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, SEED_A)
    d_tab = torch.zeros(S * m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, L.to_device(A, g.dev), m, L.LVS_ENC_ASCII7, alpha, d_tab)
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_clear(g.ctx, d_tab, m, alpha, b, d_h)
    torch.cuda.synchronize()
    tab = L.to_host(d_tab).reshape(S, m, L.CT_WORDS)
    h = L.to_host(d_h).reshape(n, L.CT_WORDS)
    oA = OL.encrypt_string(okeys, a, OL.ENC_ASCII7, SEED_A)
    otab = OL.preprocess(okeys, oA, alpha, OL.ENC_ASCII7)
    for c in range(S):
        for i in range(m):
            assert_same_ct(tab[c, i], otab[c, i], f"T[{c}][{i}]")
    oh = OL.edit_distance_clear(okeys, otab, alpha, b, OL.ENC_ASCII7)
    for j in range(n):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b) == 3
    with pytest.raises(L.LvsError) as e:
        L.lvs_edit_distance_clear(g.ctx, d_tab, m, alpha, b"xyz", d_h)
    assert e.value.code == -2
