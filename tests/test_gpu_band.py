"""Band modes (Section 3.2, Algorithm 1's |i - j| <= ell): the path
ciphertexts bit-exact with the oracle's banded loop, exact distances with the
exact half-width, the approximate mode equal to the plaintext banded loop,
the cleartext-table variant, and batch plans mixing banded and full queries
bit-identical to their lone runs."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu


def enc(g, s, encoding, seed):
    return g.L.lvs_encrypt_string(g.ck, s, encoding, seed)


def run_band(g, A, m, B, n, encoding, ell):
    L, torch = g.L, g.torch
    d_path = torch.zeros(max(1, m + n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    dA = L.to_device(A, g.dev) if m else None
    dB = L.to_device(B, g.dev) if n else None
    L.lvs_edit_distance_band(g.ctx, dA, m, dB, n, encoding, ell, d_path)
    torch.cuda.synchronize()
    return L.to_host(d_path).reshape(-1, L.CT_WORDS)[:m + n]


def path_distance(g, path):
    return g.L.lvs_decrypt_distance(g.ck, path, 0)


@pytest.mark.parametrize("a,b,enc_,ell", [(b"GATTCA", b"GTTACA", "dna", 1), (b"KID", b"SIT", "ascii", 1),
                                          (b"ACGTAC", b"CGTA", "dna", 2)])
def test_band_path_bit_exact_with_oracle(gpu, okeys, a, b, enc_, ell):
    say("band vs oracle", a, b, ell)
    g = gpu
    e = g.L.LVS_ENC_DNA2 if enc_ == "dna" else g.L.LVS_ENC_ASCII7
    oe = OL.ENC_DNA2 if enc_ == "dna" else OL.ENC_ASCII7
    sa = W.dna_codes(a) if enc_ == "dna" else a
    sb = W.dna_codes(b) if enc_ == "dna" else b
    A, B = enc(g, sa, e, 601), enc(g, sb, e, 602)
    path = run_band(g, A, len(a), B, len(b), e, ell)
    oA = OL.encrypt_string(okeys, sa, oe, 601)
    oB = OL.encrypt_string(okeys, sb, oe, 602)
    ref = OL.edit_distance_band(okeys, oA, oB, oe, ell)
    assert path.shape == ref.shape
    for k in range(len(ref)):
        assert_same_ct(path[k], ref[k], f"path[{k}]")
    assert path_distance(g, path) == P.band_distance(a, b, ell)


def test_exact_and_approximate_distances(gpu):
    """32 x 32 ASCII (the plain workload) with the exact band, half-widths 2
    and 5, and ragged pairs with the exact band."""
    g = gpu
    L = g.L
    a, b = W.plain_ascii()
    A, B = enc(g, a, L.LVS_ENC_ASCII7, 611), enc(g, b, L.LVS_ENC_ASCII7, 612)
    D = P.edit_distance(a, b)
    ex = L.lvs_band_exact(32, 32)
    assert ex == 16
    for ell in (ex, 5, 2):
        say("plain ascii band", ell)
        path = run_band(g, A, 32, B, 32, L.LVS_ENC_ASCII7, ell)
        got = path_distance(g, path)
        assert got == P.band_distance(a, b, ell)
        assert got >= D and (got == D or D > 2 * ell + 1)
    assert path_distance(g, run_band(g, A, 32, B, 32, L.LVS_ENC_ASCII7, ex)) == D
    rng = np.random.default_rng(41)
    for m, n in ((9, 23), (23, 9), (1, 12), (17, 17)):
        say("ragged band", m, n)
        sa, sb = W.random_letters(rng, m), W.random_letters(rng, n)
        path = run_band(g, enc(g, sa, L.LVS_ENC_ASCII7, 613), m, enc(g, sb, L.LVS_ENC_ASCII7, 614), n,
                        L.LVS_ENC_ASCII7, L.lvs_band_exact(m, n))
        assert path_distance(g, path) == P.edit_distance(sa, sb)


def test_empty_strings_band(gpu):
    g = gpu
    L = g.L
    B = enc(g, b"abc", L.LVS_ENC_ASCII7, 615)
    path = run_band(g, None, 0, B, 3, L.LVS_ENC_ASCII7, 1)
    assert path_distance(g, path) == 3
    path = run_band(g, B, 3, None, 0, L.LVS_ENC_ASCII7, 0)
    assert path_distance(g, path) == 3


def test_cleartext_band(gpu, okeys):
    """Section 5 table + band: the path is bit-exact with the oracle's
    cleartext banded loop and decrypts to the distance."""
    say("cleartext band")
    g = gpu
    L, torch = g.L, g.torch
    a, b = b"kitten", b"sitting"
    alpha = W.alphabet_of([b])
    A = enc(g, a, L.LVS_ENC_ASCII7, 616)
    dA = L.to_device(A, g.dev)
    d_tab = torch.zeros(len(alpha) * len(a) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, dA, len(a), L.LVS_ENC_ASCII7, alpha, d_tab)
    ell = L.lvs_band_exact(len(a), len(b))
    d_path = torch.zeros((len(a) + len(b)) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_clear_band(g.ctx, d_tab, len(a), alpha, b, ell, d_path)
    torch.cuda.synchronize()
    path = L.to_host(d_path).reshape(-1, L.CT_WORDS)
    assert path_distance(g, path) == 3
    oA = OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 616)
    otab = OL.preprocess(okeys, oA, alpha, OL.ENC_ASCII7)
    ref = OL.edit_distance_clear_band(okeys, otab, alpha, b, ell)
    for k in range(len(ref)):
        assert_same_ct(path[k], ref[k], f"path[{k}]")


def test_plan_mixing_band_and_full(gpu):
    """One graph-captured plan with banded and full queries: each result is
    bit-identical to the query run alone; the plan has the banded count of
    bootstraps."""
    say("band plan")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(43)
    specs = [(12, 12, 3), (20, 14, None), (16, 16, 8), (7, 19, L.lvs_band_exact(7, 19))]
    items, alone = [], []
    want_pbs = 0
    for k, (m, n, ell) in enumerate(specs):
        sa, sb = W.random_letters(rng, m), W.random_letters(rng, n)
        A, B = enc(g, sa, L.LVS_ENC_ASCII7, 620 + 2 * k), enc(g, sb, L.LVS_ENC_ASCII7, 621 + 2 * k)
        dA, dB = L.to_device(A, g.dev), L.to_device(B, g.dev)
        it = {"d_a": dA, "m": m, "d_b": dB, "n": n}
        if ell is None:
            it["d_h_last"] = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
            d_h = torch.zeros_like(it["d_h_last"])
            L.lvs_edit_distance(g.ctx, dA, m, dB, n, L.LVS_ENC_ASCII7, d_h)
            torch.cuda.synchronize()
            alone.append(L.to_host(d_h))
            want_pbs += 3 * m * n
        else:
            it["ell"] = ell
            it["d_path"] = torch.zeros((m + n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
            alone.append(run_band(g, A, m, B, n, L.LVS_ENC_ASCII7, ell).reshape(-1))
            want_pbs += 3 * L.lvs_band_cells(m, n, ell)
        items.append(it)
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    steps, pbs, _ = L.lvs_plan_info(plan)
    assert pbs == want_pbs
    for rep in range(2):
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        for it, ref in zip(items, alone):
            out = L.to_host(it["d_path"] if "ell" in it else it["d_h_last"])
            assert (out == ref).all(), rep
