"""Noise refresh (Section 3.1: the differences are bootstrapped again through
an identity table before their noise reaches the decoding threshold, the
noise discussion around Fig. noise5).

Every entry point with a short refresh interval is bit-exact with the
oracle run with the same interval; batch plans and the serving engine equal
their lone runs; refresh lowers the error of the bottom row on the 256 x 256
DNA alignment; with refresh off, the noise bound is enforced."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu

R = 4


class refresh_interval:
    """Sets the context's interval for a block, restoring the previous one."""

    def __init__(self, g, every):
        self.g, self.every = g, every

    def __enter__(self):
        self.prev = self.g.L.lvs_context_get_refresh(self.g.ctx)
        self.g.L.lvs_context_set_refresh(self.g.ctx, self.every)

    def __exit__(self, *exc):
        self.g.L.lvs_context_set_refresh(self.g.ctx, self.prev)


def one_shot(g, A, m, B, n, enc):
    L, torch = g.L, g.torch
    d_h = torch.zeros(max(1, n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev), m, L.to_device(B, g.dev), n, enc, d_h)
    torch.cuda.synchronize()
    return L.to_host(d_h)[:n * L.CT_WORDS].reshape(n, L.CT_WORDS)


def test_default_and_bounds(gpu):
    g = gpu
    L = g.L
    assert L.lvs_context_get_refresh(g.ctx) == L.LVS_REFRESH_DEFAULT
    for bad in (1, 3, L.LVS_REFRESH_MAX + 1):
        with pytest.raises(L.LvsError) as e:
            L.lvs_context_set_refresh(g.ctx, bad)
        assert e.value.code == -1
    assert L.lvs_context_get_refresh(g.ctx) == L.LVS_REFRESH_DEFAULT


@pytest.mark.parametrize("a,b,enc_", [(b"ACGTTGCA", b"CGTTAGCAT", "dna"), (b"kitten", b"sitting", "ascii")])
def test_refresh_bit_exact_with_oracle(gpu, okeys, a, b, enc_):
    """Refresh after diagonals 4, 8, 12, ...: the bottom row bit-exact with the
    oracle's diagonal loop refreshing on the same diagonals."""
    say("refresh vs oracle", a, b, R)
    g = gpu
    L = g.L
    e = L.LVS_ENC_DNA2 if enc_ == "dna" else L.LVS_ENC_ASCII7
    oe = OL.ENC_DNA2 if enc_ == "dna" else OL.ENC_ASCII7
    sa = W.dna_codes(a) if enc_ == "dna" else a
    sb = W.dna_codes(b) if enc_ == "dna" else b
    A = L.lvs_encrypt_string(g.ck, sa, e, 801)
    B = L.lvs_encrypt_string(g.ck, sb, e, 802)
    with refresh_interval(g, R):
        h = one_shot(g, A, len(a), B, len(b), e)
    oh = OL.edit_distance(okeys, OL.encrypt_string(okeys, sa, oe, 801), OL.encrypt_string(okeys, sb, oe, 802), oe,
                          refresh_every=R)
    for j in range(len(b)):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)
    # a different interval changes the ciphertexts, not the distance
    h0 = one_shot(g, A, len(a), B, len(b), e)
    assert not (h0 == h).all()
    assert L.lvs_decrypt_distance(g.ck, h0, len(a)) == P.edit_distance(a, b)


def test_refresh_band_bit_exact_with_oracle(gpu, okeys):
    """The band path with refresh: every path ciphertext bit-exact (the path
    keeps the values as the cell bootstraps wrote them)."""
    say("refresh band vs oracle")
    g = gpu
    L, torch = g.L, g.torch
    a, b = b"GATTACAGT", b"GTTACAGGA"
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    A = L.lvs_encrypt_string(g.ck, sa, L.LVS_ENC_DNA2, 803)
    B = L.lvs_encrypt_string(g.ck, sb, L.LVS_ENC_DNA2, 804)
    oA = OL.encrypt_string(okeys, sa, OL.ENC_DNA2, 803)
    oB = OL.encrypt_string(okeys, sb, OL.ENC_DNA2, 804)
    m, n = len(a), len(b)
    for ell in (2, P.exact_band(m, n)):
        d_path = torch.zeros((m + n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        with refresh_interval(g, R):
            L.lvs_edit_distance_band(g.ctx, L.to_device(A, g.dev), m, L.to_device(B, g.dev), n, L.LVS_ENC_DNA2,
                                     ell, d_path)
        torch.cuda.synchronize()
        path = L.to_host(d_path).reshape(m + n, L.CT_WORDS)
        ref = OL.edit_distance_band(okeys, oA, oB, OL.ENC_DNA2, ell, refresh_every=R)
        for k in range(m + n):
            assert_same_ct(path[k], ref[k], f"ell={ell} path[{k}]")
        assert L.lvs_decrypt_distance(g.ck, path, 0) == P.band_distance(a, b, ell)


def test_refresh_cleartext_bit_exact_with_oracle(gpu, okeys):
    """Section 5's table with a cleartext string, refreshed: bit-exact."""
    say("refresh cleartext vs oracle")
    g = gpu
    L, torch = g.L, g.torch
    a, b = b"saturday", b"sunday"
    alpha = bytes(sorted(set(b)))
    m, n, S = len(a), len(b), len(alpha)
    A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 805)
    d_tab = torch.zeros(S * m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, L.to_device(A, g.dev), m, L.LVS_ENC_ASCII7, alpha, d_tab)
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    with refresh_interval(g, R):
        L.lvs_edit_distance_clear(g.ctx, d_tab, m, alpha, b, d_h)
    torch.cuda.synchronize()
    h = L.to_host(d_h).reshape(n, L.CT_WORDS)
    otab = OL.preprocess(okeys, OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 805), alpha, OL.ENC_ASCII7)
    oh = OL.edit_distance_clear(okeys, otab, alpha, b, OL.ENC_ASCII7, refresh_every=R)
    for j in range(n):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b) == 3


def test_refresh_in_batch_plan_equals_alone(gpu):
    """A graph-captured plan mixing lengths (some queries past a refresh
    diagonal, some not): each bottom row equals its lone run with the same
    interval."""
    say("refresh batch plan")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(12)
    pairs = [(W.random_letters(rng, int(rng.integers(2, 14))), W.random_letters(rng, int(rng.integers(2, 14))))
             for _ in range(10)]
    items, outs, cts = [], [], []
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 8100 + 2 * k)
        B = L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 8101 + 2 * k)
        d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        cts.append((A, B))
        outs.append(d_h)
        items.append({"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b),
                      "d_h_last": d_h})
    with refresh_interval(g, 6):
        plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
        for _ in range(2):
            L.lvs_plan_run(plan)
            torch.cuda.synchronize()
            for (a, b), (A, B), d_h in zip(pairs, cts, outs):
                h = L.to_host(d_h).reshape(len(b), L.CT_WORDS)
                assert (h == one_shot(g, A, len(a), B, len(b), L.LVS_ENC_ASCII7)).all()
                assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)


def test_refresh_serving_equals_clear_path(gpu):
    """The serving engine with refresh rounds: every name's bottom row equals
    lvs_edit_distance_clear on the same table with the same interval."""
    say("refresh serving")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(13)
    names = [W.random_letters(rng, int(rng.integers(2, 16))) for _ in range(6)]
    q = W.random_letters(rng, 11)
    alpha = W.alphabet_of(names + [q])
    Q = L.lvs_encrypt_string(g.ck, q, L.LVS_ENC_ASCII7, 806)
    with refresh_interval(g, 8):
        per = L.lvs_server_request_bytes(names, len(alpha), len(q))
        srv = L.lvs_server_create(g.ctx, names, alpha, L.lvs_server_fixed_bytes(4096) + 2 * per + 4096, 4096)
        t = L.lvs_server_submit(srv, Q)
        for _ in range(400):
            L.lvs_server_step(srv)
            out = L.lvs_server_poll(srv, t)
            if out is not None:
                break
        assert out is not None
        rows = out.reshape(-1, L.CT_WORDS)
        d_tab = torch.zeros(len(alpha) * len(q) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_preprocess(g.ctx, L.to_device(Q, g.dev), len(q), L.LVS_ENC_ASCII7, alpha, d_tab)
        pos = 0
        for name in names:
            d_h = torch.zeros(len(name) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
            L.lvs_edit_distance_clear(g.ctx, d_tab, len(q), alpha, name, d_h)
            torch.cuda.synchronize()
            ref = L.to_host(d_h).reshape(len(name), L.CT_WORDS)
            assert (rows[pos:pos + len(name)] == ref).all(), name
            assert L.lvs_decrypt_distance(g.ck, ref, len(q)) == P.edit_distance(q, name)
            pos += len(name)


def test_noise_budget_with_refresh_off(gpu):
    """Refresh off: min(m, n) above the bound is refused before any launch
    (the buffers have their full sizes all the same)."""
    say("noise budget with refresh off")
    g = gpu
    L, torch = g.L, g.torch
    m = L.LVS_MAX_DEPTH_NO_REFRESH + 1
    d_eq9 = torch.zeros(m * m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    d_h = torch.zeros(m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    with refresh_interval(g, 0):
        with pytest.raises(L.LvsError) as e:
            L.lvs_edit_distance_eq9(g.ctx, d_eq9, m, m, d_h)
        assert e.value.code == -3
    del d_eq9


def bottom_row_error(g, h, want_rows):
    """Signed phase error of each h[m, j] under the extracted GLWE key."""
    L = g.L
    S = L.lvs_key_export(g.ck, None, 1).astype(np.uint64)
    phase = h[:, -1] - h[:, :-1] @ S
    mu = np.array([x % 32 for x in want_rows], dtype=np.uint64)
    return (phase - (mu << np.uint64(59))).astype(np.int64).astype(np.float64)


def test_refresh_lowers_bottom_row_noise_dna_256(gpu):
    """DNA 256 x 256 (5% edits), refresh off vs every 64 diagonals: the
    same distance; the error of h[m, j] for j >= 192 (about 2 min(m, j)
    bootstrap outputs summed without refresh, at most 2 * 32 + 1 with it)
    is at least 1.8 times smaller with refresh."""
    say("refresh noise: dna 256, R=0 and R=64")
    g = gpu
    L = g.L
    a, b = W.dna_align()
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    m, n = len(a), len(b)
    A = L.lvs_encrypt_string(g.ck, sa, L.LVS_ENC_DNA2, 807)
    B = L.lvs_encrypt_string(g.ck, sb, L.LVS_ENC_DNA2, 808)
    _, h_pl, _ = P.delta_dp(a, b)
    want = [int(h_pl[m, j]) for j in range(1, n + 1)]
    std = {}
    for every in (0, 64):
        with refresh_interval(g, every):
            h = one_shot(g, A, m, B, n, L.LVS_ENC_DNA2)
        assert L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b)
        err = bottom_row_error(g, h, want)
        assert np.abs(err).max() < 2.0 ** 57
        std[every] = err[191:].std()
    say(f"bottom-row error std (j >= 192): 2^{np.log2(std[0]):.2f} without refresh, "
        f"2^{np.log2(std[64]):.2f} with refresh every 64")
    assert std[0] > 1.8 * std[64]


def test_past_the_no_refresh_length_dna_400(gpu):
    """A 400 x 400 DNA alignment (5% edits, the DNA workload's recipe at a
    length the noise budget refuses without refresh) with the default
    refresh interval (anti-diagonals 256 and 512 refreshed): the exact
    distance, every h[m, j] decoding to its plaintext difference with a
    phase error below half the decoding threshold."""
    say("past the no-refresh length: dna 400 x 400, default refresh")
    g = gpu
    L = g.L
    a, b = W.dna_align(seed=41, length=400)
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    m, n = len(a), len(b)
    A = L.lvs_encrypt_string(g.ck, sa, L.LVS_ENC_DNA2, 841)
    B = L.lvs_encrypt_string(g.ck, sb, L.LVS_ENC_DNA2, 842)
    assert L.lvs_context_get_refresh(g.ctx) == L.LVS_REFRESH_DEFAULT
    h = one_shot(g, A, m, B, n, L.LVS_ENC_DNA2)
    assert L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b)
    _, h_pl, _ = P.delta_dp(a, b)
    err = bottom_row_error(g, h, [int(h_pl[m, j]) for j in range(1, n + 1)])
    say(f"dna 400: bottom-row error max 2^{np.log2(np.abs(err).max()):.2f}, std 2^{np.log2(err.std()):.2f}")
    assert np.abs(err).max() < 2.0 ** 57
    with refresh_interval(g, 0):
        with pytest.raises(L.LvsError) as e:
            one_shot(g, A, m, B, n, L.LVS_ENC_DNA2)
        assert e.value.code == -3
