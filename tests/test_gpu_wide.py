"""Wide symbols (Section 4.2: 4-bit subtraction sub-equalities merged as in
Algorithm 2) through the C ABI against the oracle: the eq9 matrix, the edit
distance and the Section 5 table with a cleartext symbol string, every
ciphertext bit-exact, every distance equal to Wagner-Fischer on the symbol
sequences."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P

pytestmark = pytest.mark.gpu


def symbols(width, seed):
    """Four symbols and four partners: equal, one chunk changed, one bit
    changed, random (so every merge outcome appears)."""
    rng = np.random.default_rng(seed)
    top = 2 ** width

    def draw():  # uniform below 2^width
        return int(rng.integers(0, 2 ** min(width, 62))) % top if width <= 62 else \
            int(rng.integers(0, 2 ** 62)) << 2 | int(rng.integers(0, 4))
    xs = [draw() for _ in range(4)]
    c = P.wide_chunk_count(width)
    k = int(rng.integers(0, c))
    ys = [xs[0], xs[1] ^ (1 << (4 * k)), xs[2] ^ (1 << (width - 1)), draw()]
    return xs, ys


@pytest.mark.parametrize("width", [4, 21, 64])
def test_wide_equality_bit_exact(gpu, okeys, width):
    say("wide equality", width)
    g = gpu
    L, torch = g.L, g.torch
    xs, ys = symbols(width, width)
    A = L.lvs_encrypt_symbols(g.ck, xs, width, 901)
    B = L.lvs_encrypt_symbols(g.ck, ys, width, 902)
    m, n = len(xs), len(ys)
    d_eq9 = torch.zeros(m * n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_equality_wide(g.ctx, L.to_device(A, g.dev), m, L.to_device(B, g.dev), n, width, d_eq9)
    torch.cuda.synchronize()
    eq9 = L.to_host(d_eq9).reshape(m, n, L.CT_WORDS)
    ref = OL.equality_wide(okeys, OL.encrypt_symbols(okeys, xs, width, 901), OL.encrypt_symbols(okeys, ys, width, 902),
                           width)
    for i in range(m):
        for j in range(n):
            assert_same_ct(eq9[i, j], ref[i, j], f"eq9[{i},{j}]")
            assert L.lvs_lwe_decrypt(g.ck, eq9[i, j])[0] == (9 if xs[i] == ys[j] else 0)


def test_wide_edit_distance_bit_exact(gpu, okeys):
    """21-bit symbols (Unicode code points), refresh every 4 diagonals: the
    bottom row bit-exact with the oracle."""
    say("wide edit distance")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(31)
    alphabet = [int(v) for v in rng.integers(0, 2 ** 21, size=5)]
    a = [alphabet[int(t)] for t in rng.integers(0, 5, size=6)]
    b = [alphabet[int(t)] for t in rng.integers(0, 5, size=7)]
    A = L.lvs_encrypt_symbols(g.ck, a, 21, 903)
    B = L.lvs_encrypt_symbols(g.ck, b, 21, 904)
    d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    prev = L.lvs_context_get_refresh(g.ctx)
    L.lvs_context_set_refresh(g.ctx, 4)
    try:
        L.lvs_edit_distance_wide(g.ctx, L.to_device(A, g.dev), len(a), L.to_device(B, g.dev), len(b), 21, d_h)
        torch.cuda.synchronize()
    finally:
        L.lvs_context_set_refresh(g.ctx, prev)
    h = L.to_host(d_h).reshape(len(b), L.CT_WORDS)
    ref = OL.edit_distance_wide(okeys, OL.encrypt_symbols(okeys, a, 21, 903), OL.encrypt_symbols(okeys, b, 21, 904),
                                21, refresh_every=4)
    for j in range(len(b)):
        assert_same_ct(h[j], ref[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)


def test_wide_cleartext_bit_exact(gpu, okeys):
    """Section 5 over 21-bit symbols: the table and the cleartext main pass
    bit-exact with the oracle."""
    say("wide cleartext")
    g = gpu
    L, torch = g.L, g.torch
    a = [0x1F600, 0x41, 0x1F600, 0x3042, 0x41]
    b = [0x41, 0x1F600, 0x3042, 0x3042, 0x10FFFF]
    alphabet = sorted(set(b))
    m, n, S = len(a), len(b), len(alphabet)
    A = L.lvs_encrypt_symbols(g.ck, a, 21, 905)
    d_tab = torch.zeros(S * m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess_wide(g.ctx, L.to_device(A, g.dev), m, 21, alphabet, d_tab)
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_clear_wide(g.ctx, d_tab, m, alphabet, b, d_h)
    torch.cuda.synchronize()
    tab = L.to_host(d_tab).reshape(S, m, L.CT_WORDS)
    h = L.to_host(d_h).reshape(n, L.CT_WORDS)
    otab = OL.preprocess_wide(okeys, OL.encrypt_symbols(okeys, a, 21, 905), alphabet, 21)
    for s_ in range(S):
        for i in range(m):
            assert_same_ct(tab[s_, i], otab[s_, i], f"T[{s_}][{i}]")
    oh = OL.edit_distance_clear(okeys, otab, alphabet, b, None)
    for j in range(n):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")
    assert L.lvs_decrypt_distance(g.ck, h, m) == P.edit_distance(a, b)
    with pytest.raises(L.LvsError) as e:
        L.lvs_edit_distance_clear_wide(g.ctx, d_tab, m, alphabet, [0x42], d_h)
    assert e.value.code == -2


def test_wide_larger_pair_distance(gpu):
    """A 24 x 20 pair of 32-bit symbols over a 6-symbol alphabet (9
    bootstraps per pair): exact distance; empty strings; a bad width."""
    say("wide 24x20")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(32)
    alphabet = [int(v) for v in rng.integers(0, 2 ** 32, size=6)]
    a = [alphabet[int(t)] for t in rng.integers(0, 6, size=24)]
    b = [alphabet[int(t)] for t in rng.integers(0, 6, size=20)]
    A = L.to_device(L.lvs_encrypt_symbols(g.ck, a, 32, 906), g.dev)
    B = L.to_device(L.lvs_encrypt_symbols(g.ck, b, 32, 907), g.dev)
    d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_wide(g.ctx, A, len(a), B, len(b), 32, d_h)
    torch.cuda.synchronize()
    h = L.to_host(d_h).reshape(len(b), L.CT_WORDS)
    assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)
    L.lvs_edit_distance_wide(g.ctx, None, 0, B, len(b), 32, d_h)
    torch.cuda.synchronize()
    assert L.lvs_decrypt_distance(g.ck, L.to_host(d_h).reshape(len(b), L.CT_WORDS), 0) == len(b)
    with pytest.raises(L.LvsError) as e:
        L.lvs_edit_distance_wide(g.ctx, A, len(a), B, len(b), 65, d_h)
    assert e.value.code == -1


def test_wide_batch_plan_equals_alone(gpu):
    """A graph-captured plan over 21-bit symbols mixing lengths, an empty
    string and a banded query: every result equals its lone run (the banded
    one the plaintext banded loop), replayed twice."""
    say("wide batch plan")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(33)
    alphabet = [int(v) for v in rng.integers(0, 2 ** 21, size=5)]
    lens = [(5, 7), (9, 4), (0, 3), (6, 6), (3, 8)]
    pairs = [([alphabet[int(t)] for t in rng.integers(0, 5, size=m)], [alphabet[int(t)] for t in rng.integers(0, 5, size=n)])
             for m, n in lens]
    items, cts = [], []
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_symbols(g.ck, a, 21, 950 + 2 * k)
        B = L.lvs_encrypt_symbols(g.ck, b, 21, 951 + 2 * k)
        cts.append((A, B))
        it = {"d_a": L.to_device(A, g.dev) if a else None, "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b)}
        if k == 3:
            it["ell"] = 1
            it["d_path"] = torch.zeros((len(a) + len(b)) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        else:
            it["d_h_last"] = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        items.append(it)
    plan = L.lvs_plan_create_wide(g.ctx, items, 21, graph=True)
    for rep in range(2):
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        for k, ((a, b), (A, B), it) in enumerate(zip(pairs, cts, items)):
            if k == 3:
                path = L.to_host(it["d_path"]).reshape(-1, L.CT_WORDS)
                assert L.lvs_decrypt_distance(g.ck, path, 0) == P.band_distance(a, b, 1), (rep, k)
                continue
            h = L.to_host(it["d_h_last"]).reshape(len(b), L.CT_WORDS)
            d_ref = torch.zeros_like(it["d_h_last"])
            L.lvs_edit_distance_wide(g.ctx, it["d_a"], len(a), it["d_b"], len(b), 21, d_ref)
            torch.cuda.synchronize()
            assert (h == L.to_host(d_ref).reshape(len(b), L.CT_WORDS)).all(), (rep, k)
            assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b), (rep, k)


def test_wide_server_mix_equals_alone(gpu, okeys):
    """The serving engine over 21-bit symbols: three queries submitted at
    different step boundaries against five names, in an arena that holds two
    requests (the third waits for memory); every request's rows equal its
    lone run (the wide Section 5 table, then the cleartext pass per name),
    every distance equals Wagner-Fischer, and one name's rows are bit-exact
    with the oracle."""
    say("wide server")
    g = gpu
    L, torch = g.L, g.torch
    width = 21
    rng = np.random.default_rng(34)
    alphabet = sorted({int(v) for v in rng.integers(0, 2 ** width, size=6)})
    names = [[alphabet[int(t)] for t in rng.integers(0, len(alphabet), size=n)] for n in (4, 7, 1, 9, 5)]
    queries = [[alphabet[int(t)] for t in rng.integers(0, len(alphabet), size=m)] for m in (5, 3, 8)]
    cts = [L.lvs_encrypt_symbols(g.ck, q, width, 960 + k) for k, q in enumerate(queries)]
    per = max(L.lvs_server_request_bytes_wide(names, len(alphabet), len(q), width) for q in queries)
    max_step = 4096
    srv = L.lvs_server_create_wide(g.ctx, names, alphabet, width, L.lvs_server_fixed_bytes(max_step) + 2 * per + 4096,
                                   max_step=max_step)
    arrivals = {0: [0], 1: [1], 4: [2]}
    tickets, outs = {}, {}
    for step in range(2000):
        for k in arrivals.get(step, []):
            tickets[k] = L.lvs_server_submit(srv, cts[k])
        L.lvs_server_step(srv)
        for k, t in tickets.items():
            if k not in outs:
                o = L.lvs_server_poll(srv, t)
                if o is not None:
                    outs[k] = o
        if len(outs) == len(queries):
            break
    assert len(outs) == len(queries)
    starts = np.cumsum([0] + [len(nm) for nm in names])
    for k, q in enumerate(queries):
        m = len(q)
        d_tab = torch.zeros(len(alphabet) * m * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_preprocess_wide(g.ctx, L.to_device(cts[k], g.dev), m, width, alphabet, d_tab)
        for j, nm in enumerate(names):
            rows = outs[k][starts[j]:starts[j + 1]]
            d_h = torch.zeros(len(nm) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
            L.lvs_edit_distance_clear_wide(g.ctx, d_tab, m, alphabet, nm, d_h)
            torch.cuda.synchronize()
            assert (L.to_host(d_h).reshape(len(nm), L.CT_WORDS) == rows).all(), (k, j)
            assert L.lvs_decrypt_distance(g.ck, rows, m) == P.edit_distance(q, nm), (k, j)
    # name 0 against query 0 through the oracle, table rows of its own symbols
    nm = names[0]
    sub_alpha = sorted(set(nm))
    otab = OL.preprocess_wide(okeys, OL.encrypt_symbols(okeys, queries[0], width, 960), sub_alpha, width)
    oh = OL.edit_distance_clear(okeys, otab, sub_alpha, nm, None)
    for j in range(len(nm)):
        assert_same_ct(outs[0][j], oh[j], f"name 0 h[m,{j + 1}]")
    with pytest.raises(L.LvsError) as e:
        L.lvs_server_create_wide(g.ctx, [[2 ** width]], [2 ** width], width, L.lvs_server_fixed_bytes(16) + 4096,
                                 max_step=16)
    assert e.value.code == -2
