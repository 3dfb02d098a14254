"""Batched edit distances (lvs_plan_*): every ready cell of every query in
one launch per step, captured as a HIP graph.  Bar: each query's result is
bit-identical to the same query computed alone, every graph replay equals the
eager result, and every distance equals Wagner-Fischer; sampled ciphertexts
of the batched workload are bit-exact with the oracle."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu


def encrypt_pairs(g, pairs, enc, seed0=5000):
    L = g.L
    out = []
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_string(g.ck, a, enc, seed0 + 2 * k)
        B = L.lvs_encrypt_string(g.ck, b, enc, seed0 + 2 * k + 1)
        out.append((A, B))
    return out


def alone(g, A, m, B, n, enc):
    L, torch = g.L, g.torch
    d_h = torch.zeros(max(1, n) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev) if m else None, m, L.to_device(B, g.dev) if n else None, n,
                        enc, d_h)
    torch.cuda.synchronize()
    return L.to_host(d_h)[:n * L.CT_WORDS].reshape(n, L.CT_WORDS)


def make_batch(g, pairs, cts, enc):
    L, torch = g.L, g.torch
    items, outs, keep = [], [], []
    for (a, b), (A, B) in zip(pairs, cts):
        dA = L.to_device(A, g.dev) if len(a) else None
        dB = L.to_device(B, g.dev) if len(b) else None
        d_h = torch.zeros(max(1, len(b)) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        keep += [dA, dB]
        outs.append(d_h)
        items.append({"d_a": dA, "m": len(a), "d_b": dB if dB is not None else torch.zeros(1, device=g.dev),
                      "n": len(b), "d_h_last": d_h})
    return items, outs, keep


def read(g, d_h, n):
    return g.L.to_host(d_h)[:n * g.L.CT_WORDS].reshape(n, g.L.CT_WORDS)


def test_batch_equals_alone_and_graph_replays(gpu):
    say("batch vs alone")
    g = gpu
    L, torch = g.L, g.torch
    pairs = [(b"kitten", b"sitting"), (b"KID", b"SIT"), (b"a", b"abcdefghij"), (b"flaw", b"lawn"),
             (b"", b"xyz"), (b"Saturday", b"Sunday"), (b"same", b"same")]
    cts = encrypt_pairs(g, pairs, L.LVS_ENC_ASCII7)
    items, outs, keep = make_batch(g, pairs, cts, L.LVS_ENC_ASCII7)
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    steps, pbs, mx = L.lvs_plan_info(plan)
    assert pbs == 3 * sum(len(a) * len(b) for a, b in pairs)
    assert steps == 2 + max(len(a) + len(b) for a, b in pairs if a and b) - 1
    refs = [alone(g, A, len(a), B, len(b), L.LVS_ENC_ASCII7) for (a, b), (A, B) in zip(pairs, cts)]
    for rep in range(3):
        for d in outs:
            d.zero_()
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        for k, ((a, b), d_h) in enumerate(zip(pairs, outs)):
            h = read(g, d_h, len(b))
            assert (h == refs[k]).all(), (rep, k)
            assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)
        # eager work of the program between replays
        _ = alone(g, cts[1][0], 3, cts[1][1], 3, L.LVS_ENC_ASCII7)


def test_batch_without_graph_dna(gpu):
    say("batch dna eager")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(4)
    pairs = []
    for _ in range(5):
        a = bytes(rng.integers(0, 4, size=int(rng.integers(1, 12))))
        b = bytes(rng.integers(0, 4, size=int(rng.integers(1, 12))))
        pairs.append((a, b))
    cts = encrypt_pairs(g, pairs, L.LVS_ENC_DNA2, 6000)
    items, outs, keep = make_batch(g, pairs, cts, L.LVS_ENC_DNA2)
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_DNA2, graph=False)
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    for (a, b), (A, B), d_h in zip(pairs, cts, outs):
        h = read(g, d_h, len(b))
        assert (h == alone(g, A, len(a), B, len(b), L.LVS_ENC_DNA2)).all()
        assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)


def test_batch_cleartext_variant(gpu, okeys):
    """Queries with one cleartext string: preprocessing tables (Section 5),
    then one batched plan; equal to lvs_edit_distance_clear alone and to the
    oracle for the first query."""
    say("batch cleartext")
    g = gpu
    L, torch = g.L, g.torch
    rng = np.random.default_rng(8)
    pairs = [(W.random_letters(rng, int(rng.integers(3, 9))), W.random_letters(rng, int(rng.integers(3, 9))))
             for _ in range(4)]
    alpha = W.alphabet_of([b for _, b in pairs])
    items, outs, keep, tabs = [], [], [], []
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 7000 + k)
        dA = L.to_device(A, g.dev)
        d_tab = torch.zeros(len(alpha) * len(a) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_preprocess(g.ctx, dA, len(a), L.LVS_ENC_ASCII7, alpha, d_tab)
        d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        keep += [dA]
        tabs.append(d_tab)
        outs.append(d_h)
        items.append({"d_a": dA, "m": len(a), "d_table": d_tab, "alphabet": alpha, "b_clear": b, "d_h_last": d_h})
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    for k, ((a, b), d_h, d_tab) in enumerate(zip(pairs, outs, tabs)):
        h = read(g, d_h, len(b))
        d_ref = torch.zeros_like(d_h)
        L.lvs_edit_distance_clear(g.ctx, d_tab, len(a), alpha, b, d_ref)
        torch.cuda.synchronize()
        assert (h == read(g, d_ref, len(b))).all()
        assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b)
    a, b = pairs[0]
    oA = OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 7000)
    otab = OL.preprocess(okeys, oA, alpha, OL.ENC_ASCII7)
    oh = OL.edit_distance_clear(okeys, otab, alpha, b, OL.ENC_ASCII7)
    h = read(g, outs[0], len(b))
    for j in range(len(b)):
        assert_same_ct(h[j], oh[j], f"h[m,{j + 1}]")


def test_batched_workload_sample(gpu, okeys):
    """The first 24 queries of the batched workload (lengths 8..64): exact
    distances, and each query equal to its run alone for 3 of them; the
    top-left 2 x 2 corner of query 0 bit-exact with a live oracle run."""
    say("batched workload sample")
    g = gpu
    L, torch = g.L, g.torch
    pairs = W.batched()[:24]
    cts = encrypt_pairs(g, pairs, L.LVS_ENC_ASCII7, 9000)
    items, outs, keep = make_batch(g, pairs, cts, L.LVS_ENC_ASCII7)
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    for (a, b), d_h in zip(pairs, outs):
        assert L.lvs_decrypt_distance(g.ck, read(g, d_h, len(b)), len(a)) == P.edit_distance(a, b)
    for k in (0, 7, 23):
        (a, b), (A, B) = pairs[k], cts[k]
        assert (read(g, outs[k], len(b)) == alone(g, A, len(a), B, len(b), L.LVS_ENC_ASCII7)).all()
    # corner of query 0: cells (1..2, 1..2) depend only on a[:2], b[:2]
    a, b = pairs[0]
    A, B = cts[0]
    corner = alone(g, A[:2], 2, B[:2], 2, L.LVS_ENC_ASCII7)
    oh = OL.edit_distance(okeys, OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 9000)[:2],
                          OL.encrypt_string(okeys, b, OL.ENC_ASCII7, 9001)[:2], OL.ENC_ASCII7)
    for j in range(2):
        assert_same_ct(corner[j], oh[j], f"corner h[2,{j + 1}]")
