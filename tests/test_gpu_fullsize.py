"""Parity at the workloads' full sizes, in the launch shapes bench.py times:
the batched workload's 256 pairs as one graph plan and one encrypted query
against the serving workload's 1024 cleartext names.  The oracle cannot run
these whole, so each is checked by what it can compute one by one: every
distance against Wagner-Fischer, sampled queries against their lone runs,
and the smallest query (batched) or a short name (serving) bit-exact with a
live oracle run (a name's rows depend only on the table rows of its own
symbols, so the oracle builds those alone)."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu


def test_batched_256_pairs_full_plan(gpu, okeys):
    g = gpu
    L, torch = g.L, g.torch
    pairs = W.batched()
    say("full size: batched 256 pairs, encrypting")
    cts, items = [], []
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 11000 + 2 * k)
        B = L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 11001 + 2 * k)
        cts.append((A, B))
        items.append({"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b),
                      "d_h_last": torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)})
    say("full size: batched 256 pairs, graph plan")
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    steps, pbs, _ = L.lvs_plan_info(plan)
    assert pbs == 3 * sum(len(a) * len(b) for a, b in pairs)
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    rows = [L.to_host(it["d_h_last"]).reshape(len(b), L.CT_WORDS) for (a, b), it in zip(pairs, items)]
    for k, ((a, b), h) in enumerate(zip(pairs, rows)):
        assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b), k
    del plan
    order = sorted(range(len(pairs)), key=lambda k: len(pairs[k][0]) * len(pairs[k][1]))
    smallest = order[0]
    for k in (smallest, order[-1], 100):
        (a, b), (A, B) = pairs[k], cts[k]
        say("full size: lone run of query", k, len(a), len(b))
        d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev), len(a), L.to_device(B, g.dev), len(b), L.LVS_ENC_ASCII7,
                            d_h)
        torch.cuda.synchronize()
        assert (L.to_host(d_h).reshape(len(b), L.CT_WORDS) == rows[k]).all(), k
    (a, b) = pairs[smallest]
    say("full size: oracle run of query", smallest, len(a), len(b))
    oh = OL.edit_distance(okeys, OL.encrypt_string(okeys, a, OL.ENC_ASCII7, 11000 + 2 * smallest),
                          OL.encrypt_string(okeys, b, OL.ENC_ASCII7, 11001 + 2 * smallest), OL.ENC_ASCII7)
    for j in range(len(b)):
        assert_same_ct(rows[smallest][j], oh[j], f"query {smallest} h[m,{j + 1}]")


def test_serving_query_against_1024_names(gpu, okeys):
    g = gpu
    L, torch = g.L, g.torch
    server, queries = W.serving()
    q = queries[1]
    alpha = W.alphabet_of(server)
    max_step = 8192
    per = L.lvs_server_request_bytes(server, len(alpha), len(q))
    say("full size: serving, 1024 names, query length", len(q))
    srv = L.lvs_server_create(g.ctx, server, alpha, L.lvs_server_fixed_bytes(max_step) + 2 * per + 4096,
                              max_step=max_step)
    Q = L.lvs_encrypt_string(g.ck, q, L.LVS_ENC_ASCII7, 12000)
    t = L.lvs_server_submit(srv, Q)
    out = None
    for _ in range(10000):
        L.lvs_server_step(srv)
        out = L.lvs_server_poll(srv, t)
        if out is not None:
            break
    assert out is not None
    starts = np.cumsum([0] + [len(nm) for nm in server])
    for k, nm in enumerate(server):
        assert L.lvs_decrypt_distance(g.ck, out[starts[k]:starts[k + 1]], len(q)) == P.edit_distance(q, nm), k
    # three names against the single-query cleartext path
    d_tab = torch.zeros(len(alpha) * len(q) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, L.to_device(Q, g.dev), len(q), L.LVS_ENC_ASCII7, alpha, d_tab)
    short = min(range(len(server)), key=lambda k: len(server[k]))
    for k in (short, 0, 1023):
        nm = server[k]
        d_h = torch.zeros(len(nm) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_edit_distance_clear(g.ctx, d_tab, len(q), alpha, nm, d_h)
        torch.cuda.synchronize()
        assert (L.to_host(d_h).reshape(len(nm), L.CT_WORDS) == out[starts[k]:starts[k + 1]]).all(), k
    # the shortest name against the oracle, table rows of its own symbols only
    nm = server[short]
    sub_alpha = bytes(sorted(set(nm)))
    say("full size: oracle run of name", short, nm)
    otab = OL.preprocess(okeys, OL.encrypt_string(okeys, q, OL.ENC_ASCII7, 12000), sub_alpha, OL.ENC_ASCII7)
    oh = OL.edit_distance_clear(okeys, otab, sub_alpha, nm, OL.ENC_ASCII7)
    for j in range(len(nm)):
        assert_same_ct(out[starts[short] + j], oh[j], f"name {short} h[m,{j + 1}]")
