"""Parity at the workloads' full sizes, in the launch shapes bench.py times.

Batched workload: the 256 pairs as one graph plan, keeping every bootstrap's
output (eq1, eq9 and M of every pair).  Every distance equals Wagner-Fischer;
every ciphertext of the sampled pairs (workloads.batched_sample) equals the
oracle's (digests written by tests/golden/make_oracle_vectors.py); and 1,000
bootstraps drawn uniformly from the plan's 995,328 are rebuilt from the
inputs the plan gave them and re-run live through the oracle.

Serving workload: the sampled queries against the 1024 cleartext names
through the serving engine: every distance equals Wagner-Fischer, the
sampled names' result rows equal the oracle's, and so do the query's
Section 5 table and the sampled names' M ciphertexts (single-query
preprocessing, then a cleartext plan keeping M)."""
import hashlib

import numpy as np
import pytest

from conftest import oracle_vectors
from gpu_common import assert_same_ct, gpu, okeys_kara, oracle_threads, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
from oracle import tfhe as OT
import workloads as W

pytestmark = pytest.mark.gpu

SAMPLED_PBS = 1000


def digest(ct):
    return hashlib.sha256(np.ascontiguousarray(ct, dtype=np.uint64).tobytes()).hexdigest()


def row_digest(cells):
    return hashlib.sha256(b"".join(bytes.fromhex(digest(c)) for c in cells)).hexdigest()


def diff_chain(kind, I, J):
    """h[I, J] (kind 'h') or v[I, J] (kind 'v') of Algorithm 4 as a signed
    sum of cell outputs M plus a multiple of the noise-free Enc(1):
    h[I, J] = M[I, J] - v[I, J-1], v[I, J] = M[I, J] - h[I-1, J], with
    h[0, J] = v[I, 0] = Enc(1).  Returns ([(sign, I', J')], ones)."""
    terms, sign = [], 1
    while True:
        if kind == "h":
            if I == 0:
                return terms, sign
            terms.append((sign, I, J))
            kind, J = "v", J - 1
        else:
            if J == 0:
                return terms, sign
            terms.append((sign, I, J))
            kind, I = "h", I - 1
        sign = -sign


def test_batched_256_pairs_full_plan(gpu, okeys_kara):
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    pairs = W.batched()
    meta = oracle_vectors("batched_sample")
    sample = W.batched_sample()
    assert [q["index"] for q in meta["queries"]] == sample
    assert max(len(a) + len(b) for a, b in pairs) < L.lvs_context_get_refresh(g.ctx)   # no refresh step
    cells = [len(a) * len(b) for a, b in pairs]
    off = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    total = int(off[-1])
    say("full size: batched 256 pairs, encrypting")
    cts, items = [], []
    d_eq1 = torch.zeros(total * Wd, dtype=torch.int64, device=g.dev)
    d_eq9 = torch.zeros_like(d_eq1)
    d_tr = torch.zeros_like(d_eq1)
    for k, (a, b) in enumerate(pairs):
        A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 11000 + 2 * k)
        B = L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 11001 + 2 * k)
        cts.append((A, B))
        lo, hi = int(off[k]) * Wd, int(off[k + 1]) * Wd
        items.append({"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b),
                      "d_h_last": torch.zeros(len(b) * Wd, dtype=torch.int64, device=g.dev),
                      "d_eq1": d_eq1[lo:hi], "d_eq9": d_eq9[lo:hi], "d_trace": d_tr[lo:hi]})
    say("full size: batched 256 pairs, graph plan keeping eq1 / eq9 / M")
    plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=True)
    steps, pbs, _ = L.lvs_plan_info(plan)
    assert pbs == 3 * total
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    del plan
    rows = [L.to_host(it["d_h_last"]).reshape(len(b), Wd) for (a, b), it in zip(pairs, items)]
    for k, ((a, b), h) in enumerate(zip(pairs, rows)):
        assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b), k

    say("full size: sampled pairs against the oracle digests", sample)
    for q in meta["queries"]:
        k = q["index"]
        a, b = pairs[k]
        assert (q["a"], q["b"], q["seed_a"], q["seed_b"]) == (a.decode(), b.decode(), 11000 + 2 * k, 11001 + 2 * k)
        m, n = len(a), len(b)
        lo, hi = int(off[k]) * Wd, int(off[k + 1]) * Wd
        for name, buf in (("eq1", d_eq1), ("eq9", d_eq9), ("M", d_tr)):
            mat = L.to_host(buf[lo:hi]).reshape(m, n, Wd)
            bad = [i for i in range(m) if row_digest(mat[i]) != q[f"{name}_row_sha256"][i]]
            assert not bad, (k, name, bad[:5])
        bad = [j for j in range(n) if digest(rows[k][j]) != q["h_last_sha256"][j]]
        assert not bad, (k, "h_last", bad[:5])

    say(f"full size: {SAMPLED_PBS} bootstraps drawn uniformly from the plan, re-run through the oracle")
    rng = np.random.default_rng(2024)
    draws = rng.choice(3 * total, size=SAMPLED_PBS, replace=False)
    flat = lambda buf: buf.view(-1, Wd)             # noqa: E731
    # which stored outputs the inputs and the checks need: (buffer, flat cell index)
    need = {"eq1": set(), "eq9": set(), "M": set()}
    plan_rows = []
    for u in draws:
        c, kind = divmod(int(u), 3)
        k = int(np.searchsorted(off, c, side="right") - 1)
        n = len(pairs[k][1])
        i, j = divmod(c - int(off[k]), n)
        plan_rows.append((kind, k, i, j, c))
        if kind == 0:
            need["eq1"].add(c)
        elif kind == 1:
            need["eq1"].add(c)
            need["eq9"].add(c)
        else:
            need["eq9"].add(c)
            need["M"].add(c)
            for ch in (diff_chain("v", i + 1, j), diff_chain("h", i, j + 1)):
                for _, I, J in ch[0]:
                    need["M"].add(int(off[k]) + (I - 1) * n + (J - 1))
    got = {}
    for name, buf in (("eq1", d_eq1), ("eq9", d_eq9), ("M", d_tr)):
        idx = sorted(need[name])
        rows_ = L.to_host(flat(buf)[torch.tensor(idx, dtype=torch.long, device=g.dev)].reshape(-1))
        rows_ = rows_.reshape(len(idx), Wd)
        got[name] = {c: rows_[t] for t, c in enumerate(idx)}
    one, four = OT.trivial(1, 2048), OT.trivial(4, 2048)
    inputs, luts, outs = [], [], []
    for kind, k, i, j, c in plan_rows:
        A, B = cts[k]
        n = len(pairs[k][1])
        if kind == 0:                   # eq1 = PBS(x1 - y1; LUT_eq)
            x = (A[i, 0] - B[j, 0]).astype(np.uint64)
            inputs.append(x), luts.append(OL.LUT_IDS["eq"]), outs.append(got["eq1"][c])
        elif kind == 1:                 # eq9 = PBS(2 (x2 - y2) + 1 - eq1; LUT_eq9)
            x = (OT.scale(A[i, 1], 2) - OT.scale(B[j, 1], 2) + one - got["eq1"][c]).astype(np.uint64)
            inputs.append(x), luts.append(OL.LUT_IDS["eq9"]), outs.append(got["eq9"][c])
        else:                           # M = PBS(4 - v[i+1, j] + 3 h[i, j+1] + eq9; LUT_min)
            def value(kind_, I, J):
                terms, ones = diff_chain(kind_, I, J)
                acc = OT.scale(one, ones)
                for sgn, I2, J2 in terms:
                    acc = (acc + OT.scale(got["M"][int(off[k]) + (I2 - 1) * n + (J2 - 1)], sgn)).astype(np.uint64)
                return acc
            x = (four - value("v", i + 1, j) + OT.scale(value("h", i, j + 1), 3) + got["eq9"][c]).astype(np.uint64)
            inputs.append(x), luts.append(OL.LUT_IDS["min"]), outs.append(got["M"][c])
    ref = okeys_kara.pbs_batch(np.stack(inputs), OL.lut_polys(2048), np.asarray(luts, dtype=np.int32),
                               nthreads=oracle_threads())
    bad = [t for t in range(len(outs)) if not np.array_equal(outs[t], ref[t])]
    assert not bad, [plan_rows[t][:4] for t in bad[:5]]
    kinds = np.bincount([r[0] for r in plan_rows], minlength=3)
    say("full size: sampled bootstraps bit-exact: eq1 / eq9 / cell =", kinds.tolist())


def test_serving_sampled_queries_against_1024_names(gpu):
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    server, queries = W.serving()
    meta = oracle_vectors("serving_sample")
    qidx, nidx = W.serving_sample()
    alpha = W.alphabet_of(server)
    assert meta["alphabet"] == alpha.decode() and [q["query"] for q in meta["queries"]] == qidx
    max_step = 1024                  # the step cap bench.py serves with
    per = sum(L.lvs_server_request_bytes(server, len(alpha), len(queries[qi])) for qi in qidx)
    say("full size: serving, 1024 names, queries", qidx)
    srv = L.lvs_server_create(g.ctx, server, alpha, L.lvs_server_fixed_bytes(max_step) + per + 4096,
                              max_step=max_step)
    Qs = {qi: L.lvs_encrypt_string(g.ck, queries[qi], L.LVS_ENC_ASCII7, 12000 + qi) for qi in qidx}
    tickets = {qi: L.lvs_server_submit(srv, Qs[qi]) for qi in qidx}
    outs = {}
    for _ in range(100000):
        L.lvs_server_step(srv)
        for qi, t in tickets.items():
            if qi not in outs:
                r = L.lvs_server_poll(srv, t)
                if r is not None:
                    outs[qi] = r
        if len(outs) == len(qidx):
            break
    assert len(outs) == len(qidx)
    del srv
    starts = np.cumsum([0] + [len(nm) for nm in server])
    for rec in meta["queries"]:
        qi = rec["query"]
        q = queries[qi]
        assert rec["text"] == q.decode() and rec["seed"] == 12000 + qi
        out = outs[qi]
        for k, nm in enumerate(server):
            assert L.lvs_decrypt_distance(g.ck, out[starts[k]:starts[k + 1]], len(q)) == P.edit_distance(q, nm), k
        say("full size: query", qi, "sampled names against the oracle digests")
        for nrec in rec["names"]:
            k = nrec["index"]
            rows = out[starts[k]:starts[k + 1]]
            assert [digest(c) for c in rows] == nrec["h_last_sha256"], (qi, k)
        # the query's table and the sampled names' M through the single-query path
        d_tab = torch.zeros(len(alpha) * len(q) * Wd, dtype=torch.int64, device=g.dev)
        L.lvs_preprocess(g.ctx, L.to_device(Qs[qi], g.dev), len(q), L.LVS_ENC_ASCII7, alpha, d_tab)
        torch.cuda.synchronize()
        tab = L.to_host(d_tab).reshape(len(alpha), len(q), Wd)
        assert [[digest(tab[c, i]) for i in range(len(q))] for c in range(len(alpha))] == rec["table_sha256"]
        items = []
        for nrec in rec["names"]:
            nm = server[nrec["index"]]
            items.append({"m": len(q), "d_table": d_tab, "alphabet": alpha, "b_clear": nm,
                          "d_h_last": torch.zeros(len(nm) * Wd, dtype=torch.int64, device=g.dev),
                          "d_trace": torch.zeros(len(q) * len(nm) * Wd, dtype=torch.int64, device=g.dev)})
        plan = L.lvs_plan_create(g.ctx, items, L.LVS_ENC_ASCII7, graph=False)
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        del plan
        for nrec, it in zip(rec["names"], items):
            nm = server[nrec["index"]]
            tr = L.to_host(it["d_trace"]).reshape(len(q), len(nm), Wd)
            assert [row_digest(tr[i]) for i in range(len(q))] == nrec["M_row_sha256"], (qi, nrec["index"])
            h = L.to_host(it["d_h_last"]).reshape(len(nm), Wd)
            assert (h == outs[qi][starts[nrec["index"]]:starts[nrec["index"] + 1]]).all()
