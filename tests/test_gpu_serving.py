"""Serving (lvs_server_*): continuous batching of encrypted name queries
against a cleartext name list.  Bar: every request's result rows are
bit-identical whether it runs alone or mixed with requests arriving at other
step boundaries, equal to the single-query cleartext path (lvs_preprocess +
lvs_edit_distance_clear), and decrypt to Wagner-Fischer for every name."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu

NAMES = [b"Anna", b"Bertha", b"Cy", b"Dominik", b"Eva", b"Ann"]
QUERIES = [b"Ana", b"Bertram", b"eva", b"Dominic"]


def alphabet():
    return W.alphabet_of(NAMES)


def rows_per_name(out):
    rows, k = [], 0
    for nm in NAMES:
        rows.append(out[k:k + len(nm)])
        k += len(nm)
    return rows


def enc_queries(g):
    return [g.L.lvs_encrypt_string(g.ck, q, g.L.LVS_ENC_ASCII7, 31000 + k) for k, q in enumerate(QUERIES)]


def new_server(g, requests_that_fit=None, max_step=4096):
    L = g.L
    alpha = alphabet()
    fixed = L.lvs_server_fixed_bytes(max_step)
    per = L.lvs_server_request_bytes(NAMES, len(alpha), max(len(q) for q in QUERIES))
    pool = per * (requests_that_fit or 16) + 4096
    return L.lvs_server_create(g.ctx, NAMES, alpha, fixed + pool, max_step=max_step)


def run_alone(g, ct):
    srv = new_server(g)
    t = g.L.lvs_server_submit(srv, ct)
    while True:
        g.L.lvs_server_step(srv)
        out = g.L.lvs_server_poll(srv, t)
        if out is not None:
            return out


def check_distances(g, q, out):
    for nm, rows in zip(NAMES, rows_per_name(out)):
        assert g.L.lvs_decrypt_distance(g.ck, rows, len(q)) == P.edit_distance(q, nm), (q, nm)


@pytest.mark.parametrize("max_step", [4096, 37])
def test_alone_vs_mix(gpu, max_step):
    """Every request's rows are bit-identical alone and in a mix whose
    requests join at different step boundaries; with a cap of 37 bootstraps
    per step every phase runs in parts over several steps."""
    say("serving alone vs mix, cap", max_step)
    g = gpu
    L = g.L
    cts = enc_queries(g)
    alone = [run_alone(g, ct) for ct in cts]
    for q, out in zip(QUERIES, alone):
        check_distances(g, q, out)
    # the mix: requests join at different step boundaries
    srv = new_server(g, max_step=max_step)
    tickets = {L.lvs_server_submit(srv, cts[0]): 0}
    got = {}
    step = 0
    arrive = {1: 1, 2: 3, 3: 4}          # query -> step index at which it is submitted
    while len(got) < len(cts):
        for k, at in arrive.items():
            if at == step:
                tickets[L.lvs_server_submit(srv, cts[k])] = k
        L.lvs_server_step(srv)
        step += 1
        for t, k in list(tickets.items()):
            out = L.lvs_server_poll(srv, t)
            if out is not None:
                got[k] = out
                del tickets[t]
    for k in range(len(cts)):
        assert (got[k] == alone[k]).all(), k
    steps, pbs = L.lvs_server_stats(srv)
    alpha = alphabet()
    want = sum(2 * len(alpha) * len(q) + sum(len(q) * len(nm) for nm in NAMES) for q in QUERIES)
    assert pbs == want


def test_matches_single_query_path(gpu, okeys):
    """A request's rows equal preprocess + cleartext edit distance per name,
    and (for one name) the oracle."""
    say("serving vs single-query path")
    g = gpu
    L, torch = g.L, g.torch
    alpha = alphabet()
    q = QUERIES[0]
    ct = enc_queries(g)[0]
    out = rows_per_name(run_alone(g, ct))
    dA = L.to_device(ct, g.dev)
    d_tab = torch.zeros(len(alpha) * len(q) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, dA, len(q), L.LVS_ENC_ASCII7, alpha, d_tab)
    for nm, rows in zip(NAMES, out):
        d_h = torch.zeros(len(nm) * L.CT_WORDS, dtype=torch.int64, device=g.dev)
        L.lvs_edit_distance_clear(g.ctx, d_tab, len(q), alpha, nm, d_h)
        torch.cuda.synchronize()
        assert (L.to_host(d_h).reshape(len(nm), L.CT_WORDS) == rows).all(), nm
    oA = OL.encrypt_string(okeys, q, OL.ENC_ASCII7, 31000)
    otab = OL.preprocess(okeys, oA, alpha, OL.ENC_ASCII7)
    nm = NAMES[2]
    oh = OL.edit_distance_clear(okeys, otab, alpha, nm, OL.ENC_ASCII7)
    for j in range(len(nm)):
        assert_same_ct(out[2][j], oh[j], f"{nm}[{j}]")


def test_admission_by_device_memory(gpu):
    """A pool that holds one request at a time: the others wait in the queue
    and still finish with the same results."""
    say("serving admission")
    g = gpu
    L = g.L
    cts = enc_queries(g)[:3]
    srv = new_server(g, requests_that_fit=1)
    tickets = [L.lvs_server_submit(srv, ct) for ct in cts]
    active, queued, _ = L.lvs_server_step(srv)
    assert active == 1 and queued == 2
    outs = {}
    while len(outs) < len(cts):
        L.lvs_server_step(srv)
        for k, t in enumerate(tickets):
            if k not in outs:
                out = L.lvs_server_poll(srv, t)
                if out is not None:
                    outs[k] = out
    for k, ct in enumerate(cts):
        assert (outs[k] == run_alone(g, ct)).all()


def test_request_that_never_fits(gpu):
    g = gpu
    L = g.L
    srv = new_server(g, requests_that_fit=1)
    big = L.lvs_encrypt_string(g.ck, b"x" * 40, L.LVS_ENC_ASCII7, 1)
    with pytest.raises(L.LvsError) as e:
        L.lvs_server_submit(srv, big)
    assert e.value.code == -5


def test_step_below_cap_with_more_splits(gpu):
    """A step smaller than the cap can split the key switch more ways than a
    step at the cap (about 600 preprocessing bootstraps under a 8192 cap):
    the partial sums must still fit the server's fixed region.  Steps end on
    whole device rounds and run every bootstrap once."""
    say("serving step below cap")
    g = gpu
    L = g.L
    alpha = alphabet()
    q = (b"AnnaBerthaCyDominikEvaAnnBertha" * 2)[:600 // len(alpha) + 1]
    ct = L.lvs_encrypt_string(g.ck, q, L.LVS_ENC_ASCII7, 777)
    max_step = 8192
    per = L.lvs_server_request_bytes(NAMES, len(alpha), len(q))
    srv = L.lvs_server_create(g.ctx, NAMES, alpha, L.lvs_server_fixed_bytes(max_step) + 2 * per + 4096,
                              max_step=max_step)
    t = L.lvs_server_submit(srv, ct)
    out = None
    sizes = []
    while out is None:
        sizes.append(L.lvs_server_step(srv)[2])
        out = L.lvs_server_poll(srv, t)
    check_distances(g, q, out)
    # steps past one device round end on whole rounds (one bootstrap per CU):
    # the first preprocessing round (17 letters x 36 = 612 bootstraps) runs
    # as 512 + 100
    cus = g.torch.cuda.get_device_properties(g.dev).multi_processor_count
    assert all(n <= cus or n % cus == 0 for n in sizes), sizes
    assert sum(sizes) == 2 * len(alpha) * len(q) + sum(len(q) * len(nm) for nm in NAMES)
