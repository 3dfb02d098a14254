"""Continuous batching of general queries (lvs_submit / lvs_poll) through the
C ABI: both-encrypted, cleartext-table and banded queries, submitted at
once and while others run, with a small step cap and an arena that admits
only part of them at a time.

Bar: every result ciphertext bit-identical to the query's lone call
(lvs_edit_distance, lvs_edit_distance_clear, lvs_edit_distance_band), and
every distance equal to Wagner-Fischer."""
import time

import numpy as np
import pytest

from gpu_common import gpu, say  # noqa: F401
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu


def lone_full(g, A, m, B, n, enc):
    L, torch = g.L, g.torch
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance(g.ctx, L.to_device(A, g.dev), m, L.to_device(B, g.dev), n, enc, d_h)
    torch.cuda.synchronize()
    return L.to_host(d_h).reshape(n, L.CT_WORDS)


def pairs_ascii(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m, n = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        out.append((W.random_letters(rng, m), W.random_letters(rng, n)))
    return out


def wait_all(L, eng, tickets, limit_s=300):
    t0 = time.time()
    pending = set(tickets)
    while pending:
        assert time.time() - t0 < limit_s, "engine did not finish"
        for t in list(pending):
            if L.lvs_poll(eng, t):
                pending.discard(t)
        time.sleep(0.002)


def test_engine_both_encrypted_mid_run_join(gpu):
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    pairs = pairs_ascii(8101, 5, 4, 14)
    cts = [(L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 8200 + 2 * k),
            L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 8201 + 2 * k)) for k, (a, b) in enumerate(pairs)]
    items = []
    for (a, b), (A, B) in zip(pairs, cts):
        items.append({"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b),
                      "d_h_last": torch.zeros(len(b) * Wd, dtype=torch.int64, device=g.dev)})
    per = max(L.lvs_engine_query_bytes(it, L.LVS_ENC_ASCII7) for it in items)
    cap = 37
    say("engine: 3 ASCII queries, cap", cap, "then 2 more while they run")
    eng = L.lvs_engine_create(g.ctx, L.LVS_ENC_ASCII7, L.lvs_engine_fixed_bytes(cap) + 8 * per, max_step=cap)
    first = L.lvs_submit(eng, items[:3])
    t0 = time.time()
    while L.lvs_engine_stats(eng)[0] < 4:
        assert time.time() - t0 < 120, "engine made no progress"
        time.sleep(0.001)
    steps_at_join, _, running, _ = L.lvs_engine_stats(eng)
    assert running > 0          # the later queries join while the first ones run
    later = L.lvs_submit(eng, items[3:])
    wait_all(L, eng, first + later)
    steps, boots, active, queued = L.lvs_engine_stats(eng)
    assert (active, queued) == (0, 0)
    assert boots == sum(3 * len(a) * len(b) for a, b in pairs)
    say("engine: steps", steps, "bootstraps", boots, "joined at step", steps_at_join)
    for k, ((a, b), (A, B), it) in enumerate(zip(pairs, cts, items)):
        h = L.to_host(it["d_h_last"]).reshape(len(b), Wd)
        ref = lone_full(g, A, len(a), B, len(b), L.LVS_ENC_ASCII7)
        assert np.array_equal(h, ref), k
        assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b), k
    del eng


def test_engine_clear_and_band_queries(gpu):
    """A cleartext-table query (Section 5) and a banded query (Section 3.2)
    next to a full one, in an arena that admits one query at a time."""
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    a, b = b"levenshtein", b"leuvenshtein"
    c, d = b"kitten", b"sitting"
    alpha = bytes(sorted(set(d)))
    A = L.lvs_encrypt_string(g.ck, a, L.LVS_ENC_ASCII7, 8301)
    B = L.lvs_encrypt_string(g.ck, b, L.LVS_ENC_ASCII7, 8302)
    C = L.lvs_encrypt_string(g.ck, c, L.LVS_ENC_ASCII7, 8303)
    d_tab = torch.zeros(len(alpha) * len(c) * Wd, dtype=torch.int64, device=g.dev)
    L.lvs_preprocess(g.ctx, L.to_device(C, g.dev), len(c), L.LVS_ENC_ASCII7, alpha, d_tab)
    torch.cuda.synchronize()
    ell = L.lvs_band_exact(len(a), len(b))
    items = [
        {"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b),
         "d_h_last": torch.zeros(len(b) * Wd, dtype=torch.int64, device=g.dev)},
        {"d_a": None, "m": len(c), "d_table": d_tab, "alphabet": alpha, "b_clear": d,
         "d_h_last": torch.zeros(len(d) * Wd, dtype=torch.int64, device=g.dev)},
        {"d_a": L.to_device(A, g.dev), "m": len(a), "d_b": L.to_device(B, g.dev), "n": len(b), "ell": ell,
         "d_path": torch.zeros((len(a) + len(b)) * Wd, dtype=torch.int64, device=g.dev)},
    ]
    per = max(L.lvs_engine_query_bytes(it, L.LVS_ENC_ASCII7) for it in items)
    say("engine: full, cleartext-table and banded queries, room for one at a time")
    eng = L.lvs_engine_create(g.ctx, L.LVS_ENC_ASCII7, L.lvs_engine_fixed_bytes(4096) + per + 256, max_step=4096)
    tickets = L.lvs_submit(eng, items)
    wait_all(L, eng, tickets)
    h0 = L.to_host(items[0]["d_h_last"]).reshape(len(b), Wd)
    assert np.array_equal(h0, lone_full(g, A, len(a), B, len(b), L.LVS_ENC_ASCII7))
    d_ref = torch.zeros(len(d) * Wd, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_clear(g.ctx, d_tab, len(c), alpha, d, d_ref)
    d_pref = torch.zeros((len(a) + len(b)) * Wd, dtype=torch.int64, device=g.dev)
    L.lvs_edit_distance_band(g.ctx, L.to_device(A, g.dev), len(a), L.to_device(B, g.dev), len(b),
                             L.LVS_ENC_ASCII7, ell, d_pref)
    torch.cuda.synchronize()
    assert np.array_equal(L.to_host(items[1]["d_h_last"]), L.to_host(d_ref))
    assert np.array_equal(L.to_host(items[2]["d_path"]), L.to_host(d_pref))
    h1 = L.to_host(items[1]["d_h_last"]).reshape(len(d), Wd)
    assert L.lvs_decrypt_distance(g.ck, h1, len(c)) == P.edit_distance(c, d) == 3
    path = L.to_host(items[2]["d_path"]).reshape(len(a) + len(b), Wd)
    dist = sum(((L.lvs_lwe_decrypt(g.ck, x)[0] + 16) % 32) - 16 for x in path)
    assert dist == P.edit_distance(a, b)
    del eng


def test_engine_refusals(gpu):
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    A = L.lvs_encrypt_string(g.ck, b"abcdefgh", L.LVS_ENC_ASCII7, 8401)
    item = {"d_a": L.to_device(A, g.dev), "m": 8, "d_b": L.to_device(A, g.dev), "n": 8,
            "d_h_last": torch.zeros(8 * Wd, dtype=torch.int64, device=g.dev)}
    per = L.lvs_engine_query_bytes(item, L.LVS_ENC_ASCII7)
    eng = L.lvs_engine_create(g.ctx, L.LVS_ENC_ASCII7, L.lvs_engine_fixed_bytes(256) + per // 2, max_step=256)
    with pytest.raises(L.LvsError) as e:
        L.lvs_submit(eng, [item])
    assert e.value.code == -5
    with pytest.raises(L.LvsError) as e:
        L.lvs_submit(eng, [dict(item, d_trace=item["d_h_last"])])
    assert e.value.code == -1
    with pytest.raises(L.LvsError):
        L.lvs_poll(eng, 12345)
    assert L.lvs_engine_stats(eng)[2:] == (0, 0)
    del eng


def test_engine_dna_with_refresh(gpu):
    """DNA queries with a short refresh interval (R = 4: refresh steps inside
    every query's plan), an empty string among them: each equal to its lone
    lvs_edit_distance under the same interval."""
    g = gpu
    L, torch = g.L, g.torch
    Wd = L.CT_WORDS
    rng = np.random.default_rng(8501)
    pairs = [(W.random_dna(rng, 9), W.random_dna(rng, 13)), (W.random_dna(rng, 17), W.random_dna(rng, 6)),
             (b"", W.random_dna(rng, 5)), (W.random_dna(rng, 12), W.random_dna(rng, 12))]
    saved = L.lvs_context_get_refresh(g.ctx)
    L.lvs_context_set_refresh(g.ctx, 4)
    try:
        cts = [(L.lvs_encrypt_string(g.ck, W.dna_codes(a), L.LVS_ENC_DNA2, 8600 + 2 * k),
                L.lvs_encrypt_string(g.ck, W.dna_codes(b), L.LVS_ENC_DNA2, 8601 + 2 * k))
               for k, (a, b) in enumerate(pairs)]
        items = [{"d_a": L.to_device(A, g.dev) if len(a) else None, "m": len(a), "d_b": L.to_device(B, g.dev),
                  "n": len(b), "d_h_last": torch.zeros(len(b) * Wd, dtype=torch.int64, device=g.dev)}
                 for (a, b), (A, B) in zip(pairs, cts)]
        per = max(L.lvs_engine_query_bytes(it, L.LVS_ENC_DNA2) for it in items)
        say("engine: DNA, refresh every 4 anti-diagonals")
        eng = L.lvs_engine_create(g.ctx, L.LVS_ENC_DNA2, L.lvs_engine_fixed_bytes(512) + 4 * per, max_step=512)
        wait_all(L, eng, L.lvs_submit(eng, items))
        del eng
        for k, ((a, b), (A, B), it) in enumerate(zip(pairs, cts, items)):
            h = L.to_host(it["d_h_last"]).reshape(len(b), Wd)
            if len(a):
                ref = lone_full(g, A, len(a), B, len(b), L.LVS_ENC_DNA2)
                assert np.array_equal(h, ref), k
            assert L.lvs_decrypt_distance(g.ck, h, len(a)) == P.edit_distance(a, b), k
    finally:
        L.lvs_context_set_refresh(g.ctx, saved)
