#!/usr/bin/env python3
"""Benchmark of the Leuvenshtein hot path on one MI355X.

Workload: the batched configuration -- 256 pairs of ASCII strings, lengths
uniform in [8, 64] (uniform letters), both strings encrypted, as one batch
plan: step t bootstraps every ready cell of anti-diagonal t of every query
(one bootstrap per cell, Algorithm 1/4) together with the equality
bootstraps of the next diagonals (2 per character pair, Algorithm 3), in one
key-switch launch and one blind-rotation launch (Section 6.2: the cells of
one anti-diagonal are independent).  A benchmark step is one such plan step;
the W warm-up steps start an execution of the plan, the K timed steps
continue it, and the execution is then completed untimed and every distance
checked.  The encrypted strings are resident in HBM when the timed region
starts.

Prints one JSON line.  value = bootstraps per second over the K timed
steps; full_pass = the whole plan as one HIP graph replay (all 256 queries);
plain = the same 256 queries one at a time through the plain per-diagonal
path (identical work); roofline = the blind-rotation kernel's integer
multiplies per second over the timed region (HIP events around its launches
on the context's stream) against the chip's 32-bit VALU multiply peak; the
other configurations follow (the 256 x 256 DNA alignment, the tiny DNA pair,
the 32 x 32 plain pair, serving against 1024 cleartext names);
cpu_baseline = the oracle's bootstraps per second on the host cores for a
bounded sample of the same workload's bootstraps.
"""
import argparse
import hashlib
import json
import os
import sys
import statistics
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one bootstrap (n = 742 external products, 4 primes):
# per prime and step, 4 length-2048 NTTs of 11 * 1024 butterflies plus the
# 2 x 2 products with the GGSW row over 2048 positions = 53248 modular
# multiplications; each needs 3 32-bit multiplies (Shoup / Montgomery).
MODMUL_PER_PBS = 742 * 4 * (4 * 11 * 1024 + 4 * 2048)
INT_MUL_PER_PBS = 3 * MODMUL_PER_PBS
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit multiply per lane per cycle
# (v_mul_lo_u32 / v_mul_hi_u32 issue at the full VALU rate on gfx950).
VALU_INT_MUL_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic HBM bytes of one blind-rotation launch: the NTT-domain
# bootstrapping key once (742 GGSW x 4 primes x 2 rows x 2 polynomials x 2048
# u32 residues), shared by every bootstrap of the launch, plus per bootstrap
# its key-switched input (743 u64) and its extracted output (2049 u64).
BSK_BYTES = 742 * 4 * 2 * 2 * 2048 * 4
IO_BYTES_PER_PBS = (743 + 2049) * 8
HBM_PEAK_GBS = 8000.0


def note(msg):
    """Progress on stderr; stdout carries only the result line."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    with open(os.path.join(ROOT, "paper_2508_14568_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_launch(kernel, avg_pbs_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is absent or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "blind_rotate_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_hip_sha256") != kernel_source_digest() or kernel not in t.get("bytes_per_pbs", {}):
        return None
    return round(t["bytes_per_pbs"][kernel] * avg_pbs_per_launch)


def hbm_roofline(pbs_per_launch, launch_ms):
    """The same launches against the HBM peak: algorithmic bytes (key once
    per launch, inputs and outputs per bootstrap) over the launch time."""
    nbytes = BSK_BYTES + IO_BYTES_PER_PBS * pbs_per_launch
    gbs = nbytes / (launch_ms / 1e3) / 1e9
    return {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
            "bytes_per_launch": round(nbytes)}


def cpu_baseline(workload_cts, source):
    """Oracle bootstraps per second on this host's cores (bounded sample)."""
    from oracle import leuvenshtein as OL
    from oracle import tfhe as OT
    import numpy as np
    threads = OT.default_threads()
    note(f"cpu baseline: oracle on {threads} threads")
    keys = OT.Keys(OT.default_params(), seed=1, nthreads=threads)
    polys = OL.lut_polys(keys.N)
    sample = workload_cts[: 2 * threads]
    t0 = time.perf_counter()
    ref = keys.pbs_batch(sample, polys, OL.LUT_IDS["eq"], threads)
    dt = time.perf_counter() - t0
    # the same bootstraps with the oracle's Karatsuba products (same words)
    kkeys = OT.Keys(OT.default_params(), seed=1, nthreads=threads, karatsuba=True)
    t0 = time.perf_counter()
    kref = kkeys.pbs_batch(sample, polys, OL.LUT_IDS["eq"], threads)
    dtk = time.perf_counter() - t0
    if not np.array_equal(ref, kref):
        raise SystemExit("cpu baseline: the oracle's two products disagree")
    return {"value": round(len(sample) / dt, 3), "unit": "PBS/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} equality bootstraps of {source} "
                      f"(z1 = x1_i - y1_j, LUT_eq), {threads} threads, {dt:.1f} s wall, schoolbook products",
            "karatsuba": {"value": round(len(sample) / dtk, 3), "unit": "PBS/s", "seconds": round(dtk, 2)}}


def levenshtein(a, b) -> int:
    """Cleartext distance, to check the decrypted results (two-row DP)."""
    prev = list(range(len(b) + 1))
    for i, x in enumerate(a, 1):
        cur = [i] + [0] * len(b)
        for j, y in enumerate(b, 1):
            cur[j] = prev[j - 1] if x == y else 1 + min(prev[j], cur[j - 1], prev[j - 1])
        prev = cur
    return prev[-1]


def plain_path_time(L, ctx, items, label):
    """Every query of items (dicts with d_a, m, d_b, n, d_h_last; ASCII,
    both encrypted) once through the plain per-diagonal path into its
    d_h_last, after one warm-up call: (seconds, bootstraps).  Buffers are set
    up outside the timing."""
    import torch
    dev = ctx.device
    t_plain, pbs_plain = 0.0, 0
    for k, it in enumerate([items[0]] + list(items)):
        work = L.device_buffer(L.lvs_edit_distance_workspace_bytes(it["m"], it["n"], L.LVS_ENC_ASCII7), dev)
        d_h = it["d_h_last"]
        d_h.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.lvs_edit_distance(ctx, it["d_a"], it["m"], it["d_b"], it["n"], L.LVS_ENC_ASCII7, d_h, work)
        torch.cuda.synchronize()
        if k == 0:
            continue                  # warm-up
        t_plain += time.perf_counter() - t0
        pbs_plain += 3 * it["m"] * it["n"]
        if k % 16 == 0:
            note(f"{label}: {k} of {len(items)} queries through the plain path")
    return t_plain, pbs_plain


def encrypt_pairs(L, ck, pairs, seed0, dev, enc=None):
    """Device items (d_a, m, d_b, n, d_h_last) of encrypted string pairs."""
    import torch
    enc = L.LVS_ENC_ASCII7 if enc is None else enc
    items = []
    for k, (a, b) in enumerate(pairs):
        dA = L.to_device(L.lvs_encrypt_string(ck, a, enc, seed0 + 2 * k), dev)
        dB = L.to_device(L.lvs_encrypt_string(ck, b, enc, seed0 + 2 * k + 1), dev)
        items.append({"d_a": dA, "m": len(a), "d_b": dB, "n": len(b),
                      "d_h_last": torch.zeros(max(1, len(b)) * L.CT_WORDS, dtype=torch.int64, device=dev)})
    return items


def check_distances(L, ck, pairs, items, what):
    for k, ((a, b), it) in enumerate(zip(pairs, items)):
        h = L.to_host(it["d_h_last"]).reshape(-1, L.CT_WORDS)[:len(b)]
        if L.lvs_decrypt_distance(ck, h, len(a)) != levenshtein(a, b):
            raise SystemExit(f"{what}: wrong distance for pair {k}")


def kernel_roofline(L, ctx, steps):
    """The blind-rotation form with the most time among the launches profiled
    since lvs_profile_enable: its integer multiplies per second (HIP events
    around each launch on the context's stream) against the multiply peak."""
    forms = {name: L.lvs_profile_read(ctx, k) for name, k in
             (("blind_rotate_latency_kernel", L.KERNEL_BLIND_ROTATE_LATENCY),
              ("blind_rotate_kernel", L.KERNEL_BLIND_ROTATE_THROUGHPUT),
              ("blind_rotate_w16_kernel", L.KERNEL_BLIND_ROTATE_W16),
              ("blind_rotate_pair_kernel", L.KERNEL_BLIND_ROTATE_PAIR))}
    br_ms, _, _ = L.lvs_profile_read(ctx, L.KERNEL_BLIND_ROTATE)
    ks_ms, _, _ = L.lvs_profile_read(ctx, L.KERNEL_KEYSWITCH)
    kname = max(forms, key=lambda k: forms[k][0])
    k_ms, k_launches, k_pbs = forms[kname]
    if k_launches == 0 or k_ms <= 0:
        raise SystemExit("no blind-rotation launch was timed")
    avg_launch_ms = k_ms / max(1, k_launches)
    avg_pbs_launch = k_pbs / max(1, k_launches)
    achieved = INT_MUL_PER_PBS * avg_pbs_launch / (avg_launch_ms / 1000) / 1e12
    return {
        "bound": "alu", "kernel": kname,
        "achieved": round(achieved, 3), "peak": round(VALU_INT_MUL_PEAK_TOPS, 3), "unit": "TOP/s",
        "frac": round(achieved / VALU_INT_MUL_PEAK_TOPS, 4),
        "traffic": traffic_per_launch(kname, avg_pbs_launch),
        "ops": "32-bit integer multiplies, 3 per modular multiplication, "
               f"{INT_MUL_PER_PBS} per bootstrap",
        "avg_launch_ms": round(avg_launch_ms, 4), "launches": k_launches,
        "avg_pbs_per_launch": round(avg_pbs_launch, 2),
        "hbm": hbm_roofline(avg_pbs_launch, avg_launch_ms),
        "other_form": {k: {"ms_per_step": round(v[0] / steps, 3), "launches": v[1], "pbs": v[2]}
                       for k, v in forms.items() if k != kname},
        "keyswitch_ms_per_step": round(ks_ms / steps, 3),
        "blind_rotate_ms_per_step": round(br_ms / steps, 3),
    }


def run_global_steps(L, plan, nsteps, g0, g1):
    """Plan steps g0 .. g1 - 1 of a sequence of executions (global step g is
    step g % nsteps of execution g // nsteps)."""
    g = g0
    while g < g1:
        first = g % nsteps
        count = min(nsteps - first, g1 - g)
        L.lvs_plan_run_steps(plan, first, count)
        g += count


def batched_headline(L, ck, ctx, warmup, steps, plain_sample, only_timed=False):
    """The 256-pair batched workload: K timed plan steps after W warm-up
    steps (the value), the whole plan as one graph replay, and the same
    queries through the plain per-diagonal path."""
    import torch
    import workloads as W
    pairs = W.batched()
    dev = ctx.device
    note("batched: encrypting 256 pairs")
    items = encrypt_pairs(L, ck, pairs, 20000, dev)
    note("batched: plan (256 queries, graph captured)")
    plan = L.lvs_plan_create(ctx, items, L.LVS_ENC_ASCII7, graph=True)
    nsteps, pbs, max_step = L.lvs_plan_info(plan)
    sizes = L.lvs_plan_step_bootstraps(plan)
    cells = sum(len(a) * len(b) for a, b in pairs)
    # warm-up steps, then the timed steps, continuing the same execution
    note(f"batched: {warmup} warm-up plan steps, {steps} timed")
    run_global_steps(L, plan, nsteps, 0, warmup)
    torch.cuda.synchronize()
    L.lvs_profile_enable(ctx, True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    assert stream.cuda_stream == ctx.stream_handle, "the context runs on torch's current stream"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    run_global_steps(L, plan, nsteps, warmup, warmup + steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_ms = start.elapsed_time(end)
    roofline = kernel_roofline(L, ctx, steps)
    L.lvs_profile_enable(ctx, False)
    timed_pbs = sum(sizes[g % nsteps] for g in range(warmup, warmup + steps))
    if only_timed:
        return {"timed_pbs": timed_pbs, "timed_ms": round(timed_ms, 3), "roofline": roofline}, None, None
    # complete the execution the timed steps belong to, then check it
    g_end = warmup + steps
    run_global_steps(L, plan, nsteps, g_end, -(-g_end // nsteps) * nsteps)
    torch.cuda.synchronize()
    check_distances(L, ck, pairs, items, "batched (steps)")
    head = {"timed_pbs": timed_pbs, "timed_ms": round(timed_ms, 3), "wall_s": round(wall, 3),
            "plan_steps": nsteps, "plan_pbs": pbs, "max_step": max_step, "cells": cells,
            "timed_step_range": [warmup % nsteps, (warmup + steps - 1) % nsteps],
            "roofline": roofline}
    # the whole plan as one graph replay
    note("batched: whole plan, one graph replay")
    for it in items:
        it["d_h_last"].zero_()
    L.lvs_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g_ms, g_runs, _ = L.lvs_profile_read(ctx, L.KERNEL_GRAPH)
    L.lvs_profile_enable(ctx, False)
    check_distances(L, ck, pairs, items, "batched (graph)")
    del plan
    full = {"queries": 256, "pbs": pbs, "cells": cells, "steps": nsteps, "seconds": round(dt, 3),
            "graph_ms": round(g_ms / max(1, g_runs), 3), "pbs_per_s": round(pbs / dt, 1),
            "cells_per_s": round(cells / dt, 1), "queries_per_s": round(256 / dt, 3),
            "roofline_graph": {"bound": "alu",
                               "achieved": round(INT_MUL_PER_PBS * pbs / (g_ms / g_runs / 1e3) / 1e12, 3),
                               "peak": round(VALU_INT_MUL_PEAK_TOPS, 3), "unit": "TOP/s",
                               "frac": round(INT_MUL_PER_PBS * pbs / (g_ms / g_runs / 1e3) / 1e12
                                             / VALU_INT_MUL_PEAK_TOPS, 4)}}
    # the same 256 queries one at a time through the plain path
    n_plain = 256 if plain_sample <= 0 else min(plain_sample, 256)
    note(f"batched: {n_plain} queries through the plain path")
    t_plain, pbs_plain = plain_path_time(L, ctx, items[:n_plain], "plain")
    check_distances(L, ck, pairs[:n_plain], items[:n_plain], "plain path")
    plain_pbs_s = pbs_plain / t_plain
    plain = {"queries": n_plain, "identical_work": n_plain == 256, "pbs": pbs_plain, "seconds": round(t_plain, 3),
             "pbs_per_s": round(plain_pbs_s, 1), "queries_per_s": round(n_plain / t_plain, 4),
             "batched_speedup": round(full["pbs_per_s"] / plain_pbs_s, 2)}
    return head, full, plain


def plain_config(L, ck, ctx, a, b, enc, seed, reps=5):
    """One pair through the plain per-diagonal path, after a warm-up run:
    bootstraps per second at the median of reps timed runs (each its own
    interval), the fastest and slowest run, and the checked distance."""
    import torch
    dev = ctx.device
    sa, sb = (W_codes(a), W_codes(b)) if enc == L.LVS_ENC_DNA2 else (a, b)
    dA = L.to_device(L.lvs_encrypt_string(ck, sa, enc, seed), dev)
    dB = L.to_device(L.lvs_encrypt_string(ck, sb, enc, seed + 1), dev)
    d_h = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=dev)
    work = L.device_buffer(L.lvs_edit_distance_workspace_bytes(len(a), len(b), enc), dev)
    L.lvs_edit_distance(ctx, dA, len(a), dB, len(b), enc, d_h, work)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        L.lvs_edit_distance(ctx, dA, len(a), dB, len(b), enc, d_h, work)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = statistics.median(times)
    d = L.lvs_decrypt_distance(ck, L.to_host(d_h).reshape(len(b), L.CT_WORDS), len(a))
    if d != levenshtein(a, b):
        raise SystemExit("plain config: wrong distance")
    per_cell = 3 if enc == L.LVS_ENC_ASCII7 else 2
    R = L.lvs_context_get_refresh(ctx)
    pbs = per_cell * len(a) * len(b) + refresh_pbs(len(a), len(b), R)
    return {"m": len(a), "n": len(b), "pbs": pbs, "seconds": round(dt, 4), "pbs_per_s": round(pbs / dt, 1),
            "cells_per_s": round(len(a) * len(b) / dt, 1), "distance": d, "runs": reps,
            "seconds_min": round(min(times), 4), "seconds_max": round(max(times), 4), "refresh_every": R}


def W_codes(s):
    import workloads as W
    return W.dna_codes(s)


def serving_block(L, ck, ctx, n_names, n_sat, n_poisson, rhos, progress=False, arena_gb=4, max_step=1024,
                  poisson_seed=6, query_offset=0, arrival_rate=None, stream=None):
    """The serving workload on the first n_names of its 1024 cleartext server
    names: n_sat queries submitted at once (saturated queries/s), then
    n_poisson queries per load factor rho arriving as a Poisson process at
    rho x the saturated rate for their own mix (the saturated run's bootstrap
    rate over their mean bootstraps per query; p50/p99 latency from arrival to results on the
    host).  Every query's distances to every name are checked."""
    import numpy as np
    import workloads as W
    from paper_2508_14568_amd import serving as S
    # the workload's query stream, from query_offset on (a later run draws later queries)
    server, queries = W.serving(n_queries=query_offset + 1 + n_sat + n_poisson * len(rhos))
    queries = queries[query_offset:]
    names = server[:n_names]
    alpha = W.alphabet_of(names)
    cts = [L.lvs_encrypt_string(ck, q, L.LVS_ENC_ASCII7, 40000 + k) for k, q in enumerate(queries)]
    per = L.lvs_server_request_bytes(names, len(alpha), max(len(q) for q in queries))
    cap = max(4, min(128, (arena_gb << 30) // per))
    srv = L.lvs_server_create(ctx, names, alpha, L.lvs_server_fixed_bytes(max_step) + per * cap + 4096,
                              max_step=max_step)

    def check(k, out, lat=None):
        q, row = queries[k], 0
        for nm in names:
            if L.lvs_decrypt_distance(ck, out[row:row + len(nm)], len(q)) != levenshtein(q, nm):
                raise SystemExit(f"serving: wrong distance for query {k}")
            row += len(nm)
        if progress:
            note(f"serving: query {k} done")
        if stream and lat is not None:        # each Poisson query as it finishes
            with open(stream, "a") as f:
                f.write(json.dumps({"query": query_offset + k, "latency_s": round(lat, 4)}) + "\n")

    S.run(srv, cts[:1], [0.0], on_result=lambda k, o, t: check(k, o))            # warm-up
    res = {
        "workload": f"serving: first {n_names} of 1024 cleartext names (lengths lognormal, mean 15), "
                    f"alphabet {len(alpha)} letters, encrypted queries of the same length law",
        "names": n_names, "alphabet": len(alpha), "max_requests_resident": cap, "max_step": max_step,
        "request_bytes": per, "poisson": [],
    }
    sat_qps = None
    if n_sat > 0:
        st0, pbs0 = L.lvs_server_stats(srv)
        note(f"serving: {n_names} names, saturated run of {n_sat} queries")
        lat, wall, _ = S.run(srv, cts[1:1 + n_sat], [0.0] * n_sat, on_result=lambda k, o, t: check(1 + k, o))
        st1, pbs1 = L.lvs_server_stats(srv)
        sat_qps = n_sat / wall
        res["saturated"] = {"queries": n_sat, "seconds": round(wall, 3), "queries_per_s": round(sat_qps, 4),
                            "pbs_per_s": round((pbs1 - pbs0) / wall, 1), "steps": st1 - st0,
                            "pbs_per_query": round((pbs1 - pbs0) / n_sat, 1),
                            **{k: round(v, 3) for k, v in S.percentiles(lat).items()}}
        res["latency_note"] = "seconds from submission to results on the host; with few samples p99 is the maximum"
        # the workload's own query mix (first 200 queries of its stream): mean bootstraps per query and the
        # saturated query rate the measured bootstrap rate gives for that mix
        _, mix = W.serving(n_queries=200)
        tot = sum(len(nm) for nm in names)
        mean_pbs = float(np.mean([2 * len(alpha) * len(q) + len(q) * tot for q in mix]))
        res["saturated"]["workload_mean_pbs_per_query"] = round(mean_pbs, 1)
        res["saturated"]["workload_queries_per_s"] = round(res["saturated"]["pbs_per_s"] / mean_pbs, 4)
    base = 1 + n_sat
    tot = sum(len(nm) for nm in names)
    for r, rho in enumerate(rhos if n_poisson > 0 else []):
        idx = range(base + r * n_poisson, base + (r + 1) * n_poisson)
        # load rho for the queries that will arrive: the measured bootstrap rate
        # over their own mean bootstraps per query (the saturated run's queries
        # are a different, smaller sample of the length law)
        mean_r = float(np.mean([2 * len(alpha) * len(queries[k]) + len(queries[k]) * tot for k in idx]))
        if not arrival_rate and sat_qps is None:
            raise SystemExit("serving: Poisson arrivals need a saturated run or --arrival-rate")
        rate = arrival_rate if arrival_rate else rho * res["saturated"]["pbs_per_s"] / mean_r
        arr = W.poisson_arrivals(poisson_seed + r, rate, n_poisson)
        note(f"serving: Poisson arrivals at {rate:.4f} queries/s (rho={rho}), {n_poisson} queries")
        st0, pbs0 = L.lvs_server_stats(srv)
        if stream:
            with open(stream, "a") as f:
                f.write(json.dumps({"names": n_names, "rate_per_s": round(rate, 5), "rho": rho,
                                    "arrival_seed": poisson_seed + r, "queries": n_poisson,
                                    "first_query": query_offset + idx.start, "max_step": max_step}) + "\n")
        lat, wall, _ = S.run(srv, [cts[k] for k in idx], list(arr),
                             on_result=lambda k, o, t, b=idx.start: check(b + k, o, t))
        st1, pbs1 = L.lvs_server_stats(srv)
        res["poisson"].append({"rho": rho, "queries": n_poisson, "rate_per_s": round(rate, 4),
                               "mean_pbs_per_query": round(mean_r, 1),
                               "arrival_seed": poisson_seed + r, "query_offset": query_offset,
                               "latencies_s": [round(x, 3) for x in lat],
                               "seconds": round(wall, 3), "pbs_per_s": round((pbs1 - pbs0) / wall, 1),
                               **{k: round(v, 3) for k, v in S.percentiles(lat).items()},
                               "mean": round(float(np.mean(lat)), 3)})
    return res


def band_block(L, ck, ctx, nq, approx_ell):
    """Section 3.2's skipping on the batched workload's first nq pairs: the
    exact band (max(m, n) - floor(min(m, n) / 2), the whole matrix when the
    lengths are far apart) and a fixed half-width, each as one graph plan,
    against the full-matrix plan of the same queries."""
    import torch
    import workloads as W
    pairs = W.batched()[:nq]
    dev = ctx.device
    enc = [(L.to_device(L.lvs_encrypt_string(ck, a, L.LVS_ENC_ASCII7, 50000 + 2 * k), dev),
            L.to_device(L.lvs_encrypt_string(ck, b, L.LVS_ENC_ASCII7, 50001 + 2 * k), dev))
           for k, (a, b) in enumerate(pairs)]
    res = {"workload": f"batched_ascii first {nq} of 256 pairs, lengths 8..64", "queries": nq}
    for name, ell_of in (("full", None), ("exact_band", lambda m, n: L.lvs_band_exact(m, n)),
                         (f"band_{approx_ell}", lambda m, n: approx_ell)):
        items = []
        for (a, b), (dA, dB) in zip(pairs, enc):
            it = {"d_a": dA, "m": len(a), "d_b": dB, "n": len(b)}
            if ell_of is None:
                it["d_h_last"] = torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=dev)
            else:
                it["ell"] = ell_of(len(a), len(b))
                it["d_path"] = torch.zeros((len(a) + len(b)) * L.CT_WORDS, dtype=torch.int64, device=dev)
            items.append(it)
        note(f"band: {name} plan")
        plan = L.lvs_plan_create(ctx, items, L.LVS_ENC_ASCII7, graph=True)
        steps, pbs, _ = L.lvs_plan_info(plan)
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.lvs_plan_run(plan)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        exact = over = 0
        for (a, b), it in zip(pairs, items):
            if ell_of is None:
                d = L.lvs_decrypt_distance(ck, L.to_host(it["d_h_last"]).reshape(len(b), L.CT_WORDS), len(a))
            else:
                d = L.lvs_decrypt_distance(ck, L.to_host(it["d_path"]).reshape(-1, L.CT_WORDS), 0)
            wf = levenshtein(a, b)
            if d < wf or (name != f"band_{approx_ell}" and d != wf):
                raise SystemExit(f"band: wrong distance ({name})")
            exact += d == wf
            over += d > wf
        res[name] = {"pbs": pbs, "steps": steps, "seconds": round(dt, 3), "pbs_per_s": round(pbs / dt, 1),
                     "queries_per_s": round(nq / dt, 3), "exact_results": exact, "overestimates": over}
        del plan
    res["exact_band_pbs_saving"] = round(1 - res["exact_band"]["pbs"] / res["full"]["pbs"], 4)
    res["exact_band_speedup"] = round(res["full"]["seconds"] / res["exact_band"]["seconds"], 3)
    return res


def refresh_pbs(m, n, every):
    """Bootstraps of Section 3.1's refresh steps on an m x n matrix: two per
    cell of every anti-diagonal s = every, 2 every, ... below m + n."""
    if every <= 0:
        return 0
    return sum(2 * (min(m, s - 1) - max(1, s - n) + 1) for s in range(every, m + n, every))


def wide_block(L, ck, ctx):
    """Section 4.2's wide-symbol path: a 32 x 32 pair of 21-bit symbols
    (hybrid equality, one bootstrap per 4-bit chunk plus the merges, then the
    main loop), one edit distance timed after a warm-up run."""
    import torch
    import workloads as W
    width = 21
    a, b = W.wide_symbols(width=width)
    m, n = len(a), len(b)
    dev = ctx.device
    dA = L.to_device(L.lvs_encrypt_symbols(ck, a, width, 60001), dev)
    dB = L.to_device(L.lvs_encrypt_symbols(ck, b, width, 60002), dev)
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=dev)
    work = L.device_buffer(L.lvs_edit_distance_wide_workspace_bytes(m, n, width), dev)
    note("wide: 32 x 32, 21-bit symbols")
    L.lvs_edit_distance_wide(ctx, dA, m, dB, n, width, d_h, work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.lvs_edit_distance_wide(ctx, dA, m, dB, n, width, d_h, work)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = L.lvs_decrypt_distance(ck, L.to_host(d_h).reshape(n, L.CT_WORDS), m)
    if d != levenshtein(a, b):
        raise SystemExit("wide: wrong distance")
    per_pair = L.lvs_wide_pbs_per_pair(width)
    pbs = m * n * (per_pair + 1) + refresh_pbs(m, n, L.lvs_context_get_refresh(ctx))
    return {"workload": f"wide_symbols {m}x{n}, {width}-bit symbols over 64 code points, 20% copied, seed 7",
            "equality_pbs_per_pair": per_pair, "pbs": pbs, "seconds": round(dt, 3), "pbs_per_s": round(pbs / dt, 1),
            "cells_per_s": round(m * n / dt, 1), "distance": d}


def full_configs(L, ck, ctx, serving_sat, serving_poisson):
    """The workloads the default line leaves out, at full size (a run of
    several minutes): the cleartext-string variant of the batched workload
    (Section 5 preprocessing of every query, then one plan) and longer
    serving runs against the 1024 names.  Returns a dict keyed by workload."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2508_14568_amd import serving as S
    dev = ctx.device
    out = {}

    pairs = W.batched()

    # the cleartext-string variant: preprocessing of every a over the 52 letters, then one plan
    alpha = W.LETTERS
    note("full: cleartext variant, preprocessing 256 queries")
    tabs, t_pre, pbs_pre = [], 0.0, 0
    for k, (a, b) in enumerate(pairs):
        dA = L.to_device(L.lvs_encrypt_string(ck, a, L.LVS_ENC_ASCII7, 90000 + k), dev)
        d_tab = torch.zeros(len(alpha) * len(a) * L.CT_WORDS, dtype=torch.int64, device=dev)
        work = L.device_buffer(L.lvs_preprocess_workspace_bytes(len(a), len(alpha), L.LVS_ENC_ASCII7), dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.lvs_preprocess(ctx, dA, len(a), L.LVS_ENC_ASCII7, alpha, d_tab, work)
        torch.cuda.synchronize()
        t_pre += time.perf_counter() - t0
        pbs_pre += 2 * len(alpha) * len(a)
        tabs.append(d_tab)
        del work
    citems = [{"d_a": None, "m": len(a), "d_table": t, "alphabet": alpha, "b_clear": b,
               "d_h_last": torch.zeros(len(b) * L.CT_WORDS, dtype=torch.int64, device=dev)}
              for (a, b), t in zip(pairs, tabs)]
    note("full: cleartext variant, plan run")
    plan = L.lvs_plan_create(ctx, citems, L.LVS_ENC_ASCII7, graph=True)
    steps, cpbs, _ = L.lvs_plan_info(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.lvs_plan_run(plan)
    torch.cuda.synchronize()
    dtc = time.perf_counter() - t0
    for (a, b), it in zip(pairs, citems):
        h = L.to_host(it["d_h_last"]).reshape(len(b), L.CT_WORDS)
        if L.lvs_decrypt_distance(ck, h, len(a)) != levenshtein(a, b):
            raise SystemExit("cleartext 256: wrong distance")
    del plan, citems, tabs
    out["batched_cleartext_256"] = {"pre_pbs": pbs_pre, "pre_seconds": round(t_pre, 3),
                                    "pre_pbs_per_s": round(pbs_pre / t_pre, 1),
                                    "main_pbs": cpbs, "main_seconds": round(dtc, 3),
                                    "main_pbs_per_s": round(cpbs / dtc, 1),
                                    "main_queries_per_s": round(256 / dtc, 3)}

    # serving against the full list of 1024 names
    out["serving_1024"] = serving_block(L, ck, ctx, 1024, serving_sat, serving_poisson, [0.8], progress=True,
                                        arena_gb=32)
    return out


def microbench(L, ctx):
    """Measured ceilings: the butterfly instruction mix from registers on
    every CU, and a 1 GiB device copy."""
    import torch
    ms, muls = L.lvs_microbench_modmul(ctx, 4096)
    nbytes = 1 << 30
    src = torch.zeros(nbytes // 8, dtype=torch.int64, device=ctx.device)
    dst = torch.empty_like(src)
    copy_ms = L.lvs_microbench_copy(ctx, src, dst, nbytes, 5)
    del src, dst
    return {"modmul_probe_tops": round(muls / (ms / 1e3) / 1e12, 3),
            "copy_gbs": round(2 * nbytes / (copy_ms / 1e3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed plan steps of the batched workload")
    ap.add_argument("--warmup", type=int, default=5, help="plan steps run before the timed ones")
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="batched queries also timed through the plain path (0: all 256, identical work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-names", type=int, default=1024)
    ap.add_argument("--serving-queries", type=int, default=2, help="queries of the saturated run")
    ap.add_argument("--serving-progress", action="store_true", help="a progress line per finished query")
    ap.add_argument("--serving-max-step", type=int, default=1024,
                    help="bootstraps per engine step at most (admitted requests beyond it wait a step)")
    ap.add_argument("--poisson-queries", type=int, default=0, help="queries per load factor")
    ap.add_argument("--rho", type=str, default="0.8", help="comma-separated load factors")
    ap.add_argument("--poisson-seed", type=int, default=6, help="seed of the first load factor's arrivals")
    ap.add_argument("--query-offset", type=int, default=0, help="first query of the serving workload's stream")
    ap.add_argument("--arrival-rate", type=float, default=None,
                    help="Poisson arrival rate in queries/s (default: rho x the saturated rate)")
    ap.add_argument("--serving-stream", type=str, default=None,
                    help="file that receives one JSON line per finished Poisson query")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--band-queries", type=int, default=0, help="the band modes on this many batched pairs")
    ap.add_argument("--band-ell", type=int, default=4, help="half-width of the approximate band")
    ap.add_argument("--wide", action="store_true", help="also the 32 x 32 wide-symbol pair")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--tuning", type=str, default=None,
                    help="launch shape as JSON (lvs_tuning fields) instead of the autotuner's")
    ap.add_argument("--no-microbench", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="only the serving block (latency studies)")
    ap.add_argument("--timed-only", action="store_true",
                    help="only the warm-up and timed plan steps (for profiling their launches)")
    ap.add_argument("--full-configs", action="store_true",
                    help="instead of the default line: the cleartext-string variant and longer serving runs")
    ap.add_argument("--full-serving-queries", type=int, default=8)
    ap.add_argument("--full-poisson-queries", type=int, default=16)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be positive and --warmup not negative")

    import numpy as np
    import torch
    from paper_2508_14568_amd import lvs as L
    import workloads as W

    params = L.lvs_params_default()
    ck, sk = L.lvs_keygen(params, 1)
    ctx = L.lvs_context_create(sk, params, 0)
    tuning = None
    if args.tuning:
        L.lvs_context_set_tuning(ctx, dict(L.lvs_context_get_tuning(ctx), **json.loads(args.tuning)))
        tuning = {"tuning": L.lvs_context_get_tuning(ctx), "cached": False, "given": True}
    elif not args.no_autotune:
        note("autotune")
        tuning = L.autotune(ctx)
    if args.serving_only:
        res = serving_block(L, ck, ctx, args.serving_names, args.serving_queries, args.poisson_queries,
                            [float(x) for x in args.rho.split(",") if x], max_step=args.serving_max_step,
                            progress=args.serving_progress, arena_gb=32 if args.serving_names > 256 else 4,
                            poisson_seed=args.poisson_seed, query_offset=args.query_offset,
                            arrival_rate=args.arrival_rate, stream=args.serving_stream)
        print(json.dumps({"serving": res, "tuning": tuning and tuning["tuning"]}), flush=True)
        return
    if args.full_configs:
        res = full_configs(L, ck, ctx, args.full_serving_queries, args.full_poisson_queries)
        print(json.dumps({"full_configs": res, "tuning": tuning and tuning["tuning"]}), flush=True)
        return

    head, full, plain = batched_headline(L, ck, ctx, args.warmup, args.steps, args.plain_sample, args.timed_only)
    if args.timed_only:
        if not args.no_microbench:
            head["roofline"]["measured"] = microbench(L, ctx)     # the copy kernel calibrates traffic counters
        pbs_s = head["timed_pbs"] / (head["timed_ms"] / 1e3)
        print(json.dumps({"workload": "batched_ascii_256_pairs", "steps": args.steps, "warmup": args.warmup,
                          "value": round(pbs_s, 2), "unit": "PBS/s", **head}), flush=True)
        return
    timed_s = head["timed_ms"] / 1e3
    roofline = head.pop("roofline")
    pbs_s = head["timed_pbs"] / timed_s
    if not args.no_microbench:
        note("microbenchmarks")
        roofline["measured"] = microbench(L, ctx)
        # the same achieved rate against the measured ceiling of the
        # butterfly's instruction mix (what the kernel's arithmetic can reach)
        roofline["frac_of_measured_peak"] = round(roofline["achieved"] / roofline["measured"]["modmul_probe_tops"], 4)
        full["roofline_graph"]["frac_of_measured_peak"] = round(
            full["roofline_graph"]["achieved"] / roofline["measured"]["modmul_probe_tops"], 4)
    line = {
        "metric": "PBS/s & DP cells/s; batched vs plain queries/s; p50/p99 query latency",
        "value": round(pbs_s, 2), "unit": "PBS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["timed_ms"] / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched_ascii_256_pairs", "queries": 256, "lengths": "uniform 8..64",
                   "encoding": "ascii7", "both_encrypted": True,
                   "step": "one plan step: every ready cell of one anti-diagonal of every query plus the "
                           "equality bootstraps of the next ones, one key-switch and one blind-rotation launch",
                   "params": "n=742 k=1 N=2048 q=2^64 pbs 2^23x1 ks 2^3x5", "path": "batch plan"},
        "cells_per_s": full["cells_per_s"],
        "queries_per_s": full["queries_per_s"],
        "timed": head,
        "roofline": roofline,
        "full_pass": full,
        "plain_same_queries": plain,
    }
    if tuning is not None:
        line["tuning"] = dict(tuning["tuning"], cached=tuning["cached"], samples=tuning.get("samples"))
    # the other configurations
    note("configs: dna 256 x 256, tiny dna, plain 32 x 32")
    a, b = W.dna_align()
    line["dna_align_256x256"] = plain_config(L, ck, ctx, a, b, L.LVS_ENC_DNA2, 70001, reps=3)
    a, b = W.tiny_dna()
    line["tiny_dna_6x6"] = plain_config(L, ck, ctx, a, b, L.LVS_ENC_DNA2, 70011, reps=5)
    a, b = W.plain_ascii()
    line["plain_ascii_32x32"] = plain_config(L, ck, ctx, a, b, L.LVS_ENC_ASCII7, 1001, reps=5)
    line["plain_same_queries"]["vs_plain_32x32_pbs_per_s"] = round(
        full["pbs_per_s"] / line["plain_ascii_32x32"]["pbs_per_s"], 2)
    if not args.no_serving and args.serving_names > 0:
        line["serving"] = serving_block(L, ck, ctx, args.serving_names, args.serving_queries,
                                        args.poisson_queries, [float(x) for x in args.rho.split(",") if x],
                                        max_step=args.serving_max_step, progress=args.serving_progress,
                                        arena_gb=32 if args.serving_names > 256 else 4,
                                        poisson_seed=args.poisson_seed, query_offset=args.query_offset)
    if args.band_queries > 0:
        line["band"] = band_block(L, ck, ctx, args.band_queries, args.band_ell)
    if args.wide:
        line["wide"] = wide_block(L, ck, ctx)
    if not args.no_cpu_baseline:
        pairs = W.batched()
        A = L.lvs_encrypt_string(ck, pairs[0][0], L.LVS_ENC_ASCII7, 20000)
        B = L.lvs_encrypt_string(ck, pairs[0][1], L.LVS_ENC_ASCII7, 20001)
        z1 = (A[:, None, 0, :] - B[None, :, 0, :]).reshape(-1, L.CT_WORDS).astype(np.uint64)
        line["cpu_baseline"] = cpu_baseline(z1, "the first pair of the batched workload")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
