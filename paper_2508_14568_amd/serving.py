"""Request loop around the serving engine (lvs_server_*).

Queries arrive at given times (seconds from the start); the loop submits each
one when its time has come, runs engine steps while work is admitted or
queued, and records every query's latency from arrival to the moment its
results are on the host.  All computation happens in the library.
"""
import time

import numpy as np

from . import lvs as L


def run(srv, queries_ct, arrivals, on_result=None):
    """queries_ct: list of encrypted queries ([m][2][N+1] arrays, [m][c][N+1]
    chunk ciphertexts on a wide server); arrivals:
    non-decreasing arrival times in seconds; on_result(k, rows, latency) is
    called as each query finishes.  Returns (latencies in seconds, wall
    seconds, results)."""
    order = np.argsort(np.asarray(arrivals, dtype=float), kind="stable")
    t0 = time.perf_counter()
    nxt = 0
    pending = {}                      # ticket -> query index
    lat = [None] * len(queries_ct)
    results = [None] * len(queries_ct)
    while nxt < len(order) or pending:
        now = time.perf_counter() - t0
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            k = int(order[nxt])
            pending[L.lvs_server_submit(srv, queries_ct[k])] = k
            nxt += 1
        if not pending:
            time.sleep(max(0.0, arrivals[order[nxt]] - (time.perf_counter() - t0)))
            continue
        L.lvs_server_step(srv)
        for ticket in list(pending):
            out = L.lvs_server_poll(srv, ticket)
            if out is not None:
                k = pending.pop(ticket)
                lat[k] = time.perf_counter() - t0 - arrivals[k]
                results[k] = out
                if on_result:
                    on_result(k, out, lat[k])
    return lat, time.perf_counter() - t0, results


def percentiles(lat, ps=(50, 99)):
    """Latency percentiles with the number of samples they rest on (with few
    samples a high percentile is close to the maximum)."""
    a = np.asarray([x for x in lat if x is not None], dtype=float)
    out = {f"p{p}": float(np.percentile(a, p)) for p in ps}
    out["samples"] = int(a.size)
    return out
