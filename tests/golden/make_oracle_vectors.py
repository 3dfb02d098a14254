"""Writes oracle-computed expected values for the GPU parity tests.

Calls only ``oracle`` and the seeded ``workloads`` generators (never the HIP
library).  Under fixed key and encryption seeds it records SHA-256 digests of
the intermediate ciphertexts (eq1 and eq9 of every character pair, M of every
cell, the Section 5 table) and of the result row h[m, 1..n]:

  tiny_dna, plain_ascii  every ciphertext digest, and the result row itself
  dna_align              the 256 x 256 DNA workload with the default refresh
                         interval (256): per matrix row i, the digest of the
                         row's per-cell digests (eq9 and M), and every h[m, j]
  batched_sample         the sampled pairs of the batched workload (Algorithm
                         4 in full, seeds 11000 + 2k, 11001 + 2k), as above
  serving_sample         the sampled queries of the serving workload (seed
                         12000 + q) against the sampled server names: the
                         Section 5 table over the server alphabet and every
                         name's cleartext main pass

The full-size workloads run the oracle with Karatsuba's products (pinned to
the schoolbook sums by tests/test_oracle_tfhe.py); --checkpoint DIR lets the
long dna_align run resume after an interruption.

Usage: python tests/golden/make_oracle_vectors.py [--threads T] [--checkpoint DIR] NAME...
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import leuvenshtein as L  # noqa: E402
from oracle import plaintext as P  # noqa: E402
from oracle import tfhe as T  # noqa: E402
import workloads as W  # noqa: E402

KEY_SEED = 1
SEED_A, SEED_B = 1001, 1002
REFRESH_DEFAULT = 256          # the library's default refresh interval


def digest(ct) -> str:
    return hashlib.sha256(np.ascontiguousarray(ct, dtype=np.uint64).tobytes()).hexdigest()


def row_digest(cell_digests) -> str:
    """Digest of one matrix row: SHA-256 over its cells' SHA-256 digests."""
    return hashlib.sha256(b"".join(bytes.fromhex(d) for d in cell_digests)).hexdigest()


def say(*args):
    print(time.strftime("%H:%M:%S"), *args, flush=True)


def write(name, meta):
    meta["written_by"] = "tests/golden/make_oracle_vectors.py (oracle only)"
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(meta, f)


def run_small(name: str, keys: T.Keys, threads):
    if name == "tiny_dna":
        a, b = W.tiny_dna()
        enc = L.ENC_DNA2
        sa, sb = W.dna_codes(a), W.dna_codes(b)
    else:
        a, b = W.plain_ascii()
        enc = L.ENC_ASCII7
        sa, sb = a, b
    t0 = time.time()
    A = L.encrypt_string(keys, sa, enc, SEED_A)
    B = L.encrypt_string(keys, sb, enc, SEED_B)
    h_last, rec = L.edit_distance(keys, A, B, enc, order="diagonal", record=True, nthreads=threads)
    m, n = len(a), len(b)
    dist = L.decrypt_distance(keys, m, h_last)
    assert dist == P.edit_distance(a, b), (dist, P.edit_distance(a, b))
    meta = {
        "workload": name, "a": a.decode(), "b": b.decode(), "encoding": enc, "key_seed": KEY_SEED,
        "seed_a": SEED_A, "seed_b": SEED_B, "m": m, "n": n, "distance": dist,
        "eq9_sha256": [[digest(rec["eq9"][i, j]) for j in range(n)] for i in range(m)],
        "M_sha256": [[digest(rec["M"][(i + 1, j + 1)]) for j in range(n)] for i in range(m)],
        "h_last_sha256": [digest(c) for c in h_last],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    if rec.get("eq1") is not None:
        meta["eq1_sha256"] = [[digest(rec["eq1"][i, j]) for j in range(n)] for i in range(m)]
    write(name, meta)
    np.save(os.path.join(HERE, f"oracle_{name}_h_last.npy"), np.ascontiguousarray(h_last, dtype=np.uint64))
    say(f"{name}: distance {dist}, {time.time() - t0:.0f} s")


def query_record(keys, A, B, enc, threads, refresh_every=0):
    """Algorithm 4 on one encrypted pair: row digests of eq1/eq9/M, digests
    of the result row, and the decrypted distance."""
    m, n = A.shape[0], B.shape[0]
    h_last, rec = L.edit_distance(keys, A, B, enc, order="diagonal", record=True, nthreads=threads,
                                  refresh_every=refresh_every)
    out = {
        "eq9_row_sha256": [row_digest([digest(rec["eq9"][i, j]) for j in range(n)]) for i in range(m)],
        "M_row_sha256": [row_digest([digest(rec["M"][(i + 1, j + 1)]) for j in range(n)]) for i in range(m)],
        "h_last_sha256": [digest(c) for c in h_last],
        "distance": L.decrypt_distance(keys, m, h_last),
    }
    if rec.get("eq1") is not None:
        out["eq1_row_sha256"] = [row_digest([digest(rec["eq1"][i, j]) for j in range(n)]) for i in range(m)]
    return out


def run_batched_sample(keys, threads):
    pairs = W.batched()
    idx = W.batched_sample()
    t0 = time.time()
    queries = []
    for k in idx:
        a, b = pairs[k]
        A = L.encrypt_string(keys, a, L.ENC_ASCII7, 11000 + 2 * k)
        B = L.encrypt_string(keys, b, L.ENC_ASCII7, 11001 + 2 * k)
        q = query_record(keys, A, B, L.ENC_ASCII7, threads)
        assert q["distance"] == P.edit_distance(a, b)
        q.update({"index": k, "a": a.decode(), "b": b.decode(), "seed_a": 11000 + 2 * k, "seed_b": 11001 + 2 * k})
        queries.append(q)
        say(f"batched pair {k}: {len(a)} x {len(b)}, {time.time() - t0:.0f} s")
    write("batched_sample", {"workload": "batched_sample", "key_seed": KEY_SEED, "encoding": L.ENC_ASCII7,
                             "queries": queries, "oracle_seconds": round(time.time() - t0, 1)})


def run_serving_sample(keys, threads):
    server, queries = W.serving()
    qidx, nidx = W.serving_sample()
    alpha = W.alphabet_of(server)
    t0 = time.time()
    out = []
    for qi in qidx:
        q = queries[qi]
        Q = L.encrypt_string(keys, q, L.ENC_ASCII7, 12000 + qi)
        table = L.preprocess(keys, Q, alpha, L.ENC_ASCII7, nthreads=threads)
        rec = {"query": qi, "text": q.decode(), "seed": 12000 + qi,
               "table_sha256": [[digest(table[c, i]) for i in range(len(q))] for c in range(len(alpha))],
               "names": []}
        for k in nidx:
            nm = server[k]
            h_last, r = L.edit_distance_clear(keys, table, alpha, nm, L.ENC_ASCII7, record=True, nthreads=threads)
            dist = L.decrypt_distance(keys, len(q), h_last)
            assert dist == P.edit_distance(q, nm)
            rec["names"].append({
                "index": k, "text": nm.decode(), "distance": dist,
                "M_row_sha256": [row_digest([digest(r["M"][(i + 1, j + 1)]) for j in range(len(nm))])
                                 for i in range(len(q))],
                "h_last_sha256": [digest(c) for c in h_last]})
        out.append(rec)
        say(f"serving query {qi} ({len(q)} chars) against {len(nidx)} names, {time.time() - t0:.0f} s")
    write("serving_sample", {"workload": "serving_sample", "key_seed": KEY_SEED, "alphabet": alpha.decode(),
                             "queries": out, "oracle_seconds": round(time.time() - t0, 1)})


def diagonal_loop(keys, m, n, eq9, refresh, threads, cellsha, state_path=None, t0=None):
    """Algorithm 4's main loop in anti-diagonal order with the refresh of
    every refresh-th diagonal, the steps of oracle.leuvenshtein.dp, keeping
    only each M's digest (cellsha[i-1, j-1]) and checkpointing V, H and the
    digests every 8 diagonals to state_path.  Returns H (H[1:] = h[m, 1..n])."""
    polys = L.lut_polys(keys.N)
    one, four = T.trivial(1, keys.N), T.trivial(4, keys.N)
    if state_path and os.path.exists(state_path):
        st = np.load(state_path)
        V, H, s0 = st["V"], st["H"], int(st["s"])
        cellsha[...] = st["cellsha"]
        say(f"main loop resumes at diagonal {s0}")
    else:
        V, H, s0 = np.tile(one, (m + 1, 1)), np.tile(one, (n + 1, 1)), 2
    for s in range(s0, m + n + 1):
        cells = [(i, s - i) for i in range(max(1, s - n), min(m, s - 1) + 1)]
        keys_b = np.stack([(four - V[i] + T.scale(H[j], 3) + eq9[i - 1, j - 1]).astype(T.U64) for i, j in cells])
        Ms = keys.pbs_batch(keys_b, polys, L.LUT_IDS["min"], threads)
        for (i, j), M in zip(cells, Ms):
            cellsha[i - 1, j - 1] = np.frombuffer(bytes.fromhex(digest(M)), dtype=np.uint8)
            V[i], H[j] = (M - H[j]).astype(T.U64), (M - V[i]).astype(T.U64)
        if L.refresh_due(s, m, n, refresh):
            fresh = keys.pbs_batch(np.stack([V[i] for i, _ in cells] + [H[j] for _, j in cells]), polys,
                                   L.LUT_IDS["refresh"], threads)
            for k, (i, j) in enumerate(cells):
                V[i], H[j] = fresh[k], fresh[len(cells) + k]
            say(f"refreshed diagonal {s}")
        if state_path and (s % 8 == 0 or s == m + n):
            np.savez(state_path + ".tmp.npz", V=V, H=H, s=s + 1, cellsha=cellsha)
            os.replace(state_path + ".tmp.npz", state_path)
        if t0 is not None and s % 16 == 0:
            say(f"diagonal {s} / {m + n}, {time.time() - t0:.0f} s")
    return H


def check_diagonal_loop(keys, threads):
    """diagonal_loop gives the words of oracle.leuvenshtein.edit_distance on
    a small DNA pair refreshed every 4 diagonals."""
    a, b = b"ACGTTGCA", b"AGGTCTGCA"
    A = L.encrypt_string(keys, W.dna_codes(a), L.ENC_DNA2, 5)
    B = L.encrypt_string(keys, W.dna_codes(b), L.ENC_DNA2, 6)
    h_ref, rec = L.edit_distance(keys, A, B, L.ENC_DNA2, record=True, nthreads=threads, refresh_every=4)
    m, n = len(a), len(b)
    cellsha = np.zeros((m, n, 32), dtype=np.uint8)
    H = diagonal_loop(keys, m, n, rec["eq9"], 4, threads, cellsha)
    assert (H[1:] == h_ref).all()
    for i in range(m):
        for j in range(n):
            assert bytes(cellsha[i, j]).hex() == digest(rec["M"][(i + 1, j + 1)])
    say("diagonal loop equals the oracle's edit_distance (refresh every 4)")


def run_dna_align(keys, threads, ckpt):
    """The 256 x 256 DNA pair through the oracle's diagonal loop, with
    per-cell digests kept as the cells finish (checkpointed every few
    diagonals when ckpt is set)."""
    a, b = W.dna_align()
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    m, n = len(a), len(b)
    t0 = time.time()
    A = L.encrypt_string(keys, sa, L.ENC_DNA2, SEED_A)
    B = L.encrypt_string(keys, sb, L.ENC_DNA2, SEED_B)
    Wd = keys.N + 1
    eq9_path = os.path.join(ckpt, "dna_eq9.npy") if ckpt else None
    if eq9_path and os.path.exists(eq9_path):
        eq9 = np.load(eq9_path)
        say("dna_align: equality from checkpoint")
    else:
        z = (A[:, None, 0, :] - B[None, :, 0, :]).astype(T.U64).reshape(m * n, Wd)
        parts = []
        for lo in range(0, m * n, 4096):
            parts.append(keys.pbs_batch(z[lo:lo + 4096], L.lut_polys(keys.N), L.LUT_IDS["eq9"], threads))
            say(f"dna_align: equality {lo + len(parts[-1])} / {m * n}, {time.time() - t0:.0f} s")
        eq9 = np.concatenate(parts).reshape(m, n, Wd)
        if eq9_path:
            np.save(eq9_path, eq9)
    cellsha = np.zeros((m, n, 32), dtype=np.uint8)
    state_path = os.path.join(ckpt, "dna_state.npz") if ckpt else None
    H = diagonal_loop(keys, m, n, eq9, REFRESH_DEFAULT, threads, cellsha, state_path, t0)
    h_last = H[1:]
    dist = L.decrypt_distance(keys, m, h_last)
    assert dist == P.edit_distance(a, b), (dist, P.edit_distance(a, b))
    eq9_rows = [row_digest([digest(eq9[i, j]) for j in range(n)]) for i in range(m)]
    m_rows = [row_digest([bytes(cellsha[i, j]).hex() for j in range(n)]) for i in range(m)]
    write("dna_align", {
        "workload": "dna_align", "a": a.decode(), "b": b.decode(), "encoding": L.ENC_DNA2, "key_seed": KEY_SEED,
        "seed_a": SEED_A, "seed_b": SEED_B, "m": m, "n": n, "distance": dist, "refresh_every": REFRESH_DEFAULT,
        "eq9_row_sha256": eq9_rows, "M_row_sha256": m_rows, "h_last_sha256": [digest(c) for c in h_last],
        "oracle_seconds": round(time.time() - t0, 1)})
    say(f"dna_align: distance {dist}, {time.time() - t0:.0f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["tiny_dna", "plain_ascii"])
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--checkpoint", default=None, help="directory for resumable state of dna_align")
    args = ap.parse_args()
    keys = T.Keys(T.default_params(), seed=KEY_SEED)
    for name in args.names:
        keys.karatsuba = name not in ("tiny_dna", "plain_ascii")
        if name in ("tiny_dna", "plain_ascii"):
            run_small(name, keys, args.threads)
        elif name == "batched_sample":
            run_batched_sample(keys, args.threads)
        elif name == "serving_sample":
            run_serving_sample(keys, args.threads)
        elif name == "dna_align":
            if args.checkpoint:
                os.makedirs(args.checkpoint, exist_ok=True)
            check_diagonal_loop(keys, args.threads)
            run_dna_align(keys, args.threads, args.checkpoint)
        else:
            raise SystemExit(f"unknown workload {name}")


if __name__ == "__main__":
    main()
