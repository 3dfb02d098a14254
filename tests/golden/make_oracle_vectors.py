"""Writes oracle-computed expected values for the GPU parity tests.

Calls only ``oracle`` and the seeded ``workloads`` generators (never the HIP
library).  For each workload it records, under fixed key and encryption
seeds, the SHA-256 digest of every intermediate ciphertext (eq1 and eq9 of
every character pair, M of every cell) and the full bottom-row result
h[m, 1..n].

Usage: python tests/golden/make_oracle_vectors.py [tiny_dna] [plain_ascii]
"""
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


def digest(ct) -> str:
    return hashlib.sha256(np.ascontiguousarray(ct, dtype=np.uint64).tobytes()).hexdigest()


def run(name: str, keys: T.Keys):
    if name == "tiny_dna":
        a, b = W.tiny_dna()
        enc = L.ENC_DNA2
        sa, sb = W.dna_codes(a), W.dna_codes(b)
    elif name == "plain_ascii":
        a, b = W.plain_ascii()
        enc = L.ENC_ASCII7
        sa, sb = a, b
    else:
        raise ValueError(name)
    t0 = time.time()
    A = L.encrypt_string(keys, sa, enc, SEED_A)
    B = L.encrypt_string(keys, sb, enc, SEED_B)
    h_last, rec = L.edit_distance(keys, A, B, enc, order="diagonal", record=True)
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
        "written_by": "tests/golden/make_oracle_vectors.py (oracle only)",
    }
    if rec.get("eq1") is not None:
        meta["eq1_sha256"] = [[digest(rec["eq1"][i, j]) for j in range(n)] for i in range(m)]
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(meta, f)
    np.save(os.path.join(HERE, f"oracle_{name}_h_last.npy"), np.ascontiguousarray(h_last, dtype=np.uint64))
    print(f"{name}: distance {dist}, {time.time() - t0:.0f} s", flush=True)


def main(names):
    keys = T.Keys(T.default_params(), seed=KEY_SEED)
    for name in names:
        run(name, keys)


if __name__ == "__main__":
    main(sys.argv[1:] or ["tiny_dna", "plain_ascii"])
