"""Host-side checks of liblvs that need no GPU: the C ABI loads and exports
every function include/lvs.h declares, and the library's key generation and
encryption (written independently of the oracle) agree with the oracle bit
for bit under the same seeds."""
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from oracle import leuvenshtein as OL
from oracle import tfhe as OT

HEADER = os.path.join(ROOT, "include", "lvs.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lvs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2508_14568_amd import lvs
    return lvs


def test_header_symbols_exported(L):
    lib = L.lib()
    declared = header_functions()
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lvs_[a-z0-9_]+)", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        assert hasattr(lib, f)
    # the binding wraps every declared function under the same name
    assert set(declared) <= set(L.exported_symbols())


def test_params_default(L):
    p = L.lvs_params_default()
    assert (p.n_lwe, p.glwe_k, p.poly_N, p.pbs_base_log, p.pbs_level, p.ks_base_log, p.ks_level) == \
        (742, 1, 2048, 23, 1, 3, 5)
    q = OT.default_params()
    assert (p.lwe_noise_q64, p.glwe_noise_q64) == (q.lwe_sigma_q64, q.glwe_sigma_q64)


@pytest.fixture(scope="module")
def both_keys(L):
    ck, sk = L.lvs_keygen(L.lvs_params_default(), 1)
    ok = OT.Keys(OT.default_params(), seed=1)
    return ck, sk, ok


def test_keygen_matches_oracle(L, both_keys):
    ck, sk, ok = both_keys
    assert (L.lvs_key_export(ck, sk, 0) == ok.small_key).all()
    assert (L.lvs_key_export(ck, sk, 1) == ok.big_key).all()
    bsk = L.lvs_key_export(ck, sk, 2).reshape(742, 2, 2, 2048)
    assert (bsk == ok.bsk()).all()
    ksk = L.lvs_key_export(ck, sk, 3).reshape(2048 * 5, 743)
    assert (ksk == ok.ksk()).all()


def test_encryption_matches_oracle(L, both_keys):
    ck, sk, ok = both_keys
    for mu, seed, idx in [(0, 3, 0), (9, 3, 1), (31, 77, 12345), (16, 2**63 + 5, 7)]:
        assert (L.lvs_lwe_encrypt(ck, mu, seed, idx) == ok.encrypt(mu, seed, idx)).all()
    s = b"Hello, KID"
    assert (L.lvs_encrypt_string(ck, s, L.LVS_ENC_ASCII7, 9) == OL.encrypt_string(ok, s, OL.ENC_ASCII7, 9)).all()
    d = bytes([0, 1, 2, 3, 3, 1])
    assert (L.lvs_encrypt_string(ck, d, L.LVS_ENC_DNA2, 4) == OL.encrypt_string(ok, d, OL.ENC_DNA2, 4)).all()


def test_wide_symbols_host(L, both_keys):
    """Section 4.2 wide symbols on the host: the chunk encryption equals the
    oracle's, the per-pair bootstrap count equals the method's, and symbols
    wider than the width are refused."""
    ck, sk, ok = both_keys
    from oracle import plaintext as OP
    for width in (1, 4, 5, 21, 60, 64):
        assert L.lvs_wide_chunks(width) == OP.wide_chunk_count(width)
        assert L.lvs_wide_pbs_per_pair(width) == OP.pbs_hybrid(width)
    assert L.lvs_wide_chunks(0) == 0 and L.lvs_wide_chunks(65) == 0
    syms = [0x1F600, 0x41, 0x10FFFF, 0]
    assert (L.lvs_encrypt_symbols(ck, syms, 21, 12) == OL.encrypt_symbols(ok, syms, 21, 12)).all()
    big = [2 ** 64 - 1, 2 ** 63 + 12345]
    assert (L.lvs_encrypt_symbols(ck, big, 64, 13) == OL.encrypt_symbols(ok, big, 64, 13)).all()
    with pytest.raises(L.LvsError) as e:
        L.lvs_encrypt_symbols(ck, [16], 4, 1)
    assert e.value.code == -2


def test_decrypt(L, both_keys):
    ck, sk, ok = both_keys
    for mu in range(32):
        ct = ok.encrypt(mu, 5, mu)
        got, err = L.lvs_lwe_decrypt(ck, ct)
        assert got == mu and err == ok.phase_error(ct)
    # distance from a bottom row of differences (+1, 0, -1, 0) with m = 3
    row = np.stack([ok.encrypt(v % 32, 6, k) for k, v in enumerate([1, 0, -1, 0])])
    assert L.lvs_decrypt_distance(ck, row, 3) == 3 + 1 + 0 - 1 + 0


def test_errors(L, both_keys):
    ck, sk, ok = both_keys
    with pytest.raises(L.LvsError) as e:
        L.lvs_encrypt_string(ck, b"\x80", L.LVS_ENC_ASCII7, 1)
    assert e.value.code == -2
    with pytest.raises(L.LvsError) as e:
        L.lvs_encrypt_string(ck, b"\x04", L.LVS_ENC_DNA2, 1)
    assert e.value.code == -2
    p = L.lvs_params_default()
    p.poly_N = 1024
    with pytest.raises(L.LvsError) as e:
        L.lvs_keygen(p, 1)
    assert e.value.code == -7


def test_band_counts_match_definition():
    """lvs_band_cells / lvs_band_exact against a brute-force count of
    |i - j| <= ell and the oracle's exact half-width (host logic, no GPU)."""
    from paper_2508_14568_amd import lvs as L
    from oracle import plaintext as P
    for m in range(0, 25):
        for n in range(0, 25, 4):
            for ell in range(0, 30, 5):
                want = sum(1 for i in range(1, m + 1) for j in range(1, n + 1) if abs(i - j) <= ell)
                assert L.lvs_band_cells(m, n, ell) == want
            assert L.lvs_band_exact(m, n) == P.exact_band(m, n)
    assert L.lvs_band_cells(40, 40, 7) == P.band_cell_count_formula(40, 7)


def test_plan_schedule_is_causal_and_fills_rounds():
    """lvs_plan_verify (host only): for mixes of ASCII/DNA, both-encrypted
    and cleartext, full and banded queries, every plan-written word is read
    only after an earlier step wrote it, no step races or exceeds the
    workspace bound, every bootstrap is scheduled, and filling the last
    partial round of each step never adds device rounds."""
    import numpy as np
    from paper_2508_14568_amd import lvs as L
    import workloads as W
    rng = np.random.default_rng(5)
    for enc in (L.LVS_ENC_ASCII7, L.LVS_ENC_DNA2):
        for trial in range(6):
            qs = []
            for _ in range(int(rng.integers(1, 40))):
                m, n = (int(x) for x in rng.integers(1, 50, size=2))
                kind = "enc" if rng.random() < 0.7 else "clear"
                ell = None if rng.random() < 0.6 else int(rng.integers(0, 12))
                qs.append((m, n, kind, ell))
            want = 0
            for m, n, kind, ell in qs:
                cells = L.lvs_band_cells(m, n, ell) if ell is not None else m * n
                want += cells * ((3 if enc == L.LVS_ENC_ASCII7 else 2) if kind == "enc" else 1)
            for rnd in (64, 256):
                _, jobs0, rounds0, bad0 = L.lvs_plan_verify(qs, enc, rnd, fill=False)
                _, jobs1, rounds1, bad1 = L.lvs_plan_verify(qs, enc, rnd, fill=True)
                assert bad0 == 0 and bad1 == 0, (enc, trial, rnd)
                assert jobs0 == jobs1 == want
                assert rounds1 <= rounds0
    # Section 3.1 refresh: a step after every R-th diagonal holding two
    # bootstraps per cell of that diagonal for each query with cells past it
    for enc in (L.LVS_ENC_ASCII7, L.LVS_ENC_DNA2):
        for trial, R in enumerate((4, 7, 16)):
            qs = []
            for _ in range(int(rng.integers(1, 20))):
                m, n = (int(x) for x in rng.integers(1, 50, size=2))
                kind = "enc" if rng.random() < 0.7 else "clear"
                ell = None if rng.random() < 0.6 else int(rng.integers(0, 12))
                qs.append((m, n, kind, ell))
            extra, due = 0, set()
            for m, n, kind, ell in qs:
                for s_ in range(R, m + n, R):
                    c = sum(1 for i in range(1, m + 1) if 1 <= s_ - i <= n and (ell is None or abs(2 * i - s_) <= ell))
                    extra += 2 * c
                    if c:
                        due.add(s_)
            for rnd in (64, 256):
                st0, jobs0, _, _ = L.lvs_plan_verify(qs, enc, rnd, fill=True)
                st1, jobs1, rounds1, bad1 = L.lvs_plan_verify(qs, enc, rnd, fill=True, refresh=R)
                assert bad1 == 0, (enc, R, rnd)
                assert jobs1 == jobs0 + extra
                assert st1 == st0 + len(due)
    with pytest.raises(L.LvsError):
        L.lvs_plan_verify([(4, 4, "enc", None)], L.LVS_ENC_DNA2, 64, refresh=3)
    # the 64-query batched workload: filling removes device rounds
    qs = [(len(a), len(b), "enc", None) for a, b in W.batched()[:64]]
    _, jobs, rounds_plain, bad0 = L.lvs_plan_verify(qs, L.LVS_ENC_ASCII7, 256, fill=False)
    _, _, rounds_filled, bad1 = L.lvs_plan_verify(qs, L.LVS_ENC_ASCII7, 256, fill=True)
    assert bad0 == bad1 == 0 and jobs == 3 * sum(m * n for m, n, _, _ in qs)
    assert rounds_filled < 0.97 * rounds_plain


def test_wide_plan_schedule_is_causal():
    """lvs_plan_verify_wide (host only): the wide-symbol plans that run the
    hybrid equality (Section 4.2) inside the main loop read every word that
    a bootstrap or a group sum writes only after an earlier step wrote it,
    have no in-step races, stay within the workspace bound and schedule
    every bootstrap: (chunks + merges) per in-band pair, one per cell, two
    per cell of a refreshed diagonal.  Widths cover one chunk (no merging),
    one merging level and two; a 32 x 32 pair of 21-bit symbols takes one
    device round per anti-diagonal plus two lead-in rounds."""
    import numpy as np
    from paper_2508_14568_amd import lvs as L

    def want(qs, width, R):
        per = L.lvs_wide_pbs_per_pair(width)
        tot = 0
        for m, n, ell in qs:
            cells = L.lvs_band_cells(m, n, ell) if ell is not None else m * n
            tot += cells * (per + 1)
            for s in range(R, m + n, R) if R else ():
                tot += 2 * sum(1 for i in range(max(1, s - n), min(m, s - 1) + 1)
                               if ell is None or abs(2 * i - s) <= ell)
        return tot

    rng = np.random.default_rng(9)
    for width in (4, 21, 64):
        for trial in range(4):
            qs = []
            for _ in range(int(rng.integers(1, 8))):
                m, n = (int(x) for x in rng.integers(0, 30, size=2))
                ell = None if rng.random() < 0.7 else int(rng.integers(0, 6))
                qs.append((m, n, ell))
            for R in (0, 4, 7):
                for rnd in (64, 256):
                    _, jobs, _, bad = L.lvs_plan_verify_wide(qs, width, rnd, refresh=R)
                    assert bad == 0, (width, trial, R, rnd)
                    assert jobs == want(qs, width, R), (width, trial, R)
    _, jobs, rounds, bad = L.lvs_plan_verify_wide([(32, 32, None)], 21, 256)
    assert bad == 0 and jobs == 32 * 32 * 8 and rounds == 65
    with pytest.raises(L.LvsError):
        L.lvs_plan_verify_wide([(4, 4, None)], 65, 256)


def test_wire_round_trip(L, both_keys):
    """Client key, server key and ciphertexts survive export and import word
    for word; the imported client key encrypts and decrypts as the original."""
    ck, sk, _ = both_keys
    rec_ck = L.lvs_export(L.LVS_WIRE_CLIENT_KEY, ck)
    kind, ck2 = L.lvs_import_key(rec_ck)
    assert kind == L.LVS_WIRE_CLIENT_KEY
    assert len(rec_ck) == 4 + 4 + 28 + 16 + 16 + 742 + 2048 + 8
    for k in (0, 1):
        assert np.array_equal(L.lvs_key_export(ck, sk, k), L.lvs_key_export(ck2, sk, k))
    ct = L.lvs_encrypt_string(ck, b"kitten", L.LVS_ENC_ASCII7, 77)
    assert np.array_equal(ct, L.lvs_encrypt_string(ck2, b"kitten", L.LVS_ENC_ASCII7, 77))
    rec_sk = L.lvs_export(L.LVS_WIRE_SERVER_KEY, sk)
    kind, sk2 = L.lvs_import_key(rec_sk)
    assert kind == L.LVS_WIRE_SERVER_KEY
    for k in (2, 3):
        assert np.array_equal(L.lvs_key_export(ck, sk, k), L.lvs_key_export(ck, sk2, k))
    rec_ct = L.lvs_export(L.LVS_WIRE_CIPHERTEXTS, ct)
    back = L.lvs_import_ciphertexts(rec_ct)
    assert back.shape == (12, L.CT_WORDS) and np.array_equal(back, ct.reshape(12, L.CT_WORDS))
    assert [L.lvs_lwe_decrypt(ck2, c)[0] for c in back[0::2]] == [c & 15 for c in b"kitten"]
    assert L.lvs_import_ciphertexts(L.lvs_export(L.LVS_WIRE_CIPHERTEXTS, ct[:0])).shape == (0, L.CT_WORDS)


def test_wire_rejects_malformed(L, both_keys):
    ck, _, _ = both_keys
    ct = L.lvs_encrypt_string(ck, b"abc", L.LVS_ENC_ASCII7, 5)
    rec = bytearray(L.lvs_export(L.LVS_WIRE_CIPHERTEXTS, ct))
    bad = bytearray(rec)
    bad[100] ^= 1                                   # a payload byte: checksum mismatch
    with pytest.raises(L.LvsError, match="checksum") as e:
        L.lvs_import_ciphertexts(bytes(bad))
    assert e.value.code == -1
    with pytest.raises(L.LvsError, match="length"):
        L.lvs_import_ciphertexts(bytes(rec[:-1]))
    with pytest.raises(L.LvsError, match="not an lvs record"):
        L.lvs_import_ciphertexts(b"XXXX" + bytes(rec[4:]))
    with pytest.raises(L.LvsError, match="no key"):
        L.lvs_import_key(bytes(rec))
    kd = bytearray(L.lvs_export(L.LVS_WIRE_CLIENT_KEY, ck))
    with pytest.raises(L.LvsError, match="no ciphertexts"):
        L.lvs_import_ciphertexts(bytes(kd))
    kd[16] ^= 1                                     # poly_N: a parameter set the kernels lack
    with pytest.raises(L.LvsError) as e:
        L.lvs_import_key(bytes(kd))
    assert e.value.code == -7
    with pytest.raises(L.LvsError, match="unknown kind"):
        L.lvs_export(9, ck)
    with pytest.raises(L.LvsError, match="not a server key"):
        L.lvs_export(L.LVS_WIRE_SERVER_KEY, ck)


def test_wire_export_rejects_oversized_count(L):
    """A ciphertext count whose record size would not fit in size_t is an
    error, not a wrapped length (the size query passes no buffer)."""
    import ctypes
    n = ctypes.c_size_t()
    dummy = (ctypes.c_uint64 * 1)()
    rc = L.lib().lvs_export(L.LVS_WIRE_CIPHERTEXTS, dummy, ctypes.c_size_t(2 ** 64 // (8 * L.CT_WORDS) + 1), None,
                            ctypes.byref(n))
    assert rc == -1
    assert "too many ciphertexts" in L.lib().lvs_last_error().decode()
