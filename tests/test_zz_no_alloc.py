"""The no-allocation bootstrap entry point (lvs_pbs_batch_static) through the
C ABI, against lvs_pbs_batch on the same inputs: bit-identical outputs on two
calls in a row, the second with a smaller batch (the device array keeps the
first call's contents), and a clear error past the maximum batch.

Bar: every word equal (integer arithmetic throughout, no tolerance)."""
import numpy as np
import pytest

from gpu_common import gpu, say  # noqa: F401

pytestmark = pytest.mark.gpu


def encrypt_batch(g, B, seed):
    rng = np.random.default_rng(seed)
    mus = rng.integers(0, 32, size=B)
    return np.stack([g.L.lvs_lwe_encrypt(g.ck, int(mu), seed, k) for k, mu in enumerate(mus)])


def both_paths(g, cts, lut_id=0, lut_ids=None):
    L, torch = g.L, g.torch
    B = cts.shape[0]
    d_in = L.to_device(np.ascontiguousarray(cts, dtype=np.uint64), g.dev)
    d_ref = torch.zeros_like(d_in)
    d_out = torch.full_like(d_in, -1)
    L.lvs_pbs_batch(g.ctx, d_in, B, d_ref, lut_id=lut_id, lut_ids=lut_ids)
    L.lvs_pbs_batch_static(g.ctx, d_in, B, d_out, lut_id=lut_id, lut_ids=lut_ids)
    torch.cuda.synchronize()
    return L.to_host(d_ref).reshape(B, L.CT_WORDS), L.to_host(d_out).reshape(B, L.CT_WORDS)


def test_static_matches_workspace_entry_point(gpu):
    g = gpu
    L = g.L
    B1 = L.LVS_PBS_STATIC_MAX
    say("no-alloc bootstraps: first call, B =", B1, "per-ciphertext tables")
    cts1 = encrypt_batch(g, B1, 7101)
    ids = np.random.default_rng(7102).integers(0, 4, size=B1).astype(np.uint8)
    ref1, out1 = both_paths(g, cts1, lut_ids=ids)
    bad = np.nonzero((ref1 != out1).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} of {B1} outputs differ, first {bad[:5]}"
    say("no-alloc bootstraps: second call, B = 37, one table")
    cts2 = encrypt_batch(g, 37, 7103)
    ref2, out2 = both_paths(g, cts2, lut_id=L.LVS_LUT_MIN)
    bad = np.nonzero((ref2 != out2).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} of 37 outputs differ, first {bad[:5]}"
    # the outputs decrypt to the tables' values (not only equal to each other)
    mus2 = np.random.default_rng(7103).integers(0, 32, size=37)
    lut_min = [0, 0, 0, 1, 1, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0]
    want = [lut_min[mu] if mu < 16 else (-lut_min[mu - 16]) % 32 for mu in mus2]
    assert [L.lvs_lwe_decrypt(g.ck, o)[0] for o in out2] == want


def test_static_rejects_past_maximum(gpu):
    g = gpu
    L, torch = g.L, g.torch
    B = L.LVS_PBS_STATIC_MAX + 1
    d_in = torch.zeros(B * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    d_out = torch.zeros_like(d_in)
    with pytest.raises(L.LvsError) as e:
        L.lvs_pbs_batch_static(g.ctx, d_in, B, d_out)
    assert e.value.code == -1 and "LVS_PBS_STATIC_MAX" in str(e.value)
    with pytest.raises(L.LvsError):
        L.lvs_pbs_batch_static(g.ctx, d_in, 4, d_out, lut_id=8)
