"""GPU bootstraps through the C ABI (lvs_pbs_batch) against the oracle.

Bar: bit-exact ciphertexts (every word equal) and exact decryptions, since
keys, encryptions and every step of the bootstrap are integer arithmetic in
Z/2^64 fixed by the seed (no tolerance)."""
import numpy as np
import pytest

from conftest import golden
from gpu_common import assert_same_ct, gpu, okeys, okeys_kara, oracle_threads, say  # noqa: F401
from oracle import plaintext as P
from oracle import tfhe as T

pytestmark = pytest.mark.gpu


def run_pbs(g, cts, lut_id=0, lut_ids=None):
    L, torch = g.L, g.torch
    cts = np.ascontiguousarray(cts, dtype=np.uint64).reshape(-1, L.CT_WORDS)
    B = cts.shape[0]
    d_in = L.to_device(cts, g.dev)
    d_out = torch.zeros_like(d_in)
    d_ids = None
    if lut_ids is not None:
        d_ids = np.asarray(lut_ids, dtype=np.uint8)
    L.lvs_pbs_batch(g.ctx, d_in, B, d_out, lut_id=lut_id, lut_ids=d_ids)
    torch.cuda.synchronize()
    return L.to_host(d_out).reshape(B, L.CT_WORDS)


def test_table1_exhaustive_bit_exact(gpu, okeys):
    """Table table_lutrelu: f(x) = x - 4 over all 32 inputs of the 5-bit
    space; every output ciphertext equals the oracle's."""
    say("table1 exhaustive")
    g = gpu
    g.L.lvs_context_set_lut(g.ctx, g.L.LVS_LUT_USER, P.LUT_X_MINUS_4)
    cts = np.stack([g.L.lvs_lwe_encrypt(g.ck, x, 501, x) for x in range(32)])
    out = run_pbs(g, cts, lut_id=g.L.LVS_LUT_USER)
    ref = okeys.pbs_batch(cts, T.test_polynomial(P.LUT_X_MINUS_4, 2048)[None, :], 0)
    for x in range(32):
        assert_same_ct(out[x], ref[x], f"x={x}")
    dec = [g.L.lvs_lwe_decrypt(g.ck, o)[0] % 16 for o in out]
    assert dec == golden("table1_lut_x_minus_4.json")["outputs"]


@pytest.mark.parametrize("name", ["eq", "eq9", "min", "refresh", "max", "max9", "table2"])
def test_tables_exhaustive(gpu, okeys_kara, name):
    """All 32 inputs through LUT_eq, LUT_eq9, the negated-key LUT_min, the
    refresh table, the merging tables LUT_max / LUT_max9 and the printed
    Table LUTmin; decryptions exact, every output bit-exact with the oracle."""
    say("tables exhaustive", name)
    g = gpu
    lut = {"eq": P.LUT_EQ, "eq9": P.LUT_EQ9, "min": P.lut_min_negated(), "refresh": P.LUT_REFRESH,
           "max": P.LUT_MAX, "max9": P.LUT_MAX9, "table2": P.lut_min_plain()}[name]
    slot = {"eq": g.L.LVS_LUT_EQ, "eq9": g.L.LVS_LUT_EQ9, "min": g.L.LVS_LUT_MIN, "refresh": g.L.LVS_LUT_REFRESH,
            "max": g.L.LVS_LUT_MAX, "max9": g.L.LVS_LUT_MAX9, "table2": 7}[name]
    if name == "table2":
        g.L.lvs_context_set_lut(g.ctx, 7, lut)
    cts = np.stack([g.L.lvs_lwe_encrypt(g.ck, x, 600 + slot, x) for x in range(32)])
    out = run_pbs(g, cts, lut_id=slot)
    assert [g.L.lvs_lwe_decrypt(g.ck, o)[0] for o in out] == [P.negacyclic_read(lut, x) for x in range(32)]
    if name == "table2":
        assert [g.L.lvs_lwe_decrypt(g.ck, o)[0] % 16 for o in out] == golden("table2_lutmin.json")["outputs"]
    ref = okeys_kara.pbs_batch(cts, T.test_polynomial(lut, 2048)[None, :], 0, nthreads=oracle_threads())
    for x in range(32):
        assert_same_ct(out[x], ref[x], f"{name} x={x}")


def test_mixed_luts_ragged_batch(gpu, okeys):
    """37 bootstraps (not a multiple of the key-switch tile of 8) with a
    per-ciphertext table id; every output bit-exact."""
    say("mixed luts ragged")
    g = gpu
    rng = np.random.default_rng(7)
    B = 37
    mus = rng.integers(0, 32, size=B)
    ids = rng.integers(0, 3, size=B).astype(np.uint8)
    cts = np.stack([g.L.lvs_lwe_encrypt(g.ck, int(mu), 700, k) for k, mu in enumerate(mus)])
    out = run_pbs(g, cts, lut_ids=ids)
    polys = np.stack([T.test_polynomial(P.LUT_EQ, 2048), T.test_polynomial(P.LUT_EQ9, 2048),
                      T.test_polynomial(P.lut_min_negated(), 2048)])
    ref = okeys.pbs_batch(cts, polys, ids.astype(np.int32))
    for b in range(B):
        assert_same_ct(out[b], ref[b], f"b={b}")


def test_batch_sizes_deterministic(gpu):
    """Outputs do not depend on the batch a ciphertext sits in, nor on the
    run (bit-identical), for sizes 1, 2, 255 and 1031."""
    say("batch sizes")
    g = gpu
    rng = np.random.default_rng(3)
    mus = rng.integers(0, 32, size=1031)
    cts = np.stack([g.L.lvs_lwe_encrypt(g.ck, int(mu), 800, k) for k, mu in enumerate(mus)])
    full = run_pbs(g, cts, lut_id=g.L.LVS_LUT_MIN)
    again = run_pbs(g, cts, lut_id=g.L.LVS_LUT_MIN)
    assert (full == again).all()
    want = [P.negacyclic_read(P.lut_min_negated(), int(mu)) for mu in mus]
    assert [g.L.lvs_lwe_decrypt(g.ck, o)[0] for o in full] == want
    for lo, B in [(0, 1), (5, 2), (100, 255)]:
        part = run_pbs(g, cts[lo:lo + B], lut_id=g.L.LVS_LUT_MIN)
        assert (part == full[lo:lo + B]).all()


def test_noisy_inputs_decode(gpu, okeys):
    """Inputs whose phase sits up to 3/8 of a box away from the encoded value
    still bootstrap to the table entry, with fresh (small) output noise."""
    say("noisy inputs")
    g = gpu
    cts = []
    xs = [0, 0, 5, 17, 31, 12]
    offs = [3 * 2**56, -3 * 2**56, 2**57, -2**57, 2**56, -(2**56)]
    for k, (x, off) in enumerate(zip(xs, offs)):
        ct = g.L.lvs_lwe_encrypt(g.ck, x, 900, k)
        ct[2048] = np.uint64((int(ct[2048]) + off) % 2**64)
        cts.append(ct)
    out = run_pbs(g, np.stack(cts), lut_id=g.L.LVS_LUT_EQ9)
    ref = okeys.pbs_batch(np.stack(cts), T.test_polynomial(P.LUT_EQ9, 2048)[None, :], 0)
    for k, x in enumerate(xs):
        mu, err = g.L.lvs_lwe_decrypt(g.ck, out[k])
        assert mu == P.negacyclic_read(P.LUT_EQ9, x)
        assert abs(err) < 2**52
        assert_same_ct(out[k], ref[k], f"noisy {k}")


def test_argument_errors(gpu):
    g = gpu
    L, torch = g.L, g.torch
    d = torch.zeros(4 * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    small = torch.zeros(8, dtype=torch.int64, device=g.dev)
    with pytest.raises(L.LvsError) as e:
        L.lvs_pbs_batch(g.ctx, d[:2 * L.CT_WORDS], 2, d[2 * L.CT_WORDS:], lut_id=0, d_work=small)
    assert e.value.code == -5
    with pytest.raises(L.LvsError) as e:
        L.lvs_pbs_batch(g.ctx, d, 2, d[L.CT_WORDS:], lut_id=0)
    assert e.value.code == -1
    with pytest.raises(L.LvsError) as e:
        L.lvs_pbs_batch(g.ctx, d[:L.CT_WORDS], 1, d[L.CT_WORDS:2 * L.CT_WORDS], lut_id=8)
    assert e.value.code == -1
    L.lvs_pbs_batch(g.ctx, d, 0, d, lut_id=0)      # empty batch: no work, no error
