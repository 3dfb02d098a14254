"""Character equality on the GPU over whole alphabets (Algorithm 3 for
7-bit ASCII, one bootstrap for 2-bit DNA): every pair's eq9 decrypts to
9 [x == y], and a seeded sample of pairs is bit-exact with the oracle."""
import numpy as np
import pytest

from gpu_common import assert_same_ct, gpu, okeys, say  # noqa: F401
from oracle import leuvenshtein as OL

pytestmark = pytest.mark.gpu

DELTA_LOG = 59


def decode_all(L, ck, cts):
    """Plaintexts (mod 32) of (k, N+1) ciphertexts under the extracted key."""
    S = L.lvs_key_export(ck, None, 1).astype(np.uint64)
    phase = cts[:, -1] - cts[:, :-1] @ S
    return ((phase + np.uint64(1 << (DELTA_LOG - 1))) >> np.uint64(DELTA_LOG)).astype(np.int64) % 32


@pytest.mark.parametrize("enc", ["ascii", "dna"])
def test_equality_whole_alphabet(gpu, okeys, enc):
    g = gpu
    L, torch = g.L, g.torch
    code = L.LVS_ENC_ASCII7 if enc == "ascii" else L.LVS_ENC_DNA2
    size = 128 if enc == "ascii" else 4
    say("equality over the whole alphabet", enc, size)
    s = bytes(range(size))
    A = L.lvs_encrypt_string(g.ck, s, code, 2101)
    B = L.lvs_encrypt_string(g.ck, s, code, 2102)
    d_eq9 = torch.zeros(size * size * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_equality(g.ctx, L.to_device(A, g.dev), size, L.to_device(B, g.dev), size, code, d_eq9)
    torch.cuda.synchronize()
    eq9 = L.to_host(d_eq9).reshape(size * size, L.CT_WORDS)
    del d_eq9
    mu = decode_all(L, g.ck, eq9).reshape(size, size)
    assert (mu == 9 * np.eye(size, dtype=np.int64)).all()
    # a seeded sample (and two equal pairs) bit-exact with the oracle
    oenc = OL.ENC_ASCII7 if enc == "ascii" else OL.ENC_DNA2
    OA = OL.encrypt_string(okeys, s, oenc, 2101)
    OB = OL.encrypt_string(okeys, s, oenc, 2102)
    rng = np.random.default_rng(2103)
    picks = [(int(i), int(j)) for i, j in rng.integers(0, size, size=(4, 2))] + [(1, 1), (size - 1, size - 1)]
    for i, j in picks:
        _, ref = OL.equality(okeys, OA[i:i + 1], OB[j:j + 1], oenc)
        assert_same_ct(eq9[i * size + j], ref[0, 0], f"eq9[{i},{j}]")
