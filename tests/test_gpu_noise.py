"""Noise of the DP state along the wavefront with refresh off (the reason
for Section 3.1's refresh bootstraps).  v and h telescope
along the diagonal (v[i,j] = M[i,j] - M[i-1,j] + v[i-1,j-1]), so the error of
a cell's key grows with min(i, j).  On the 256 x 256 DNA alignment every
bootstrap output M is recorded; every key 4 - v + 3 h + eq9 is rebuilt on the
host from them and decrypted with the client key: each must decode to its
plaintext key, its variance must follow Section 3.1's equation (14 bootstrap
output variances per level of the diagonal chain, with the output error
measured on the same bootstraps) and stay below the decoding threshold (half
a box, 2^58) with the key switch's and modulus switch's noise still to
come."""
import numpy as np
import pytest

from gpu_common import gpu, say  # noqa: F401
from oracle import plaintext as P
import workloads as W

pytestmark = pytest.mark.gpu

DELTA = 1 << 59


def test_key_noise_dna_256(gpu):
    g = gpu
    L, torch = g.L, g.torch
    a, b = W.dna_align()
    sa, sb = W.dna_codes(a), W.dna_codes(b)
    m, n = len(a), len(b)
    say("noise: dna 256 with trace")
    dA = L.to_device(L.lvs_encrypt_string(g.ck, sa, L.LVS_ENC_DNA2, 501), g.dev)
    dB = L.to_device(L.lvs_encrypt_string(g.ck, sb, L.LVS_ENC_DNA2, 502), g.dev)
    d_eq9 = torch.zeros(m * n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    d_tr = torch.zeros_like(d_eq9)
    d_h = torch.zeros(n * L.CT_WORDS, dtype=torch.int64, device=g.dev)
    L.lvs_equality(g.ctx, dA, m, dB, n, L.LVS_ENC_DNA2, d_eq9)
    prev = L.lvs_context_get_refresh(g.ctx)
    L.lvs_context_set_refresh(g.ctx, 0)          # the growth without refresh
    try:
        L.lvs_edit_distance_eq9(g.ctx, d_eq9, m, n, d_h, d_trace=d_tr)
        torch.cuda.synchronize()
    finally:
        L.lvs_context_set_refresh(g.ctx, prev)
    eq9 = L.to_host(d_eq9).reshape(m, n, L.CT_WORDS)
    tr = L.to_host(d_tr).reshape(m, n, L.CT_WORDS)
    del d_eq9, d_tr
    S = L.lvs_key_export(g.ck, None, 1).astype(np.uint64)          # the 2048-bit extracted key
    v_pl, h_pl, _ = P.delta_dp(a, b)
    eq_pl = np.array([[1 if x == y else 0 for y in b] for x in a])
    one = np.zeros(L.CT_WORDS, dtype=np.uint64)
    one[-1] = np.uint64(1 << 59)
    four = one * np.uint64(4)
    H = [one.copy() for _ in range(n + 1)]                          # h[i-1, j]
    err = np.zeros((m, n), dtype=np.float64)
    for i in range(1, m + 1):
        V = one.copy()                                              # v[i, 0]
        keys = np.zeros((n, L.CT_WORDS), dtype=np.uint64)
        for j in range(1, n + 1):
            keys[j - 1] = four - V + np.uint64(3) * H[j] + eq9[i - 1, j - 1]
            M = tr[i - 1, j - 1]
            v_new, h_new = M - H[j], M - V
            V, H[j] = v_new, h_new
        phase = keys[:, -1] - keys[:, :-1] @ S
        mu = ((phase + np.uint64(DELTA // 2)) >> np.uint64(59)).astype(np.int64) % 32
        want = (1 - v_pl[i, 0:n]) + 3 * (1 + h_pl[i - 1, 1:n + 1]) + 9 * eq_pl[i - 1]
        # v_pl[i, j-1] for j = 1..n is v_pl[i, 0:n]
        assert (mu == want % 32).all(), i
        e = (phase - (mu.astype(np.uint64) << np.uint64(59))).astype(np.int64)
        err[i - 1] = e.astype(np.float64)
    assert L.lvs_decrypt_distance(g.ck, L.to_host(d_h).reshape(n, L.CT_WORDS), m) == P.edit_distance(a, b)
    d = np.minimum.outer(np.arange(1, m + 1), np.arange(1, n + 1))
    worst = np.abs(err).max()
    lo = err[d <= 8].std()
    hi = err[d >= 192].std()
    # every bootstrap output's own error (the trace holds all m n of them)
    Mf = tr.reshape(m * n, L.CT_WORDS)
    ph = Mf[:, -1] - Mf[:, :-1] @ S
    mv = (ph + np.uint64(DELTA // 2)) >> np.uint64(59)
    eps = (ph - (mv << np.uint64(59))).astype(np.int64).astype(np.float64).std()
    # Section 3.1's key noise for the key of Eq. eq_keyeq2: each level of the
    # diagonal chain adds M[i,j-1], M[i-1,j-1], M[i-1,j] with weights 1, 2, 3
    # (1 + 4 + 9 = 14 output variances); the chain ends on the top row (one
    # more output), on the left column (weight 3: nine) or in the corner
    # (none), and eq9 adds one
    ii, jj = np.meshgrid(np.arange(1, m + 1), np.arange(1, n + 1), indexing="ij")
    base = np.where(ii < jj, 1, np.where(ii > jj, 9, 0))
    model = 14 * (d - 1) + base + 1
    fit_lo = err[d <= 8].var() / (eps ** 2 * model[d <= 8].mean())
    fit_hi = err[d >= 192].var() / (eps ** 2 * model[d >= 192].mean())
    say(f"bootstrap output error std 2^{np.log2(eps):.2f}; key error: max 2^{np.log2(worst):.2f}, "
        f"std 2^{np.log2(lo):.2f} (min(i,j) <= 8), 2^{np.log2(hi):.2f} (>= 192); "
        f"measured / model variance {fit_lo:.3f}, {fit_hi:.3f}")
    # a bootstrap's output error is about 2^48 (mostly the 41 bits the
    # one-level gadget drops: 742 * 1024 * 2^80 / 12)
    assert 2.0 ** 47.5 < eps < 2.0 ** 49
    assert 0.75 < fit_lo < 1.33 and 0.75 < fit_hi < 1.33
    assert 4.0 < hi / lo < 12.0
    assert worst < 2.0 ** 57                # half the decoding threshold (a box is 2^59 wide)
    # Section 3.1 asks the noise to stay below the decoding threshold with a
    # small failure probability: a value is lost when the key's error plus the
    # key switch's and the modulus switch's (computed from the parameters:
    # 2048 x 5 balanced base-8 digits, mean square 5.5, times the key
    # switching key's noise; the rounding of the input to 15 bits; the
    # rounding of 742 mask words and the body to multiples of 2^52) passes
    # 2^58.  With the measured key errors the two-sided Gaussian tail gives
    # the failure probability of one bootstrap at both ends of the wavefront.
    from math import erfc, log2, sqrt
    sig_ksk = float(L.lvs_params_default().lwe_noise_q64)
    var_kms = 2048 * 5 * 5.5 * sig_ksk ** 2 + 2048 * 0.5 * 2.0 ** 98 / 12 + 372 * 2.0 ** 104 / 12
    p_lo = erfc(2.0 ** 58 / sqrt(lo ** 2 + var_kms) / sqrt(2))
    p_hi = erfc(2.0 ** 58 / sqrt(hi ** 2 + var_kms) / sqrt(2))
    say(f"key switch + modulus switch error 2^{0.5 * log2(var_kms):.2f}; failure probability per bootstrap "
        f"2^{log2(p_lo):.1f} (min(i,j) <= 8), 2^{log2(p_hi):.1f} (>= 192, refresh off)")
    assert p_lo < 2.0 ** -38 and p_hi < 2.0 ** -29
