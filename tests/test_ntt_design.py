"""The external product's arithmetic, simulated with Python integers in the
blind rotation's 32-bit wrapping form (no GPU): per prime, the lazy forward
transform (Cooley-Tukey with the psi^brv table, natural order in,
bit-reversed out, a butterfly adding at most 2p, never reduced), Montgomery
products with the key transform scaled by N^-1 (Q/p)^-1 2^32, the lazy
inverse transform (Gentleman-Sande, reduced to below 2p after stages 3 and 7,
the last stage feeding the CRT unreduced), then the explicit CRT.  Every
intermediate value is checked against the bounds the kernel relies on (below
2^31, subtrahends below the added bound, Montgomery inputs below p 2^32),
and the result against the exact negacyclic product mod 2^64, at random
inputs and at the extremes: every digit -2^22 or 2^22 - 1, every key word
-2^63 or 2^63 - 1 (read signed), so |X| reaches 2 N 2^22 2^63 = 2^97."""
import numpy as np
import pytest

from test_crt_design import C, P, lift

N = 2048
LOG_N = 11
M32 = (1 << 32) - 1


def bitrev(x, bits=LOG_N):
    return int(format(x, f"0{bits}b")[::-1], 2)


def tables(p):
    x = 2
    while True:
        psi = pow(x, (p - 1) // (2 * N), p)
        if pow(psi, N, p) == p - 1:
            break
        x += 1
    psi_inv = pow(psi, p - 2, p)
    fwd = [pow(psi, bitrev(k), p) for k in range(N)]
    inv = [pow(psi_inv, bitrev(k), p) for k in range(N)]
    return fwd, inv


TABLES = {p: tables(p) for p in P}


def shoup(a, w, p):
    """a w mod p in [0, 2p) with the Shoup companion floor(w 2^32 / p)."""
    assert a < (1 << 32)
    ws = (w << 32) // p
    q = (a * ws) >> 32
    r = (a * w - q * p) & M32
    assert r < 2 * p
    return r


def forward_lazy(x, p):
    x = list(x)
    fwd = TABLES[p][0]
    for S in range(LOG_N):
        m, t = 1 << S, N >> (S + 1)
        for i in range(m):
            w = fwd[m + i]
            for j in range(2 * i * t, 2 * i * t + t):
                a, b = x[j], x[j + t]
                tt = shoup(b, w, p)
                x[j], x[j + t] = a + tt, a + 2 * p - tt
        assert max(x) < 2 * p * (S + 2)          # a stage adds at most 2p
    assert max(x) < 24 * p < (1 << 31)
    return x


def forward_exact(x, p):
    """The same transform with every value reduced (the key's conversion)."""
    x = [v % p for v in x]
    fwd = TABLES[p][0]
    for S in range(LOG_N):
        m, t = 1 << S, N >> (S + 1)
        for i in range(m):
            w = fwd[m + i]
            for j in range(2 * i * t, 2 * i * t + t):
                a, b = x[j], x[j + t] * w % p
                x[j], x[j + t] = (a + b) % p, (a - b) % p
    return x


def redc(T, p):
    assert T < p * (1 << 32)
    mont = (-pow(p, -1, 1 << 32)) % (1 << 32)
    m = (T & M32) * mont & M32
    r = (T + m * p) >> 32
    assert r < 2 * p
    return r


def inverse_lazy_then_crt_inputs(x, p):
    """Stages 0..9 with the kernel's bounds, then the last stage as the CRT
    step forms it: (u0 + u1, Shoup(u0 + 8p - u1)) for positions c, c + N/2."""
    x = list(x)
    inv = TABLES[p][1]
    q = (1 << 32) // p
    for U in range(LOG_N - 1):
        t, m = 1 << U, N >> (U + 1)
        since = U if U <= 3 else (U - 4 if U <= 7 else U - 8)
        bound = (2 * p) << since
        for i in range(m):
            w = inv[m + i]
            for j in range(2 * i * t, 2 * i * t + t):
                a, b = x[j], x[j + t]
                assert a < bound and b < bound
                s = a + b
                if U in (3, 7):
                    s = s - ((s * q) >> 32) * p
                    assert s < 2 * p
                x[j], x[j + t] = s, shoup(a + bound - b, w, p)
        assert max(x) < (1 << 31)
    w = inv[1]
    lo, hi = [0] * (N // 2), [0] * (N // 2)
    for c in range(N // 2):
        u0, u1 = x[c], x[c + N // 2]
        assert u0 < 8 * p and u1 < 8 * p
        lo[c], hi[c] = u0 + u1, shoup(u0 + 8 * p - u1, w, p)
        assert lo[c] < 16 * p < (1 << 30)
    return lo + hi


def external_product_sim(d0, d1, k0, k1):
    """X = d0 * k0 + d1 * k1 (negacyclic) mod 2^64 through the kernel's path."""
    res = []
    for p, c in zip(P, C):
        scale = pow(N, -1, p) * c * (1 << 32) % p
        x0 = forward_lazy([d + p for d in d0], p)          # residues d + p in [0, 2p)
        x1 = forward_lazy([d + p for d in d1], p)
        K0 = [v * scale % p for v in forward_exact(k0, p)]
        K1 = [v * scale % p for v in forward_exact(k1, p)]
        prod = [redc(a * ka + b * kb, p) for a, b, ka, kb in zip(x0, x1, K0, K1)]
        res.append(inverse_lazy_then_crt_inputs(prod, p))
    return np.array([lift([r[i] for r in res]) for i in range(N)], dtype=np.uint64)


def negacyclic_mod64(d, k):
    d = np.array([v & ((1 << 64) - 1) for v in d], dtype=np.uint64)
    k = np.array([v & ((1 << 64) - 1) for v in k], dtype=np.uint64)
    out = np.zeros(N, dtype=np.uint64)
    for j in range(N):
        shifted = np.roll(k, j)
        shifted[:j] = np.uint64(0) - shifted[:j]        # X^N = -1
        out += d[j] * shifted
    return out


@pytest.mark.parametrize("case", ["random", "extreme_neg", "extreme_mixed"])
def test_external_product_matches_exact(case):
    rng = np.random.default_rng({"random": 1, "extreme_neg": 2, "extreme_mixed": 3}[case])
    lo_d, hi_d = -(1 << 22), (1 << 22) - 1
    if case == "random":
        d0 = [int(v) for v in rng.integers(lo_d, hi_d + 1, size=N)]
        d1 = [int(v) for v in rng.integers(lo_d, hi_d + 1, size=N)]
        k0 = [int(v) for v in rng.integers(-(1 << 63), (1 << 63) - 1, size=N, dtype=np.int64)]
        k1 = [int(v) for v in rng.integers(-(1 << 63), (1 << 63) - 1, size=N, dtype=np.int64)]
    elif case == "extreme_neg":
        d0 = d1 = [lo_d] * N
        k0 = k1 = [-(1 << 63)] * N
    else:
        d0 = [lo_d if rng.random() < 0.5 else hi_d for _ in range(N)]
        d1 = [lo_d if rng.random() < 0.5 else hi_d for _ in range(N)]
        k0 = [-(1 << 63) if rng.random() < 0.5 else (1 << 63) - 1 for _ in range(N)]
        k1 = [-(1 << 63) if rng.random() < 0.5 else (1 << 63) - 1 for _ in range(N)]
    got = external_product_sim(d0, d1, k0, k1)
    want = negacyclic_mod64(d0, k0) + negacyclic_mod64(d1, k1)
    assert (got == want).all()
