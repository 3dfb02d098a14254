"""The external product's arithmetic, simulated with Python integers in the
blind rotation's 32-bit wrapping form (no GPU): per prime, the lazy forward
transform (Cooley-Tukey with the psi^brv table, natural order in,
bit-reversed out, a butterfly adding at most 2p, never reduced), Montgomery
products with the key transform scaled by N^-1 (Q/p)^-1 2^32, the lazy
inverse transform (Gentleman-Sande, reduced to below 2p after stages 3 and 7,
the last stage feeding the CRT unreduced), then the explicit CRT.  The
eight-wave forms run the in-lane inverse stages with a sign and offset plan
(products negated, sums formed as b - a or with the next stage's bound added
where the next stage takes them so, so that a butterfly's sum and product
input take one instruction each); it is simulated in lockstep with the plain
inverse transform and must feed every Shoup product, every reduction and the
CRT the very same integers.  Every
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


def redc_offset(T, p):
    """Montgomery reduction of an input offset by 2p at its high word (below 4p)."""
    assert T < p * (1 << 32) + (2 * p << 32)
    mont = (-pow(p, -1, 1 << 32)) % (1 << 32)
    m = (T & M32) * mont & M32
    r = (T + m * p) >> 32
    assert r < 4 * p
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


def plan_mode(J, RED, chain0, el):
    """The plan's pairs at stage J of a five-stage segment (element bit J): 1 b
    negated, 2 a offset by the stage's bound (along the chain of sums of sums
    of the row segment, up to its reduction)."""
    chain = chain0 and J <= RED and (el & ((1 << J) - 1)) == 0
    return 2 if chain else 1


def plan_chain(J, RED, chain0, el):
    return chain0 and J <= RED and (el & ((1 << J) - 1)) == 0


def inverse_plan_then_crt_inputs(x, reg, p):
    """Stages 0..9 as the eight-wave forms run them, from the products x and
    the registers reg the products leave (x + 2p at even positions): in-lane
    segments of five stages (positions' bits 0..4 and 5..9, reductions at the
    segments' stages 3 and 2), the registers wrapping mod 2^32; stage 4
    negates the positions with bit 5 set and stage 9 those with bit 10 set
    (the waves holding them).  Runs the plain butterflies alongside and
    asserts that the Shoup and reduction inputs are identical and every
    register is the plain value or its negation plus a multiple of p; the
    CRT step's last stage takes u0 - u1 and u0 + u1 + 8p."""
    x = list(x)
    reg = list(reg)
    inv = TABLES[p][1]
    q = (1 << 32) // p
    for U in range(LOG_N - 1):
        t, m = 1 << U, N >> (U + 1)
        base, RED, chain0 = (0, 3, True) if U < 5 else (5, 2, False)
        J = U - base
        since = U if U <= 3 else (U - 4 if U <= 7 else U - 8)
        since_n = (U + 1) if U + 1 <= 3 else ((U - 3) if U + 1 <= 7 else U - 7)
        B, Bn = (2 * p) << since, (2 * p) << since_n

        def next_b(pos):
            if J == 4:
                return (pos >> (base + 5)) & 1           # the negated half: bit 5 (row), bit 10 (column)
            return (pos >> (base + J + 1)) & 1

        for i in range(m):
            w = inv[m + i]
            for j in range(2 * i * t, 2 * i * t + t):
                el = (j >> base) & 31
                a, b = x[j], x[j + t]
                ra, rb = reg[j], reg[j + t]
                md = plan_mode(J, RED, chain0, el)
                xin = (ra + rb + B if md == 1 else ra - rb) & M32
                assert xin == a + B - b                     # the plain product input, exactly
                s_plain = a + b
                if U in (3, 7):
                    sm = (ra - rb if md == 1 else ra + rb - B) & M32
                    assert sm == s_plain < (1 << 32)         # the plain reduction input
                    qq = ((sm * q) >> 32) * p
                    s_plain = s_plain - ((s_plain * q) >> 32) * p
                    rs = (qq - sm) if next_b(j) else (sm - qq)
                elif J == 4:
                    assert md == 1
                    rs = (rb - ra) if next_b(j) else (ra - rb)
                elif plan_chain(J + 1, RED, chain0, el):
                    assert md == 2
                    c = 0 if next_b(j) else Bn
                    rs = ra + rb + c - B
                else:
                    assert md == 1
                    rs = (rb - ra) if next_b(j) else (ra - rb)
                d_plain = shoup(xin, w, p)
                ws = (w << 32) // p
                qd = (xin * ws) >> 32
                rd = (qd * p - xin * w) if next_b(j + t) else (xin * w - qd * p)
                x[j], x[j + t] = s_plain, d_plain
                reg[j], reg[j + t] = rs & M32, rd & M32
                for r, v in ((reg[j], s_plain), (reg[j + t], d_plain)):
                    assert any((sg * v + c * p - r) % (1 << 32) == 0 for sg in (1, -1) for c in range(-32, 33))
        if U == 4:
            assert all(reg[k] == (x[k] if not (k >> 5) & 1 else (-x[k]) & M32) for k in range(N))
        if U == 9:
            assert all(reg[k] == (x[k] if not (k >> 10) & 1 else (-x[k]) & M32) for k in range(N))
    w = inv[1]
    lo, hi = [0] * (N // 2), [0] * (N // 2)
    for c in range(N // 2):
        u0, u1 = reg[c], reg[c + N // 2]
        lo[c], hi[c] = (u0 - u1) & M32, shoup((u0 + u1 + 8 * p) & M32, w, p)
    return lo + hi


def external_product_sim(d0, d1, k0, k1, planned=False):
    """X = d0 * k0 + d1 * k1 (negacyclic) mod 2^64 through the kernel's path
    (planned: the eight-wave forms' inverse stages)."""
    res = []
    for p, c in zip(P, C):
        scale = pow(N, -1, p) * c * (1 << 32) % p
        x0 = forward_lazy([d + p for d in d0], p)          # residues d + p in [0, 2p)
        x1 = forward_lazy([d + p for d in d1], p)
        K0 = [v * scale % p for v in forward_exact(k0, p)]
        K1 = [v * scale % p for v in forward_exact(k1, p)]
        prod = [redc(a * ka + b * kb, p) for a, b, ka, kb in zip(x0, x1, K0, K1)]
        plain = inverse_lazy_then_crt_inputs(prod, p)
        if planned:
            # even positions (the a elements of inverse stage 0) add 2p at the
            # high word of the Montgomery input, which leaves its low word alone
            reg = [redc_offset(a * ka + b * kb + (0 if k & 1 else (2 * p) << 32), p) if not k & 1 else prod[k]
                   for k, (a, b, ka, kb) in enumerate(zip(x0, x1, K0, K1))]
            assert all(reg[k] == prod[k] + (0 if k & 1 else 2 * p) for k in range(N))
            assert inverse_plan_then_crt_inputs(prod, reg, p) == plain
        res.append(plain)
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


@pytest.mark.parametrize("planned", [False, True], ids=["plain", "planned"])
@pytest.mark.parametrize("case", ["random", "extreme_neg", "extreme_mixed"])
def test_external_product_matches_exact(case, planned):
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
    got = external_product_sim(d0, d1, k0, k1, planned)
    want = negacyclic_mod64(d0, k0) + negacyclic_mod64(d1, k1)
    assert (got == want).all()
