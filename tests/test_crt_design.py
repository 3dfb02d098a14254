"""The explicit CRT of the blind rotation, checked with Python integers at
its bounds (no GPU).  The products of the external product are integers X
with |X| <= N * 2^22 * 2^63 = 2^96 (a balanced 23-bit digit times a 64-bit
key word, summed over N = 2048 terms); the kernel holds X as residues y_i of
X (Q/p_i)^-1 mod p_i, each any representative below 2^30 (the inverse
transform leaves them unreduced), for the four largest primes p_i < 2^26
with p_i = 1 mod 2N, and adds X mod 2^64 to the accumulator as

    acc + sum y_i (Q/p_i) - K Q  (mod 2^64),
    K = (2^23 + sum floor(y_i floor(2^56/p_i) / 2^32)) >> 24  (32-bit words),

i.e. K is the integer nearest sum y_i / p_i from a 24-bit fixed-point sum of
32-bit high products; the 64-bit sum takes the products with the low words of
Q/p_i and -Q as 64-bit multiply-adds and those with the high words as 32-bit
low products added at bit 32.  This checks that reading against exact integer
arithmetic at random X, at +-2^97 and near every point where sum y_i / p_i is
half an integer away from K, for residues at both ends of their range, with
every 32-bit intermediate asserted below 2^32."""
import random

N = 2048


def is_prime(n):
    if n < 2:
        return False
    for d in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % d == 0:
            return n == d
    d, s = n - 1, 0
    while d % 2 == 0:
        d, s = d // 2, s + 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes():
    out, k = [], ((1 << 26) - 1) // (2 * N)
    while len(out) < 4:
        p = k * 2 * N + 1
        if p < (1 << 26) and is_prime(p):
            out.append(p)
        k -= 1
    return out


P = primes()
Q = P[0] * P[1] * P[2] * P[3]
M = [Q // p for p in P]
G = [(1 << 57) // p for p in P]
C = [pow(Q // p, -1, p) for p in P]
MASK = (1 << 64) - 1


def lift(y, acc=0):
    """The kernel's formula, in 32- and 64-bit wrapping arithmetic: acc + X mod 2^64."""
    s = 1 << 23
    h = 0
    r = acc
    for yi, gi, mi in zip(y, G, M):
        assert 0 <= yi < (1 << 30)
        s += (yi * (gi >> 1)) >> 32                # __umulhi(y_i, floor(2^56 / p_i))
        assert s < (1 << 32)
        r = (r + yi * (mi & 0xFFFFFFFF)) & MASK    # 64-bit multiply-add, low word of Q/p_i
        h = (h + yi * ((mi & MASK) >> 32)) & 0xFFFFFFFF
    k = s >> 24
    nq = (-Q) & MASK
    r = (r + k * (nq & 0xFFFFFFFF)) & MASK
    h = (h + k * (nq >> 32)) & 0xFFFFFFFF
    return (r + (h << 32)) & MASK


def residues(X, rng, pick):
    """y_i = X (Q/p_i)^-1 mod p_i plus a multiple of p_i, below 2^30:
    pick 'low' (reduced), 'high' (largest) or 'random'."""
    y = []
    for p, c in zip(P, C):
        r = X * c % p
        top = ((1 << 30) - 1 - r) // p
        k = {"low": 0, "high": top, "random": rng.randint(0, top)}[pick]
        y.append(r + k * p)
    return y


def test_primes_and_range():
    assert all(p < (1 << 26) and p % (2 * N) == 1 for p in P)
    assert min(P) > 2 ** 25.9                   # sum y_i / p_i < 64.1, so the 24-bit sum stays below 2^31
    assert all(g >> 1 == (1 << 56) // p for g, p in zip(G, P))
    assert len(set(P)) == 4
    assert Q / (1 << 97) > 2 ** 6.9             # |X| <= 2^97 keeps X / Q within 2^-6.9 of 0
    # the bound of X: a balanced digit |d| <= 2^22 times |key word| <= 2^63, N terms
    assert N * (1 << 22) * (1 << 63) <= (1 << 97)


def test_lift_exact_at_random_and_extreme_values():
    rng = random.Random(2508)
    xs = [0, 1, -1, (1 << 97), -(1 << 97), (1 << 96) - 1, -(1 << 96) + 1, (1 << 64), -(1 << 64)]
    xs += [rng.randint(-(1 << 97), 1 << 97) for _ in range(3000)]
    xs += [rng.randint(-(1 << 40), 1 << 40) for _ in range(500)]
    for X in xs:
        for pick in ("low", "high", "random"):
            assert lift(residues(X, rng, pick)) == X & MASK, (X, pick)
            acc = rng.getrandbits(64)
            assert lift(residues(X, rng, pick), acc) == (acc + X) & MASK, (X, pick)


def test_lift_exact_where_the_rounding_is_tightest():
    """X = K Q + r with K Q's neighbours: sum y_i / p_i = K' + X / Q, so the
    fixed-point sum is hardest to round when X / Q is farthest from 0, i.e.
    |X| at its bound; walk X over the last 2^20 values below +-2^97 with
    every residue pick."""
    rng = random.Random(14568)
    for sign in (1, -1):
        for _ in range(400):
            X = sign * ((1 << 97) - rng.randint(0, 1 << 20))
            for pick in ("low", "high", "random"):
                assert lift(residues(X, rng, pick)) == X & MASK
