"""Seeded synthetic inputs for the five benchmark workloads.

This module only draws strings (and serving arrival times); it holds none of
the method's arithmetic and is the one piece of code that both the HIP
library's tests/benchmark and the CPU oracle use.

The paper (arXiv 2508.14568) names no dataset: its timings use ASCII strings
(Section 6) and a 210-base DNA pair for the MPC comparison (Section 6.3).  The
recipes below stand in for them:

  tiny_dna      2 DNA strings of 6 bases, uniform over ACGT.
  plain_ascii   one pair of 32 ASCII letters; the second string is uniform
                except that round(0.2 * 32) = 6 positions, drawn without
                replacement, copy the first string's letter.
  batched       256 pairs, lengths m, n uniform in [8, 64], uniform letters.
  dna_align     a 256-base string and a copy with 5% random edits (each
                position independently: substitution, insertion or deletion
                with equal chance), truncated or padded to 256 bases.
  serving       1024 server names and a stream of query names, lengths
                clip(round(LogNormal(ln 15 - s^2/2, s = 0.5)), 2, 64); half the
                queries copy a server name with 1-2 random edits; Poisson
                arrivals.
  wide_symbols  a pair of 32-symbol strings over 64 distinct symbols drawn
                uniformly below 2^21 (the range of Unicode code points); the
                second string is uniform except that 20% of its positions,
                drawn without replacement, copy the first string's symbol.
"""
import math

import numpy as np

LETTERS = bytes(range(ord("A"), ord("Z") + 1)) + bytes(range(ord("a"), ord("z") + 1))
DNA = b"ACGT"


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_letters(rng, length: int) -> bytes:
    return bytes(LETTERS[k] for k in rng.integers(0, len(LETTERS), size=length))


def random_dna(rng, length: int) -> bytes:
    return bytes(DNA[k] for k in rng.integers(0, 4, size=length))


def dna_codes(s: bytes) -> bytes:
    """A, C, G, T -> 0, 1, 2, 3."""
    return bytes(DNA.index(c) for c in s)


def tiny_dna(seed: int = 1):
    rng = _rng(seed)
    return random_dna(rng, 6), random_dna(rng, 6)


def plain_ascii(seed: int = 2, length: int = 32, copy_frac: float = 0.2):
    rng = _rng(seed)
    a = random_letters(rng, length)
    b = bytearray(random_letters(rng, length))
    k = int(round(copy_frac * length))
    for pos in rng.choice(length, size=k, replace=False):
        b[pos] = a[pos]
    return a, bytes(b)


def batched(seed: int = 3, count: int = 256, lo: int = 8, hi: int = 64):
    rng = _rng(seed)
    pairs = []
    for _ in range(count):
        m, n = (int(x) for x in rng.integers(lo, hi + 1, size=2))
        pairs.append((random_letters(rng, m), random_letters(rng, n)))
    return pairs


def mutate(rng, s: bytes, p: float, alphabet: bytes) -> bytes:
    out = bytearray()
    for c in s:
        if rng.random() < p:
            kind = int(rng.integers(0, 3))
            if kind == 0:                       # substitution by another symbol
                choices = [x for x in alphabet if x != c]
                out.append(choices[int(rng.integers(0, len(choices)))])
            elif kind == 1:                     # insertion before c
                out.append(alphabet[int(rng.integers(0, len(alphabet)))])
                out.append(c)
            # kind == 2: deletion
        else:
            out.append(c)
    return bytes(out)


def dna_align(seed: int = 4, length: int = 256, p: float = 0.05):
    rng = _rng(seed)
    a = random_dna(rng, length)
    b = mutate(rng, a, p, DNA)
    if len(b) > length:
        b = b[:length]
    elif len(b) < length:
        b = b + random_dna(rng, length - len(b))
    return a, b


def name_length(rng, sigma: float = 0.5, mean: float = 15.0, lo: int = 2, hi: int = 64) -> int:
    mu = math.log(mean) - sigma * sigma / 2
    return int(min(hi, max(lo, round(rng.lognormal(mu, sigma)))))


def serving(seed: int = 5, n_server: int = 1024, n_queries: int = 200):
    """Server list, queries, and which queries copy a server name."""
    rng = _rng(seed)
    server = [random_letters(rng, name_length(rng)) for _ in range(n_server)]
    queries = []
    for _ in range(n_queries):
        if rng.random() < 0.5:
            base = server[int(rng.integers(0, n_server))]
            q = base
            for _ in range(int(rng.integers(1, 3))):
                q = _one_edit(rng, q)
            q = q[:64] if len(q) > 64 else q
            queries.append(q if len(q) >= 1 else base)
        else:
            queries.append(random_letters(rng, name_length(rng)))
    return server, queries


def _one_edit(rng, s: bytes) -> bytes:
    kind = int(rng.integers(0, 3)) if len(s) > 1 else 1
    pos = int(rng.integers(0, len(s) + (1 if kind == 1 else 0)))
    c = LETTERS[int(rng.integers(0, len(LETTERS)))]
    if kind == 0:
        return s[:pos] + bytes([c]) + s[pos + 1:]
    if kind == 1:
        return s[:pos] + bytes([c]) + s[pos:]
    return s[:pos] + s[pos + 1:]


def poisson_arrivals(seed: int, rate_per_s: float, count: int):
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def batched_sample(seed: int = 33, count: int = 8, total: int = 256):
    """Indices of the batched pairs whose every ciphertext is checked."""
    return sorted(int(k) for k in _rng(seed).choice(total, size=count, replace=False))


def serving_sample(seed: int = 55, queries: int = 2, names: int = 32, n_queries: int = 200, n_server: int = 1024):
    """Queries and server names whose every ciphertext is checked."""
    rng = _rng(seed)
    q = sorted(int(k) for k in rng.choice(n_queries, size=queries, replace=False))
    nm = sorted(int(k) for k in rng.choice(n_server, size=names, replace=False))
    return q, nm


def alphabet_of(strings) -> bytes:
    return bytes(sorted(set(b"".join(strings))))


def wide_symbols(seed: int = 7, length: int = 32, width: int = 21, alphabet: int = 64, copy_frac: float = 0.2):
    rng = _rng(seed)
    symbols = []
    while len(symbols) < alphabet:
        v = int(rng.integers(0, 2 ** width))
        if v not in symbols:
            symbols.append(v)
    a = [symbols[int(k)] for k in rng.integers(0, alphabet, size=length)]
    b = [symbols[int(k)] for k in rng.integers(0, alphabet, size=length)]
    for pos in rng.choice(length, size=int(round(copy_frac * length)), replace=False):
        b[pos] = a[pos]
    return a, b
