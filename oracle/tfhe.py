"""Oracle, TFHE layer -- TEST INFRASTRUCTURE ONLY.

Python face of ``tfhe_ref.c`` (plain schoolbook TFHE over Z/2^64) plus the
pieces that are clearer in numpy: the lookup-table test polynomials and the
linear operations on ciphertexts.  Only ``tests/``, the package smoke check and
the benchmark's CPU-baseline leg may import this module.

Paper references (arXiv 2508.14568):
  * Section 2.2 (TFHE): 5-bit plaintext space with a padding bit, linear
    operations are cheap, a programmable bootstrap applies any lookup table,
    and inputs with the padding bit set return the negated table entry
    (Table "LUT for f(x) = x - 4").
  * The scheme internals (key switch, modulus switch, blind rotation, sample
    extraction) are cited, not given; the readings used here are the ones
    listed in the design notes and pinned by the tests.
"""
import ctypes
import os

import numpy as np

from . import build as _build

U64 = np.uint64
DELTA_LOG = 59                      # value x in Z_32 encodes as x * 2^59
DELTA = 1 << DELTA_LOG


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("N", ctypes.c_int),
                ("pbs_base_log", ctypes.c_int), ("pbs_level", ctypes.c_int),
                ("ks_base_log", ctypes.c_int), ("ks_level", ctypes.c_int),
                ("lwe_sigma_q64", ctypes.c_uint64), ("glwe_sigma_q64", ctypes.c_uint64)]


def default_params() -> Params:
    """n=742, k=1, N=2048, q=2^64, bootstrap gadget 2^23 x 1, key switch 2^3 x 5;
    noise std 7.069849454709433e-06 and 2.9403601535432533e-16 of q."""
    return Params(742, 2048, 23, 1, 3, 5, 130415703530680, 5424)


def toy_params() -> Params:
    """Small insecure parameters with the same structure, for fast pins."""
    return Params(32, 512, 23, 1, 3, 5, 130415703530680, 5424)


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        u64p, i64p, u32p, u8p = P(ctypes.c_uint64), P(ctypes.c_int64), P(ctypes.c_uint32), P(ctypes.c_uint8)
        L.orc_stream_key.restype = ctypes.c_uint64
        L.orc_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_draw.restype = ctypes.c_uint64
        L.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_gaussian.restype = ctypes.c_uint64
        L.orc_gaussian.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_negacyclic_mac.restype = None
        L.orc_negacyclic_mac.argtypes = [u64p, u64p, i64p, ctypes.c_int]
        L.orc_negacyclic_mac_karatsuba.restype = None
        L.orc_negacyclic_mac_karatsuba.argtypes = [u64p, u64p, i64p, ctypes.c_int]
        L.orc_keys_set_karatsuba.restype = None
        L.orc_keys_set_karatsuba.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_monomial_mul.restype = None
        L.orc_monomial_mul.argtypes = [u64p, u64p, ctypes.c_int, ctypes.c_int]
        L.orc_decompose.restype = None
        L.orc_decompose.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, i64p]
        L.orc_keygen.restype = ctypes.c_void_p
        L.orc_keygen.argtypes = [P(Params), ctypes.c_uint64, ctypes.c_int]
        L.orc_keys_free.restype = None
        L.orc_keys_free.argtypes = [ctypes.c_void_p]
        for f in ("orc_keys_small", "orc_keys_big"):
            getattr(L, f).restype = u8p
            getattr(L, f).argtypes = [ctypes.c_void_p]
        for f in ("orc_keys_bsk", "orc_keys_ksk"):
            getattr(L, f).restype = u64p
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.orc_encrypt.restype = None
        L.orc_encrypt.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.orc_phase.restype = ctypes.c_uint64
        L.orc_phase.argtypes = [ctypes.c_void_p, u64p]
        L.orc_phase_small.restype = ctypes.c_uint64
        L.orc_phase_small.argtypes = [ctypes.c_void_p, u64p]
        L.orc_keyswitch.restype = None
        L.orc_keyswitch.argtypes = [ctypes.c_void_p, u64p, u64p]
        L.orc_modswitch.restype = None
        L.orc_modswitch.argtypes = [ctypes.c_int, ctypes.c_int, u64p, u32p]
        L.orc_blind_rotate.restype = None
        L.orc_blind_rotate.argtypes = [ctypes.c_void_p, u64p, u32p, u64p]
        L.orc_sample_extract.restype = None
        L.orc_sample_extract.argtypes = [ctypes.c_int, u64p, u64p]
        L.orc_pbs.restype = None
        L.orc_pbs.argtypes = [ctypes.c_void_p, u64p, u64p, u64p]
        L.orc_pbs_batch.restype = None
        L.orc_pbs_batch.argtypes = [ctypes.c_void_p, u64p, P(ctypes.c_int32), u64p, ctypes.c_size_t, u64p,
                                    ctypes.c_int]
        _LIB = L
    return _LIB


def _p(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ----------------------------------------------------------------- PRNG

def stream_key(seed: int, tag: int) -> int:
    return int(lib().orc_stream_key(seed, tag))


def draw(key: int, i: int) -> int:
    return int(lib().orc_draw(key, i))


def gaussian(key: int, idx: int, sigma_q64: int) -> int:
    return int(lib().orc_gaussian(key, idx, sigma_q64))


# ------------------------------------------------ polynomial arithmetic

def negacyclic_mul(a: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Schoolbook product of a (u64 torus coefficients) and d (small signed
    integers) in Z_{2^64}[X]/(X^N + 1)."""
    a = np.ascontiguousarray(a, dtype=U64)
    d = np.ascontiguousarray(d, dtype=np.int64)
    out = np.zeros_like(a)
    lib().orc_negacyclic_mac(_p(out, ctypes.c_uint64), _p(a, ctypes.c_uint64), _p(d, ctypes.c_int64), a.size)
    return out


def negacyclic_mul_karatsuba(a: np.ndarray, d: np.ndarray) -> np.ndarray:
    """The same product through Karatsuba's recursion (exact in Z/2^64; N a
    power of two)."""
    a = np.ascontiguousarray(a, dtype=U64)
    d = np.ascontiguousarray(d, dtype=np.int64)
    out = np.zeros_like(a)
    lib().orc_negacyclic_mac_karatsuba(_p(out, ctypes.c_uint64), _p(a, ctypes.c_uint64), _p(d, ctypes.c_int64),
                                       a.size)
    return out


def monomial_mul(a: np.ndarray, e: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=U64)
    out = np.zeros_like(a)
    lib().orc_monomial_mul(_p(out, ctypes.c_uint64), _p(a, ctypes.c_uint64), int(e), a.size)
    return out


def decompose(c: int, base_log: int, level: int) -> list:
    out = (ctypes.c_int64 * level)()
    lib().orc_decompose(ctypes.c_uint64(c & (2**64 - 1)), base_log, level, out)
    return [int(v) for v in out]


# ---------------------------------------------------------- lookup tables

def test_polynomial(f16, N: int) -> np.ndarray:
    """Test polynomial of a 16-entry table f: Z_16 -> Z_32.  Coefficient t
    holds f(t // (N/16)) * 2^59, then the whole polynomial is multiplied by
    X^(-N/32) so that every plaintext value sits in the middle of its box
    (Section 2.2: the table is read by the bootstrap's rotation; the right half
    of the 5-bit space returns the negated entry)."""
    box = N // 16
    v = np.array([(int(f16[t // box]) % 32) << DELTA_LOG for t in range(N)], dtype=U64)
    return monomial_mul(v, 2 * N - box // 2)


# ------------------------------------------------------------------ keys

class Keys:
    """Client and server keys drawn from one seed (see tfhe_ref.c)."""

    def __init__(self, params: Params = None, seed: int = 0, nthreads: int = None, karatsuba: bool = False):
        self.params = params or default_params()
        self.seed = seed
        self.n, self.N = self.params.n, self.params.N
        self._h = lib().orc_keygen(ctypes.byref(self.params), seed, nthreads or default_threads())
        if not self._h:
            raise MemoryError("oracle keygen failed")
        self.karatsuba = karatsuba

    @property
    def karatsuba(self) -> bool:
        """Whether the blind rotation multiplies through Karatsuba's recursion
        instead of the schoolbook sum (same words; about 4x faster)."""
        return self._kara

    @karatsuba.setter
    def karatsuba(self, on: bool):
        self._kara = bool(on)
        lib().orc_keys_set_karatsuba(self._h, int(self._kara))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            try:
                _LIB.orc_keys_free(h)
            except TypeError:       # interpreter shutdown
                pass
            self._h = None

    @property
    def small_key(self) -> np.ndarray:
        return np.ctypeslib.as_array(lib().orc_keys_small(self._h), shape=(self.n,)).copy()

    @property
    def big_key(self) -> np.ndarray:
        return np.ctypeslib.as_array(lib().orc_keys_big(self._h), shape=(self.N,)).copy()

    def bsk(self) -> np.ndarray:
        R = 2 * self.params.pbs_level
        return np.ctypeslib.as_array(lib().orc_keys_bsk(self._h), shape=(self.n, R, 2, self.N)).copy()

    def ksk(self) -> np.ndarray:
        rows = self.N * self.params.ks_level
        return np.ctypeslib.as_array(lib().orc_keys_ksk(self._h), shape=(rows, self.n + 1)).copy()

    # --- encryption --------------------------------------------------------
    def encrypt(self, mu: int, seed: int, index: int) -> np.ndarray:
        ct = np.zeros(self.N + 1, dtype=U64)
        lib().orc_encrypt(self._h, int(mu) % 32, seed, index, _p(ct, ctypes.c_uint64))
        return ct

    def phase(self, ct: np.ndarray) -> int:
        ct = np.ascontiguousarray(ct, dtype=U64)
        return int(lib().orc_phase(self._h, _p(ct, ctypes.c_uint64)))

    def phase_small(self, ct: np.ndarray) -> int:
        ct = np.ascontiguousarray(ct, dtype=U64)
        return int(lib().orc_phase_small(self._h, _p(ct, ctypes.c_uint64)))

    def decrypt(self, ct: np.ndarray) -> int:
        """Value in Z_32: the phase rounded to the nearest multiple of 2^59."""
        return (((self.phase(ct) >> (DELTA_LOG - 1)) + 1) >> 1) % 32

    def decrypt_signed(self, ct: np.ndarray) -> int:
        v = self.decrypt(ct)
        return v - 32 if v >= 16 else v

    def phase_error(self, ct: np.ndarray) -> int:
        """Signed distance between the phase and the nearest encoded value."""
        ph = self.phase(ct)
        err = (ph - (self.decrypt(ct) << DELTA_LOG)) % 2**64
        return err - 2**64 if err >= 2**63 else err

    # --- bootstrap pieces ---------------------------------------------------
    def keyswitch(self, ct: np.ndarray) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=U64)
        out = np.zeros(self.n + 1, dtype=U64)
        lib().orc_keyswitch(self._h, _p(ct, ctypes.c_uint64), _p(out, ctypes.c_uint64))
        return out

    def modswitch(self, small: np.ndarray) -> np.ndarray:
        small = np.ascontiguousarray(small, dtype=U64)
        out = np.zeros(self.n + 1, dtype=np.uint32)
        lib().orc_modswitch(self.n, self.N, _p(small, ctypes.c_uint64), _p(out, ctypes.c_uint32))
        return out

    def blind_rotate(self, testpoly: np.ndarray, ms: np.ndarray) -> np.ndarray:
        testpoly = np.ascontiguousarray(testpoly, dtype=U64)
        ms = np.ascontiguousarray(ms, dtype=np.uint32)
        acc = np.zeros(2 * self.N, dtype=U64)
        lib().orc_blind_rotate(self._h, _p(testpoly, ctypes.c_uint64), _p(ms, ctypes.c_uint32),
                               _p(acc, ctypes.c_uint64))
        return acc

    def sample_extract(self, acc: np.ndarray) -> np.ndarray:
        acc = np.ascontiguousarray(acc, dtype=U64)
        out = np.zeros(self.N + 1, dtype=U64)
        lib().orc_sample_extract(self.N, _p(acc, ctypes.c_uint64), _p(out, ctypes.c_uint64))
        return out

    def pbs(self, ct: np.ndarray, testpoly: np.ndarray) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=U64)
        testpoly = np.ascontiguousarray(testpoly, dtype=U64)
        out = np.zeros(self.N + 1, dtype=U64)
        lib().orc_pbs(self._h, _p(testpoly, ctypes.c_uint64), _p(ct, ctypes.c_uint64), _p(out, ctypes.c_uint64))
        return out

    def pbs_batch(self, cts: np.ndarray, testpolys: np.ndarray, lut_ids, nthreads: int = None) -> np.ndarray:
        """Independent bootstraps: row b of cts through testpolys[lut_ids[b]]."""
        cts = np.ascontiguousarray(cts, dtype=U64).reshape(-1, self.N + 1)
        testpolys = np.ascontiguousarray(testpolys, dtype=U64).reshape(-1, self.N)
        ids = np.ascontiguousarray(np.broadcast_to(np.asarray(lut_ids, dtype=np.int32), (cts.shape[0],)))
        assert ids.size == 0 or (ids.min() >= 0 and ids.max() < testpolys.shape[0])
        out = np.zeros_like(cts)
        if cts.shape[0]:
            lib().orc_pbs_batch(self._h, _p(testpolys, ctypes.c_uint64), _p(ids, ctypes.c_int32),
                                _p(cts, ctypes.c_uint64), cts.shape[0], _p(out, ctypes.c_uint64),
                                nthreads or default_threads())
        return out


# --------------------------------------------------------- linear operations
# Ciphertexts are u64 vectors (a_0..a_{N-1}, b); numpy's uint64 arithmetic
# wraps modulo 2^64, which is the torus arithmetic of the scheme.

def trivial(mu: int, N: int) -> np.ndarray:
    """Noise-free encryption of mu: a = 0, b = mu * 2^59."""
    ct = np.zeros(N + 1, dtype=U64)
    ct[N] = U64((int(mu) % 32) << DELTA_LOG)
    return ct


def scale(ct: np.ndarray, k: int) -> np.ndarray:
    return (ct * U64(k % 2**64)).astype(U64)
