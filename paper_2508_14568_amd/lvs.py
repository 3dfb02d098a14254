"""Python binding of liblvs (argument marshalling only).

Every function mirrors the C entry point of the same name declared in
``include/lvs.h``; all computation happens in the library's host code and HIP
kernels.  PyTorch supplies device memory (tensors used as raw buffers) and the
HIP stream.  The library must be built (``paper_2508_14568_amd.build``); there
is no fallback: loading fails loudly when it is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblvs.so")

LVS_ENC_ASCII7 = 0
LVS_ENC_DNA2 = 1
LVS_LUT_EQ, LVS_LUT_EQ9, LVS_LUT_MIN, LVS_LUT_REFRESH, LVS_LUT_MAX, LVS_LUT_MAX9 = 0, 1, 2, 3, 4, 5
LVS_LUT_USER, LVS_LUT_SLOTS = 6, 8
LVS_REFRESH_DEFAULT, LVS_REFRESH_MIN, LVS_REFRESH_MAX, LVS_MAX_DEPTH_NO_REFRESH = 256, 4, 512, 256
LVS_MAX_LEN = 1 << 20
CT_WORDS = 2049

ERRORS = {-1: "LVS_E_INVAL", -2: "LVS_E_ALPHABET", -3: "LVS_E_NOISE_BUDGET", -4: "LVS_E_NOMEM_HOST",
          -5: "LVS_E_NOMEM_DEVICE", -6: "LVS_E_DEVICE", -7: "LVS_E_PARAMS"}


class LvsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lvs_params(ctypes.Structure):
    _fields_ = [("n_lwe", ctypes.c_uint32), ("glwe_k", ctypes.c_uint32), ("poly_N", ctypes.c_uint32),
                ("pbs_base_log", ctypes.c_uint32), ("pbs_level", ctypes.c_uint32),
                ("ks_base_log", ctypes.c_uint32), ("ks_level", ctypes.c_uint32),
                ("lwe_noise_q64", ctypes.c_uint64), ("glwe_noise_q64", ctypes.c_uint64)]


_L = None
VP, SZ, U64, I32, U32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32

# name -> (restype, argtypes)
_SIGS = {
    "lvs_last_error": (ctypes.c_char_p, []),
    "lvs_params_default": (I32, [ctypes.POINTER(lvs_params)]),
    "lvs_ct_words": (SZ, []),
    "lvs_keygen": (I32, [ctypes.POINTER(lvs_params), U64, ctypes.POINTER(VP), ctypes.POINTER(VP)]),
    "lvs_lwe_encrypt": (I32, [VP, U32, U64, U64, VP]),
    "lvs_lwe_decrypt": (I32, [VP, VP, ctypes.POINTER(U32), ctypes.POINTER(ctypes.c_int64)]),
    "lvs_encrypt_string": (I32, [VP, VP, SZ, I32, U64, VP]),
    "lvs_decrypt_distance": (I32, [VP, VP, SZ, SZ, ctypes.POINTER(ctypes.c_int64)]),
    "lvs_key_export": (I32, [VP, VP, I32, VP, ctypes.POINTER(SZ)]),
    "lvs_export": (I32, [I32, VP, SZ, VP, ctypes.POINTER(SZ)]),
    "lvs_import_key": (I32, [VP, SZ, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(VP)]),
    "lvs_import_ciphertexts": (I32, [VP, SZ, VP, ctypes.POINTER(SZ)]),
    "lvs_context_bytes": (I32, [ctypes.POINTER(lvs_params), ctypes.POINTER(SZ)]),
    "lvs_context_create": (I32, [VP, I32, VP, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_context_set_stream": (I32, [VP, VP]),
    "lvs_context_set_lut": (I32, [VP, I32, ctypes.POINTER(ctypes.c_int32)]),
    "lvs_sync": (I32, [VP]),
    "lvs_pbs_workspace_bytes": (SZ, [SZ]),
    "lvs_pbs_batch": (I32, [VP, VP, VP, I32, SZ, VP, VP, SZ]),
    "lvs_pbs_batch_static": (I32, [VP, VP, VP, I32, SZ, VP]),
    "lvs_equality_workspace_bytes": (SZ, [SZ, SZ, I32]),
    "lvs_equality": (I32, [VP, VP, SZ, VP, SZ, I32, VP, VP, SZ]),
    "lvs_edit_distance_eq9_workspace_bytes": (SZ, [SZ, SZ]),
    "lvs_edit_distance_eq9": (I32, [VP, VP, SZ, SZ, VP, VP, VP, SZ]),
    "lvs_edit_distance_workspace_bytes": (SZ, [SZ, SZ, I32]),
    "lvs_edit_distance": (I32, [VP, VP, SZ, VP, SZ, I32, VP, VP, SZ]),
    "lvs_preprocess_workspace_bytes": (SZ, [SZ, SZ, I32]),
    "lvs_preprocess": (I32, [VP, VP, SZ, I32, VP, SZ, VP, VP, SZ]),
    "lvs_edit_distance_clear_workspace_bytes": (SZ, [SZ, SZ]),
    "lvs_edit_distance_clear": (I32, [VP, VP, SZ, VP, SZ, VP, SZ, VP, VP, SZ]),
    "lvs_band_exact": (SZ, [SZ, SZ]),
    "lvs_band_cells": (SZ, [SZ, SZ, SZ]),
    "lvs_edit_distance_band_workspace_bytes": (SZ, [SZ, SZ, I32, SZ]),
    "lvs_edit_distance_band": (I32, [VP, VP, SZ, VP, SZ, I32, SZ, VP, VP, SZ]),
    "lvs_edit_distance_clear_band_workspace_bytes": (SZ, [SZ, SZ, SZ]),
    "lvs_edit_distance_clear_band": (I32, [VP, VP, SZ, VP, SZ, VP, SZ, SZ, VP, VP, SZ]),
    "lvs_plan_workspace_bytes": (I32, [VP, SZ, I32, ctypes.POINTER(SZ)]),
    "lvs_plan_create": (I32, [VP, VP, SZ, I32, I32, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_plan_verify_wide": (I32, [VP, SZ, ctypes.c_uint, SZ, SZ, ctypes.POINTER(SZ), ctypes.POINTER(SZ),
                                   ctypes.POINTER(SZ), ctypes.POINTER(SZ)]),
    "lvs_plan_verify": (I32, [VP, SZ, I32, SZ, I32, SZ, ctypes.POINTER(SZ), ctypes.POINTER(SZ),
                              ctypes.POINTER(SZ), ctypes.POINTER(SZ)]),
    "lvs_context_set_refresh": (I32, [VP, SZ]),
    "lvs_wide_chunks": (SZ, [ctypes.c_uint]),
    "lvs_wide_pbs_per_pair": (SZ, [ctypes.c_uint]),
    "lvs_encrypt_symbols": (I32, [VP, VP, SZ, ctypes.c_uint, U64, VP]),
    "lvs_equality_wide_workspace_bytes": (SZ, [SZ, SZ, ctypes.c_uint]),
    "lvs_equality_wide": (I32, [VP, VP, SZ, VP, SZ, ctypes.c_uint, VP, VP, SZ]),
    "lvs_edit_distance_wide_workspace_bytes": (SZ, [SZ, SZ, ctypes.c_uint]),
    "lvs_edit_distance_wide": (I32, [VP, VP, SZ, VP, SZ, ctypes.c_uint, VP, VP, SZ]),
    "lvs_preprocess_wide_workspace_bytes": (SZ, [SZ, SZ, ctypes.c_uint]),
    "lvs_preprocess_wide": (I32, [VP, VP, SZ, ctypes.c_uint, VP, SZ, VP, VP, SZ]),
    "lvs_edit_distance_clear_wide": (I32, [VP, VP, SZ, VP, SZ, VP, SZ, VP, VP, SZ]),
    "lvs_plan_wide_workspace_bytes": (I32, [VP, SZ, ctypes.c_uint, ctypes.POINTER(SZ)]),
    "lvs_plan_create_wide": (I32, [VP, VP, SZ, ctypes.c_uint, I32, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_context_get_refresh": (I32, [VP, ctypes.POINTER(SZ)]),
    "lvs_plan_run": (I32, [VP]),
    "lvs_plan_info": (I32, [VP, ctypes.POINTER(SZ), ctypes.POINTER(SZ), ctypes.POINTER(SZ)]),
    "lvs_plan_run_steps": (I32, [VP, SZ, SZ]),
    "lvs_plan_step_bootstraps": (I32, [VP, VP, SZ]),
    "lvs_server_fixed_bytes": (SZ, [SZ]),
    "lvs_server_request_bytes": (SZ, [VP, VP, SZ, SZ, SZ]),
    "lvs_server_create": (I32, [VP, VP, VP, SZ, VP, SZ, SZ, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_server_create_wide": (I32, [VP, VP, VP, SZ, VP, SZ, ctypes.c_uint, SZ, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_server_request_bytes_wide": (SZ, [VP, SZ, SZ, SZ, ctypes.c_uint]),
    "lvs_server_submit": (I32, [VP, VP, SZ, ctypes.POINTER(U64)]),
    "lvs_server_step": (I32, [VP, ctypes.POINTER(SZ), ctypes.POINTER(SZ), ctypes.POINTER(SZ)]),
    "lvs_server_poll": (I32, [VP, U64, VP, ctypes.POINTER(ctypes.c_int)]),
    "lvs_server_stats": (I32, [VP, ctypes.POINTER(U64), ctypes.POINTER(U64)]),
    "lvs_engine_fixed_bytes": (SZ, [SZ]),
    "lvs_engine_query_bytes": (I32, [VP, I32, ctypes.POINTER(SZ)]),
    "lvs_engine_create": (I32, [VP, I32, SZ, VP, SZ, ctypes.POINTER(VP)]),
    "lvs_submit": (I32, [VP, VP, SZ, VP]),
    "lvs_poll": (I32, [VP, U64, I32, ctypes.POINTER(ctypes.c_int)]),
    "lvs_engine_stats": (I32, [VP, ctypes.POINTER(U64), ctypes.POINTER(U64), ctypes.POINTER(SZ),
                               ctypes.POINTER(SZ)]),
    "lvs_context_get_tuning": (I32, [VP, VP]),
    "lvs_context_set_tuning": (I32, [VP, VP]),
    "lvs_autotune_workspace_bytes": (SZ, [SZ]),
    "lvs_autotune": (I32, [VP, SZ, VP, SZ, VP, VP, SZ, ctypes.POINTER(SZ)]),
    "lvs_microbench_workspace_bytes": (SZ, [VP]),
    "lvs_microbench_modmul": (I32, [VP, I32, VP, SZ, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    "lvs_microbench_copy": (I32, [VP, VP, VP, SZ, I32, ctypes.POINTER(ctypes.c_double)]),
    "lvs_profile_enable": (I32, [VP, I32]),
    "lvs_profile_read": (I32, [VP, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U64), ctypes.POINTER(U64)]),
    "lvs_free": (None, [VP]),
}


def lib():
    """The loaded liblvs.so; raises if it has not been built."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"liblvs.so not built ({LIB_PATH}); run paper_2508_14568_amd.build.build()")
        # PyTorch first: its HIP runtime (same soname) then serves the library
        # too, so both share one runtime, one device list and one allocator.
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _L = L
    return _L


def exported_symbols():
    return sorted(_SIGS)


def _check(rc):
    if rc != 0:
        raise LvsError(rc, lib().lvs_last_error().decode())


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ handles

class _Handle:
    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and _L is not None:
            _L.lvs_free(self.ptr)
            self.ptr = None

    @property
    def _as_parameter_(self):
        return self.ptr


# ------------------------------------------------------------- host side

def lvs_params_default() -> lvs_params:
    p = lvs_params()
    _check(lib().lvs_params_default(ctypes.byref(p)))
    return p


def lvs_keygen(params: lvs_params, seed: int):
    ck, sk = VP(), VP()
    _check(lib().lvs_keygen(ctypes.byref(params), seed, ctypes.byref(ck), ctypes.byref(sk)))
    return _Handle(ck), _Handle(sk)


def lvs_lwe_encrypt(ck, mu: int, seed: int, index: int) -> np.ndarray:
    out = np.zeros(CT_WORDS, dtype=np.uint64)
    _check(lib().lvs_lwe_encrypt(ck, mu, seed, index, _np_ptr(out)))
    return out


def lvs_lwe_decrypt(ck, ct: np.ndarray):
    ct = np.ascontiguousarray(ct, dtype=np.uint64)
    mu, err = U32(), ctypes.c_int64()
    _check(lib().lvs_lwe_decrypt(ck, _np_ptr(ct), ctypes.byref(mu), ctypes.byref(err)))
    return int(mu.value), int(err.value)


def nsym(encoding: int) -> int:
    return 2 if encoding == LVS_ENC_ASCII7 else 1


def lvs_encrypt_string(ck, s: bytes, encoding: int, seed: int) -> np.ndarray:
    s = bytes(s)
    out = np.zeros((len(s), nsym(encoding), CT_WORDS), dtype=np.uint64)
    buf = (ctypes.c_uint8 * max(1, len(s))).from_buffer_copy(s or b"\0")
    _check(lib().lvs_encrypt_string(ck, buf, len(s), encoding, seed, _np_ptr(out)))
    return out


def lvs_decrypt_distance(ck, h_last: np.ndarray, m: int) -> int:
    h_last = np.ascontiguousarray(h_last, dtype=np.uint64).reshape(-1, CT_WORDS)
    out = ctypes.c_int64()
    _check(lib().lvs_decrypt_distance(ck, _np_ptr(h_last), m, h_last.shape[0], ctypes.byref(out)))
    return int(out.value)


def lvs_key_export(ck, sk, kind: int) -> np.ndarray:
    n = SZ()
    _check(lib().lvs_key_export(ck, sk, kind, None, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.uint8)
    _check(lib().lvs_key_export(ck, sk, kind, _np_ptr(out), ctypes.byref(n)))
    return out if kind < 2 else out.view(np.uint64)


# ------------------------------------------------------------ wire format

LVS_WIRE_CLIENT_KEY, LVS_WIRE_SERVER_KEY, LVS_WIRE_CIPHERTEXTS = 1, 2, 3


def lvs_export(kind: int, obj) -> bytes:
    """Record of a key handle (LVS_WIRE_CLIENT_KEY / _SERVER_KEY) or of host
    ciphertexts (LVS_WIRE_CIPHERTEXTS: an array of [..][N+1] words)."""
    count, arr = 0, None
    if kind == LVS_WIRE_CIPHERTEXTS:
        arr = np.ascontiguousarray(obj, dtype=np.uint64).reshape(-1, CT_WORDS)
        count, ptr = arr.shape[0], _np_ptr(arr)
    else:
        ptr = obj
    n = SZ()
    _check(lib().lvs_export(kind, ptr, count, None, ctypes.byref(n)))
    buf = (ctypes.c_uint8 * n.value)()
    _check(lib().lvs_export(kind, ptr, count, buf, ctypes.byref(n)))
    return bytes(buf)


def lvs_import_key(record: bytes):
    """(kind, key handle) from a key record."""
    buf = (ctypes.c_uint8 * max(1, len(record))).from_buffer_copy(record or b"\0")
    kind, out = ctypes.c_int(), VP()
    _check(lib().lvs_import_key(buf, len(record), ctypes.byref(kind), ctypes.byref(out)))
    return kind.value, _Handle(out)


def lvs_import_ciphertexts(record: bytes) -> np.ndarray:
    """[count][N+1] words from a ciphertext record."""
    buf = (ctypes.c_uint8 * max(1, len(record))).from_buffer_copy(record or b"\0")
    n = SZ()
    _check(lib().lvs_import_ciphertexts(buf, len(record), None, ctypes.byref(n)))
    out = np.zeros((n.value, CT_WORDS), dtype=np.uint64)
    _check(lib().lvs_import_ciphertexts(buf, len(record), _np_ptr(out) if n.value else None, ctypes.byref(n)))
    return out


# ------------------------------------------------------------ device side

def _torch():
    import torch
    return torch


def device_buffer(nbytes: int, device):
    """Raw device memory from torch's allocator (256-byte aligned)."""
    torch = _torch()
    return torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.int64, device=device)


def to_device(arr: np.ndarray, device):
    torch = _torch()
    a = np.ascontiguousarray(arr, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


class Context(_Handle):
    """A device context; keeps its torch arena alive."""

    def __init__(self, ptr, arena, device, stream_handle=0):
        super().__init__(ptr)
        self.arena = arena
        self.device = device
        self.stream_handle = stream_handle      # the HIP stream the context enqueues on


def lvs_context_bytes(params: lvs_params) -> int:
    n = SZ()
    _check(lib().lvs_context_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def lvs_context_create(sk, params: lvs_params, device=0, stream=None) -> Context:
    torch = _torch()
    dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
    nbytes = lvs_context_bytes(params)
    arena = device_buffer(nbytes, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    out = VP()
    _check(lib().lvs_context_create(sk, dev.index or 0, VP(st.cuda_stream), _dptr(arena), nbytes, ctypes.byref(out)))
    return Context(out, arena, dev, st.cuda_stream)


def lvs_context_set_stream(ctx: Context, stream):
    _check(lib().lvs_context_set_stream(ctx, VP(stream.cuda_stream)))
    ctx.stream_handle = stream.cuda_stream


def lvs_context_set_lut(ctx: Context, slot: int, f16):
    arr = (ctypes.c_int32 * 16)(*[int(v) for v in f16])
    _check(lib().lvs_context_set_lut(ctx, slot, arr))


def lvs_context_set_refresh(ctx: Context, every: int):
    """Noise-refresh interval in anti-diagonals (0: off)."""
    _check(lib().lvs_context_set_refresh(ctx, every))


def lvs_context_get_refresh(ctx: Context) -> int:
    out = SZ()
    _check(lib().lvs_context_get_refresh(ctx, ctypes.byref(out)))
    return out.value


def lvs_sync(ctx: Context):
    _check(lib().lvs_sync(ctx))


def lvs_pbs_workspace_bytes(B: int) -> int:
    return lib().lvs_pbs_workspace_bytes(B)


def lvs_pbs_batch(ctx: Context, d_in, B: int, d_out, lut_id: int = 0, lut_ids=None, d_work=None):
    """lut_ids: optional host sequence of per-ciphertext table slots."""
    need = lvs_pbs_workspace_bytes(B)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ids = None
    if lut_ids is not None:
        ids = np.ascontiguousarray(np.asarray(lut_ids, dtype=np.uint8))
        assert ids.size == B
    _check(lib().lvs_pbs_batch(ctx, _dptr(d_in), None if ids is None else _np_ptr(ids), lut_id, B, _dptr(d_out),
                               _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


LVS_PBS_STATIC_MAX = 1024


def lvs_pbs_batch_static(ctx: Context, d_in, B: int, d_out, lut_id: int = 0, lut_ids=None):
    """lvs_pbs_batch without a workspace (the library's device array); B at
    most LVS_PBS_STATIC_MAX.  lut_ids: optional host sequence of slots."""
    ids = None
    if lut_ids is not None:
        ids = np.ascontiguousarray(np.asarray(lut_ids, dtype=np.uint8))
        assert ids.size == B
    _check(lib().lvs_pbs_batch_static(ctx, _dptr(d_in), None if ids is None else _np_ptr(ids), lut_id, B,
                                      _dptr(d_out)))


def lvs_equality_workspace_bytes(m: int, n: int, encoding: int) -> int:
    return lib().lvs_equality_workspace_bytes(m, n, encoding)


def lvs_equality(ctx: Context, d_a, m: int, d_b, n: int, encoding: int, d_eq9, d_work=None):
    need = lvs_equality_workspace_bytes(m, n, encoding)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    _check(lib().lvs_equality(ctx, _dptr(d_a), m, _dptr(d_b), n, encoding, _dptr(d_eq9), _dptr(d_work),
                              d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_eq9_workspace_bytes(m: int, n: int) -> int:
    return lib().lvs_edit_distance_eq9_workspace_bytes(m, n)


def lvs_edit_distance_eq9(ctx: Context, d_eq9, m: int, n: int, d_h_last, d_trace=None, d_work=None):
    need = lvs_edit_distance_eq9_workspace_bytes(m, n)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    _check(lib().lvs_edit_distance_eq9(ctx, _dptr(d_eq9), m, n, _dptr(d_h_last), _dptr(d_trace), _dptr(d_work),
                                       d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_workspace_bytes(m: int, n: int, encoding: int) -> int:
    return lib().lvs_edit_distance_workspace_bytes(m, n, encoding)


def lvs_edit_distance(ctx: Context, d_a, m: int, d_b, n: int, encoding: int, d_h_last, d_work=None):
    need = lvs_edit_distance_workspace_bytes(m, n, encoding)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    _check(lib().lvs_edit_distance(ctx, _dptr(d_a), m, _dptr(d_b), n, encoding, _dptr(d_h_last), _dptr(d_work),
                                   d_work.numel() * d_work.element_size()))
    return d_work


def lvs_preprocess_workspace_bytes(m: int, alen: int, encoding: int) -> int:
    return lib().lvs_preprocess_workspace_bytes(m, alen, encoding)


def lvs_preprocess(ctx: Context, d_a, m: int, encoding: int, alphabet: bytes, d_table, d_work=None):
    need = lvs_preprocess_workspace_bytes(m, len(alphabet), encoding)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ab = (ctypes.c_uint8 * max(1, len(alphabet))).from_buffer_copy(bytes(alphabet) or b"\0")
    _check(lib().lvs_preprocess(ctx, _dptr(d_a), m, encoding, ab, len(alphabet), _dptr(d_table), _dptr(d_work),
                                d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_clear_workspace_bytes(m: int, n: int) -> int:
    return lib().lvs_edit_distance_clear_workspace_bytes(m, n)


def lvs_edit_distance_clear(ctx: Context, d_table, m: int, alphabet: bytes, b: bytes, d_h_last, d_work=None):
    need = lvs_edit_distance_clear_workspace_bytes(m, len(b))
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ab = (ctypes.c_uint8 * max(1, len(alphabet))).from_buffer_copy(bytes(alphabet) or b"\0")
    bb = (ctypes.c_uint8 * max(1, len(b))).from_buffer_copy(bytes(b) or b"\0")
    _check(lib().lvs_edit_distance_clear(ctx, _dptr(d_table), m, ab, len(alphabet), bb, len(b), _dptr(d_h_last),
                                         _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


# ----------------------------------------------------------- wide symbols

def lvs_wide_chunks(width: int) -> int:
    return lib().lvs_wide_chunks(width)


def lvs_wide_pbs_per_pair(width: int) -> int:
    return lib().lvs_wide_pbs_per_pair(width)


def _u64_array(values):
    arr = np.ascontiguousarray(np.asarray([int(v) for v in values] or [0], dtype=np.uint64))
    return arr


def lvs_encrypt_symbols(ck, syms, width: int, seed: int) -> np.ndarray:
    """(len, c, N+1) ciphertexts of the 4-bit chunks of each symbol."""
    c = lvs_wide_chunks(width)
    if c == 0:
        raise LvsError(-1, "width must be 1..64")
    arr = _u64_array(syms)
    out = np.zeros((len(syms), c, CT_WORDS), dtype=np.uint64)
    _check(lib().lvs_encrypt_symbols(ck, _np_ptr(arr), len(syms), width, seed, _np_ptr(out)))
    return out


def lvs_equality_wide_workspace_bytes(m: int, n: int, width: int) -> int:
    return lib().lvs_equality_wide_workspace_bytes(m, n, width)


def lvs_equality_wide(ctx: Context, d_a, m: int, d_b, n: int, width: int, d_eq9, d_work=None):
    need = lvs_equality_wide_workspace_bytes(m, n, width)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    _check(lib().lvs_equality_wide(ctx, _dptr(d_a), m, _dptr(d_b), n, width, _dptr(d_eq9), _dptr(d_work),
                                   d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_wide_workspace_bytes(m: int, n: int, width: int) -> int:
    return lib().lvs_edit_distance_wide_workspace_bytes(m, n, width)


def lvs_edit_distance_wide(ctx: Context, d_a, m: int, d_b, n: int, width: int, d_h_last, d_work=None):
    need = lvs_edit_distance_wide_workspace_bytes(m, n, width)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    _check(lib().lvs_edit_distance_wide(ctx, _dptr(d_a), m, _dptr(d_b), n, width, _dptr(d_h_last), _dptr(d_work),
                                        d_work.numel() * d_work.element_size()))
    return d_work


def lvs_preprocess_wide_workspace_bytes(m: int, alen: int, width: int) -> int:
    return lib().lvs_preprocess_wide_workspace_bytes(m, alen, width)


def lvs_preprocess_wide(ctx: Context, d_a, m: int, width: int, alphabet, d_table, d_work=None):
    need = lvs_preprocess_wide_workspace_bytes(m, len(alphabet), width)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ab = _u64_array(alphabet)
    _check(lib().lvs_preprocess_wide(ctx, _dptr(d_a), m, width, _np_ptr(ab), len(alphabet), _dptr(d_table),
                                     _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_clear_wide(ctx: Context, d_table, m: int, alphabet, b, d_h_last, d_work=None):
    need = lvs_edit_distance_clear_workspace_bytes(m, len(b))
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ab, bb = _u64_array(alphabet), _u64_array(b)
    _check(lib().lvs_edit_distance_clear_wide(ctx, _dptr(d_table), m, _np_ptr(ab), len(alphabet), _np_ptr(bb), len(b),
                                              _dptr(d_h_last), _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


# ------------------------------------------------------------- band modes

def lvs_band_exact(m: int, n: int) -> int:
    return lib().lvs_band_exact(m, n)


def lvs_band_cells(m: int, n: int, ell: int) -> int:
    return lib().lvs_band_cells(m, n, ell)


def lvs_edit_distance_band_workspace_bytes(m: int, n: int, encoding: int, ell: int) -> int:
    return lib().lvs_edit_distance_band_workspace_bytes(m, n, encoding, ell)


def lvs_edit_distance_band(ctx: Context, d_a, m: int, d_b, n: int, encoding: int, ell: int, d_path, d_work=None):
    """d_path: [m+n][N+1] device buffer for the band path."""
    if d_work is None:
        d_work = device_buffer(lvs_edit_distance_band_workspace_bytes(m, n, encoding, ell), ctx.device)
    _check(lib().lvs_edit_distance_band(ctx, _dptr(d_a), m, _dptr(d_b), n, encoding, ell, _dptr(d_path),
                                        _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


def lvs_edit_distance_clear_band_workspace_bytes(m: int, n: int, ell: int) -> int:
    return lib().lvs_edit_distance_clear_band_workspace_bytes(m, n, ell)


def lvs_edit_distance_clear_band(ctx: Context, d_table, m: int, alphabet: bytes, b: bytes, ell: int, d_path,
                                 d_work=None):
    need = lvs_edit_distance_clear_band_workspace_bytes(m, len(b), ell)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    ab = (ctypes.c_uint8 * max(1, len(alphabet))).from_buffer_copy(bytes(alphabet) or b"\0")
    bb = (ctypes.c_uint8 * max(1, len(b))).from_buffer_copy(bytes(b) or b"\0")
    _check(lib().lvs_edit_distance_clear_band(ctx, _dptr(d_table), m, ab, len(alphabet), bb, len(b), ell,
                                              _dptr(d_path), _dptr(d_work), d_work.numel() * d_work.element_size()))
    return d_work


# ------------------------------------------------------------ batch plans

LVS_PLAN_GRAPH = 1


class lvs_query(ctypes.Structure):
    _fields_ = [("d_a", VP), ("m", SZ), ("d_b", VP), ("n", SZ), ("d_table", VP), ("alphabet", VP), ("alen", SZ),
                ("b_clear", VP), ("d_h_last", VP), ("banded", ctypes.c_int32), ("ell", SZ), ("d_path", VP),
                ("d_trace", VP), ("d_eq1", VP), ("d_eq9", VP)]


class Plan(_Handle):
    """A batch plan; keeps the query structs, host strings and workspace alive."""

    def __init__(self, ptr, keep):
        super().__init__(ptr)
        self._keep = keep


def make_queries(items):
    """items: dicts with d_a, m, d_h_last and either d_b, n or d_table,
    alphabet (bytes), b_clear (bytes); optionally ell and d_path (band) and
    the checking outputs d_trace, d_eq1, d_eq9 ([m][n][N+1] device buffers)."""
    arr = (lvs_query * max(1, len(items)))()
    keep = []
    for k, it in enumerate(items):
        q = arr[k]
        q.d_a = _dptr(it.get("d_a"))
        q.m = it["m"]
        q.d_h_last = _dptr(it.get("d_h_last"))
        q.d_trace = _dptr(it.get("d_trace"))
        q.d_eq1 = _dptr(it.get("d_eq1"))
        q.d_eq9 = _dptr(it.get("d_eq9"))
        if it.get("ell") is not None:
            q.banded = 1
            q.ell = it["ell"]
            q.d_path = _dptr(it.get("d_path"))
        if it.get("d_b") is not None:
            q.d_b = _dptr(it["d_b"])
            q.n = it["n"]
        else:
            ab = (ctypes.c_uint8 * max(1, len(it["alphabet"]))).from_buffer_copy(bytes(it["alphabet"]) or b"\0")
            bc = (ctypes.c_uint8 * max(1, len(it["b_clear"]))).from_buffer_copy(bytes(it["b_clear"]) or b"\0")
            keep += [ab, bc]
            q.d_table = _dptr(it.get("d_table"))
            q.alphabet = ctypes.cast(ab, VP)
            q.alen = len(it["alphabet"])
            q.b_clear = ctypes.cast(bc, VP)
            q.n = len(it["b_clear"])
    return arr, keep


def lvs_plan_workspace_bytes(items, encoding: int) -> int:
    arr, keep = make_queries(items)
    n = SZ()
    _check(lib().lvs_plan_workspace_bytes(arr, len(items), encoding, ctypes.byref(n)))
    return n.value


def lvs_plan_create(ctx: Context, items, encoding: int, graph: bool = False, d_work=None) -> Plan:
    arr, keep = make_queries(items)
    need = lvs_plan_workspace_bytes(items, encoding)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    out = VP()
    _check(lib().lvs_plan_create(ctx, arr, len(items), encoding, LVS_PLAN_GRAPH if graph else 0, _dptr(d_work),
                                 d_work.numel() * d_work.element_size(), ctypes.byref(out)))
    return Plan(out, (arr, keep, d_work, items))


def lvs_plan_wide_workspace_bytes(items, width: int) -> int:
    arr, keep = make_queries(items)
    n = SZ()
    _check(lib().lvs_plan_wide_workspace_bytes(arr, len(items), width, ctypes.byref(n)))
    return n.value


def lvs_plan_create_wide(ctx: Context, items, width: int, graph: bool = False, d_work=None) -> Plan:
    """Batch plan over wide symbols: items as for lvs_plan_create, both strings
    encrypted by lvs_encrypt_symbols with this width."""
    arr, keep = make_queries(items)
    need = lvs_plan_wide_workspace_bytes(items, width)
    if d_work is None:
        d_work = device_buffer(need, ctx.device)
    out = VP()
    _check(lib().lvs_plan_create_wide(ctx, arr, len(items), width, LVS_PLAN_GRAPH if graph else 0, _dptr(d_work),
                                      d_work.numel() * d_work.element_size(), ctypes.byref(out)))
    return Plan(out, (arr, keep, d_work, items))


def lvs_plan_verify(queries, encoding: int, round_: int, fill: bool = True, refresh: int = 0):
    """queries: (m, n, kind, ell) tuples with kind 'enc' (both encrypted) or
    'clear' (cleartext b over alphabet bytes(range(n)) of n distinct symbols);
    ell None for the full matrix.  Buffers get placeholder addresses.
    refresh: the noise-refresh interval (0: off).
    Returns (steps, bootstraps, rounds, violations)."""
    arr = (lvs_query * max(1, len(queries)))()
    keep = []
    addr = 1 << 32
    for k, (m, n, kind, ell) in enumerate(queries):
        q = arr[k]
        q.m, q.n = m, n
        q.d_a = addr
        addr += (m + 1) * 2 * CT_WORDS * 8
        if kind == "enc":
            q.d_b = addr
            addr += (n + 1) * 2 * CT_WORDS * 8
        else:
            ab = (ctypes.c_uint8 * max(1, n)).from_buffer_copy(bytes(range(n)) or b"\0")
            keep.append(ab)
            q.d_table = addr
            addr += (n + 1) * (m + 1) * CT_WORDS * 8
            q.alphabet = ctypes.cast(ab, VP)
            q.alen = n
            q.b_clear = ctypes.cast(ab, VP)
        if ell is None:
            q.d_h_last = addr
            addr += (n + 1) * CT_WORDS * 8
        else:
            q.banded, q.ell, q.d_path = 1, ell, addr
            addr += (m + n + 1) * CT_WORDS * 8
    st, jb, rd, bad = SZ(), SZ(), SZ(), SZ()
    _check(lib().lvs_plan_verify(arr, len(queries), encoding, round_, 1 if fill else 0, refresh, ctypes.byref(st),
                                 ctypes.byref(jb), ctypes.byref(rd), ctypes.byref(bad)))
    return st.value, jb.value, rd.value, bad.value



def lvs_plan_verify_wide(queries, width: int, round_: int, refresh: int = 0):
    """queries: (m, n, ell) tuples of wide-symbol queries (both strings
    encrypted), ell None for the full matrix.  Buffers get placeholder
    addresses.  Returns (steps, bootstraps, rounds, violations)."""
    c = lvs_wide_chunks(width)
    arr = (lvs_query * max(1, len(queries)))()
    addr = 1 << 32
    for k, (m, n, ell) in enumerate(queries):
        q = arr[k]
        q.m, q.n = m, n
        q.d_a = addr
        addr += (m + 1) * max(c, 1) * CT_WORDS * 8
        q.d_b = addr
        addr += (n + 1) * max(c, 1) * CT_WORDS * 8
        if ell is None:
            q.d_h_last = addr
            addr += (n + 1) * CT_WORDS * 8
        else:
            q.banded, q.ell, q.d_path = 1, ell, addr
            addr += (m + n + 1) * CT_WORDS * 8
    st, jb, rd, bad = SZ(), SZ(), SZ(), SZ()
    _check(lib().lvs_plan_verify_wide(arr, len(queries), width, round_, refresh, ctypes.byref(st), ctypes.byref(jb),
                                      ctypes.byref(rd), ctypes.byref(bad)))
    return st.value, jb.value, rd.value, bad.value

def lvs_plan_run(plan: Plan):
    _check(lib().lvs_plan_run(plan))


def lvs_plan_run_steps(plan: Plan, first: int, count: int):
    _check(lib().lvs_plan_run_steps(plan, first, count))


def lvs_plan_step_bootstraps(plan: Plan):
    steps = lvs_plan_info(plan)[0]
    out = (SZ * max(1, steps))()
    _check(lib().lvs_plan_step_bootstraps(plan, out, steps))
    return [int(out[k]) for k in range(steps)]


def lvs_plan_info(plan: Plan):
    st, pb, mx = SZ(), SZ(), SZ()
    _check(lib().lvs_plan_info(plan, ctypes.byref(st), ctypes.byref(pb), ctypes.byref(mx)))
    return st.value, pb.value, mx.value


# --------------------------------------------------------------- serving

class Server(_Handle):
    """A serving engine; keeps its arena and name table alive."""

    def __init__(self, ptr, keep, total_len):
        super().__init__(ptr)
        self._keep = keep
        self.total_len = total_len


def _names_buf(names):
    cat = b"".join(bytes(x) for x in names)
    buf = (ctypes.c_uint8 * max(1, len(cat))).from_buffer_copy(cat or b"\0")
    lens = (SZ * max(1, len(names)))(*[len(x) for x in names])
    return buf, lens


def lvs_server_fixed_bytes(max_step: int) -> int:
    return lib().lvs_server_fixed_bytes(max_step)


def lvs_server_request_bytes(names, alen: int, m: int) -> int:
    buf, lens = _names_buf(names)
    return lib().lvs_server_request_bytes(buf, lens, len(names), alen, m)


def lvs_server_create(ctx: Context, names, alphabet: bytes, arena_bytes: int, max_step: int = 65536) -> Server:
    buf, lens = _names_buf(names)
    ab = (ctypes.c_uint8 * len(alphabet)).from_buffer_copy(bytes(alphabet))
    arena = device_buffer(arena_bytes, ctx.device)
    out = VP()
    _check(lib().lvs_server_create(ctx, buf, lens, len(names), ab, len(alphabet), max_step, _dptr(arena),
                                   arena.numel() * arena.element_size(), ctypes.byref(out)))
    return Server(out, (buf, lens, ab, arena, ctx), sum(len(x) for x in names))


def _wide_names_buf(names):
    cat = [int(v) for x in names for v in x]
    buf = _u64_array(cat or [0])
    lens = (SZ * max(1, len(names)))(*[len(x) for x in names])
    return buf, lens


def lvs_server_request_bytes_wide(names, alen: int, m: int, width: int) -> int:
    _, lens = _wide_names_buf(names)
    return lib().lvs_server_request_bytes_wide(lens, len(names), alen, m, width)


def lvs_server_create_wide(ctx: Context, names, alphabet, width: int, arena_bytes: int,
                           max_step: int = 65536) -> Server:
    """names: sequences of symbols below 2^width; alphabet: their symbols."""
    buf, lens = _wide_names_buf(names)
    ab = _u64_array(list(alphabet))
    arena = device_buffer(arena_bytes, ctx.device)
    out = VP()
    _check(lib().lvs_server_create_wide(ctx, _np_ptr(buf), lens, len(names), _np_ptr(ab), len(alphabet), width,
                                        max_step, _dptr(arena), arena.numel() * arena.element_size(),
                                        ctypes.byref(out)))
    return Server(out, (buf, lens, ab, arena, ctx), sum(len(x) for x in names))


def lvs_server_submit(srv: Server, query_ct: np.ndarray) -> int:
    q = np.ascontiguousarray(query_ct, dtype=np.uint64)
    m = q.shape[0]
    t = U64()
    _check(lib().lvs_server_submit(srv, _np_ptr(q), m, ctypes.byref(t)))
    return t.value


def lvs_server_step(srv: Server):
    """(running requests, queued requests, bootstraps of the step)."""
    a, q, j = SZ(), SZ(), SZ()
    _check(lib().lvs_server_step(srv, ctypes.byref(a), ctypes.byref(q), ctypes.byref(j)))
    return a.value, q.value, j.value


def lvs_server_poll(srv: Server, ticket: int):
    """None while running, else the [sum n_k][N+1] result rows."""
    done = ctypes.c_int()
    _check(lib().lvs_server_poll(srv, ticket, None, ctypes.byref(done)))
    if not done.value:
        return None
    out = np.zeros((srv.total_len, CT_WORDS), dtype=np.uint64)
    _check(lib().lvs_server_poll(srv, ticket, _np_ptr(out), ctypes.byref(done)))
    return out


def lvs_server_stats(srv: Server):
    st, pb = U64(), U64()
    _check(lib().lvs_server_stats(srv, ctypes.byref(st), ctypes.byref(pb)))
    return st.value, pb.value


# ------------------------------------------------- continuous batching

class Engine(_Handle):
    """A continuous-batching engine over lvs_query items; keeps its arena and
    the submitted queries' buffers alive until their tickets are polled done."""

    def __init__(self, ptr, keep):
        super().__init__(ptr)
        self._keep = keep
        self._inflight = {}


def lvs_engine_fixed_bytes(max_step: int) -> int:
    return lib().lvs_engine_fixed_bytes(max_step)


def lvs_engine_query_bytes(item, encoding: int) -> int:
    arr, keep = make_queries([item])
    n = SZ()
    _check(lib().lvs_engine_query_bytes(arr, encoding, ctypes.byref(n)))
    return n.value


def lvs_engine_create(ctx: Context, encoding: int, arena_bytes: int, max_step: int = 4096) -> Engine:
    arena = device_buffer(arena_bytes, ctx.device)
    out = VP()
    _check(lib().lvs_engine_create(ctx, encoding, max_step, _dptr(arena), arena.numel() * arena.element_size(),
                                   ctypes.byref(out)))
    return Engine(out, (arena, ctx))


def lvs_submit(eng: Engine, items):
    """Queues query dicts (as for lvs_plan_create); returns their tickets.
    The caller's current stream is synchronised first: the engine runs on a
    stream of its own and reads the queries' device buffers as they are."""
    _torch().cuda.current_stream().synchronize()
    arr, keep = make_queries(items)
    tickets = (U64 * max(1, len(items)))()
    _check(lib().lvs_submit(eng, arr, len(items), tickets))
    out = [int(tickets[k]) for k in range(len(items))]
    for t, it in zip(out, items):
        eng._inflight[t] = it
    return out


def lvs_poll(eng: Engine, ticket: int, wait: bool = False) -> bool:
    """True once the query's results are complete in its d_h_last (d_path)."""
    done = ctypes.c_int()
    _check(lib().lvs_poll(eng, ticket, 1 if wait else 0, ctypes.byref(done)))
    if done.value:
        eng._inflight.pop(ticket, None)
    return bool(done.value)


def lvs_engine_stats(eng: Engine):
    """(steps, bootstraps, running queries, queued queries)."""
    st, pb, a, q = U64(), U64(), SZ(), SZ()
    _check(lib().lvs_engine_stats(eng, ctypes.byref(st), ctypes.byref(pb), ctypes.byref(a), ctypes.byref(q)))
    return st.value, pb.value, a.value, q.value


# ------------------------------------------------------------------ tuning

class lvs_tuning(ctypes.Structure):
    _fields_ = [("br_grid", ctypes.c_int32), ("latency_form_max", ctypes.c_int32), ("latency_waves", ctypes.c_int32),
                ("throughput_waves", ctypes.c_int32), ("ks_tile", ctypes.c_int32)]


class lvs_tune_sample(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("form", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("ms", ctypes.c_double)]


def lvs_context_get_tuning(ctx: Context) -> dict:
    t = lvs_tuning()
    _check(lib().lvs_context_get_tuning(ctx, ctypes.byref(t)))
    return {"br_grid": t.br_grid, "latency_form_max": t.latency_form_max, "latency_waves": t.latency_waves,
            "throughput_waves": t.throughput_waves, "ks_tile": t.ks_tile}


def lvs_context_set_tuning(ctx: Context, tuning: dict):
    t = lvs_tuning(int(tuning["br_grid"]), int(tuning["latency_form_max"]), int(tuning.get("latency_waves", 8)),
                   int(tuning.get("throughput_waves", 8)), int(tuning.get("ks_tile", 8)))
    _check(lib().lvs_context_set_tuning(ctx, ctypes.byref(t)))


def lvs_autotune_workspace_bytes(max_batch: int) -> int:
    return lib().lvs_autotune_workspace_bytes(max_batch)


def lvs_autotune(ctx: Context, max_batch: int, d_work=None):
    """(installed tuning, list of timings) from the library's autotuner."""
    if d_work is None:
        d_work = device_buffer(lvs_autotune_workspace_bytes(max_batch), ctx.device)
    best = lvs_tuning()
    samples = (lvs_tune_sample * 64)()
    n = SZ()
    _check(lib().lvs_autotune(ctx, max_batch, _dptr(d_work), d_work.numel() * d_work.element_size(),
                              ctypes.byref(best), samples, 64, ctypes.byref(n)))
    rows = [{"batch": x.batch, "form": x.form, "grid": x.grid, "ms": round(x.ms, 4)} for x in samples[:n.value]]
    return {"br_grid": best.br_grid, "latency_form_max": best.latency_form_max,
            "latency_waves": best.latency_waves, "throughput_waves": best.throughput_waves,
            "ks_tile": best.ks_tile}, rows


def _tuning_key(ctx: Context) -> str:
    import hashlib
    torch = _torch()
    prop = torch.cuda.get_device_properties(ctx.device)
    with open(LIB_PATH, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    return f"{getattr(prop, 'gcnArchName', prop.name)}/{prop.multi_processor_count}cu/{digest}"


def autotune(ctx: Context, max_batch: int = None, cache: str = None) -> dict:
    """Installs a launch shape for this device and library build: from the
    JSON cache when it holds one, else from lvs_autotune (then cached).
    cache: file path (default $LVS_TUNING_CACHE or ~/.cache/lvs/tuning.json)."""
    import json
    torch = _torch()
    if max_batch is None:
        max_batch = 4 * torch.cuda.get_device_properties(ctx.device).multi_processor_count
    path = cache or os.environ.get("LVS_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "lvs", "tuning.json")
    key = _tuning_key(ctx)
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    hit = table.get(key)
    if hit and hit.get("max_batch") == max_batch:
        lvs_context_set_tuning(ctx, hit["tuning"])
        return dict(hit, cached=True)
    tuning, rows = lvs_autotune(ctx, max_batch)
    entry = {"tuning": tuning, "max_batch": max_batch, "samples": rows}
    table[key] = entry
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(table, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass                      # an unwritable cache only costs a re-tune
    return dict(entry, cached=False)


# ------------------------------------------------------------ measurement

KERNEL_BLIND_ROTATE = 0              # every form
KERNEL_KEYSWITCH = 1
KERNEL_GRAPH = 2
KERNEL_BLIND_ROTATE_LATENCY = 3      # eight-wave form, one workgroup per CU
KERNEL_BLIND_ROTATE_THROUGHPUT = 4   # four-wave form, two workgroups per CU
KERNEL_BLIND_ROTATE_W16 = 5          # sixteen-wave form, one workgroup per CU
KERNEL_BLIND_ROTATE_PAIR = 6         # eight-wave form, two workgroups per CU


def lvs_microbench_modmul(ctx: Context, iters: int = 4096):
    """(ms, 32-bit multiplies) of the butterfly instruction-mix probe."""
    work = device_buffer(lib().lvs_microbench_workspace_bytes(ctx), ctx.device)
    ms, muls = ctypes.c_double(), ctypes.c_double()
    _check(lib().lvs_microbench_modmul(ctx, iters, _dptr(work), work.numel() * work.element_size(),
                                       ctypes.byref(ms), ctypes.byref(muls)))
    return ms.value, muls.value


def lvs_microbench_copy(ctx: Context, d_src, d_dst, nbytes: int, reps: int = 5) -> float:
    """Mean ms of one nbytes vector copy."""
    ms = ctypes.c_double()
    _check(lib().lvs_microbench_copy(ctx, _dptr(d_src), _dptr(d_dst), nbytes, reps, ctypes.byref(ms)))
    return ms.value


def lvs_profile_enable(ctx: Context, enable: bool):
    _check(lib().lvs_profile_enable(ctx, 1 if enable else 0))


def lvs_profile_read(ctx: Context, kernel: int):
    """(total milliseconds, launches, bootstraps) recorded for a kernel."""
    ms, n, u = ctypes.c_double(), U64(), U64()
    _check(lib().lvs_profile_read(ctx, kernel, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
    return ms.value, n.value, u.value
