"""ctypes declarations of librnsfhe.so (the C ABI of include/rnsfhe.h).

Importing this module loads the library and raises if it is missing: there is
no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RF_LIBRARY") or os.path.join(_PKG, "librnsfhe.so")

RF_OK, RF_EINVAL, RF_ELEVEL, RF_EWORKSPACE, RF_EHIP, RF_EUNSUPPORTED = 0, -1, -2, -4, -5, -6
RF_CKKS, RF_BFV, RF_BGV = 0, 1, 2
RF_OP_HMULT_RELIN, RF_OP_ROTATE, RF_OP_RESCALE, RF_OP_KEYSWITCH, RF_OP_MODSWITCH = 1, 2, 3, 4, 5
RF_OP_ENCODE, RF_OP_DECODE = 6, 7

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t


class rf_params(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32),
        ("log_n", _u32),
        ("log_nmax", _u32),
        ("n_q", _u32),
        ("q", _u64p),
        ("n_p", _u32),
        ("p", _u64p),
        ("alpha", _u32),
        ("t", ctypes.c_uint64),
        ("n_b", _u32),
        ("b", _u64p),
        ("m_sk", ctypes.c_uint64),
    ]


class rf_batch_item(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("a", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("rlk", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("n_limbs", _u32),
    ]


class rf_tuning(ctypes.Structure):
    _fields_ = [
        ("ntt_small_below", _u32),
        ("ntt_small_tile", _u32),
        ("ntt_small_radix", _u32),
        ("modup_chunk", _u32),
        ("ntt_fused_small_below", _u32),
    ]


# torch ships its own HIP runtime; it has to be in the process before the
# library is loaded, so that the library binds to that runtime.  Loaded the
# other way round, the library pulls in the system's runtime first, torch's
# HIP libraries bind to it, and torch then finds no GPU.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError("librnsfhe.so is not built (run __graft_entry__.build() or "
                      "python paper_2503_22227_amd/build.py): %s" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

_SIGS = {
    "rf_ctx_create": (ctypes.c_int, [ctypes.POINTER(rf_params), ctypes.c_int, ctypes.POINTER(_vp)]),
    "rf_ctx_destroy": (None, [_vp]),
    "rf_workspace_bytes": (_sz, [_vp, ctypes.c_int, _u32]),
    "rf_ctx_set_tuning": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(rf_tuning)]),
    "rf_ctx_get_tuning": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(rf_tuning)]),
    "rf_ntt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "rf_intt": (ctypes.c_int, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "rf_hmult_relin": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "rf_hmult_relin_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u32, _vp]),
    "rf_rotate": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _u32, _vp, _sz, _vp]),
    "rf_keyswitch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, ctypes.c_int, _vp, _sz, _vp]),
    "rf_rescale": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "rf_modswitch": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "rf_tensor": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "rf_automorphism": (ctypes.c_int, [_vp, _vp, _vp, _u32, _u32, _u32, _vp]),
    "rf_galois_element": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int, _u32p]),
    "rf_key_ntt": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "rf_keygen_switch": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp]),
    "rf_encrypt_sk": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp]),
    "rf_decrypt": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "rf_crt_centered": (ctypes.c_int, [_vp, _vp, _vp, _u32, ctypes.c_double, _vp]),
    "rf_encode_ckks": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _vp, _sz, _vp]),
    "rf_decode_ckks": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "rf_add": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _u32, _vp]),
    "rf_sub": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _u32, _vp]),
    "rf_mul_scalar": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _u32, _u32, _vp]),
    "rf_add_scalar": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _u32, _vp]),
    "rf_mul_plain": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32, _u32, _vp]),
    "rf_batch_workspace_bytes": (_sz, [ctypes.POINTER(rf_batch_item), _u32]),
    "rf_batch_create": (ctypes.c_int, [ctypes.POINTER(rf_batch_item), _u32, _vp, _sz, ctypes.POINTER(_vp)]),
    "rf_batch_destroy": (None, [_vp]),
    "rf_batch_set_grid": (ctypes.c_int, [_vp, _u32, _u32]),
    "rf_batch_set_modup_chunk": (ctypes.c_int, [_vp, _u32]),
    "rf_batch_stage_units": (ctypes.c_int, [_vp, _u32]),
    "rf_batch_hmult_relin": (ctypes.c_int, [_vp, _vp]),
    "rf_batch_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "rf_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "rf_profile_read": (ctypes.c_int, [ctypes.c_char_p, _sz]),
    "rf_last_error": (ctypes.c_char_p, []),
    "rf_version": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class RFError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.rf_last_error().decode(errors="replace")
        super().__init__("%s failed with code %d: %s" % (where, code, msg))
        self.code = code


def check(code: int, where: str) -> None:
    if code != RF_OK:
        raise RFError(code, where)


def profile_enable(on: bool) -> None:
    check(lib.rf_profile_enable(1 if on else 0), "rf_profile_enable")


def profile_read() -> dict:
    """{kernel: (launches, total_ms)} of the launches since the last read."""
    buf = ctypes.create_string_buffer(1 << 16)
    n = lib.rf_profile_read(buf, len(buf))
    if n < 0:
        check(n, "rf_profile_read")
    out = {}
    for line in buf.value.decode().splitlines():
        name, count, ms = line.split()
        out[name] = (int(count), float(ms))
    return out
