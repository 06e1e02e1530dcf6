"""ctypes loader for the oracle's plain C core (``core.c``); test infrastructure only.

The shared object is compiled with gcc next to the source when it is missing
(``build_core``); ``__graft_entry__.build()`` rebuilds it on every call.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "core.c")
_LIB = os.path.join(_HERE, "_oracle_core.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build_core() -> str:
    """Compile core.c into a shared object with gcc; returns its path."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_core()
        L = ctypes.CDLL(_LIB)
        u64 = ctypes.c_uint64
        L.orc_mulmod.restype = u64
        L.orc_mulmod.argtypes = [u64, u64, u64]
        L.orc_powmod.restype = u64
        L.orc_powmod.argtypes = [u64, u64, u64]
        for name in ("orc_ntt_fwd", "orc_ntt_inv"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [_u64p, ctypes.c_int, u64, u64]
        for name in ("orc_mul", "orc_add", "orc_sub"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [_u64p, _u64p, _u64p, u64, u64]
        L.orc_mul_scalar.restype = None
        L.orc_mul_scalar.argtypes = [_u64p, u64, _u64p, u64, u64]
        L.orc_bconv.restype = None
        L.orc_bconv.argtypes = [_u64p, ctypes.c_int, _u64p, _u64p, ctypes.c_int, _u64p, _u64p,
                                _u64p, u64, ctypes.c_int]
        L.orc_automorphism_coeff.restype = None
        L.orc_automorphism_coeff.argtypes = [_u64p, _u64p, ctypes.c_int, u64, u64]
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def ntt_fwd(a: np.ndarray, log_n: int, q: int, psi: int) -> np.ndarray:
    """Forward NTT of one limb (returns a new array)."""
    out = u64(a).copy()
    lib().orc_ntt_fwd(ptr(out), log_n, q, psi)
    return out


def ntt_inv(a: np.ndarray, log_n: int, q: int, psi: int) -> np.ndarray:
    out = u64(a).copy()
    lib().orc_ntt_inv(ptr(out), log_n, q, psi)
    return out


def _binary(name, a, b, q):
    a = u64(a)
    b = u64(b)
    out = np.empty_like(a)
    getattr(lib(), name)(ptr(a), ptr(b), ptr(out), a.size, q)
    return out


def mul(a, b, q):
    return _binary("orc_mul", a, b, q)


def add(a, b, q):
    return _binary("orc_add", a, b, q)


def sub(a, b, q):
    return _binary("orc_sub", a, b, q)


def mul_scalar(a, c: int, q: int):
    a = u64(a)
    out = np.empty_like(a)
    lib().orc_mul_scalar(ptr(a), int(c) % q, ptr(out), a.size, q)
    return out


def bconv(x: np.ndarray, in_mod, in_factor, out_mod, cross, centred: bool = False) -> np.ndarray:
    """Fast base conversion; x is [n_in][n]; cross[i][m]; returns [n_out][n].
    ``centred`` takes each y_i = [x_i * in_factor_i]_{in_mod_i} in (-in_mod_i/2, in_mod_i/2]."""
    x = u64(x)
    n_in, n = x.shape
    n_out = len(out_mod)
    out = np.empty((n_out, n), dtype=np.uint64)
    im = u64(list(in_mod))
    inf = u64(list(in_factor))
    om = u64(list(out_mod))
    cr = u64(np.array(cross, dtype=object).reshape(n_in, n_out).astype(np.uint64))
    lib().orc_bconv(ptr(x), n_in, ptr(im), ptr(inf), n_out, ptr(om), ptr(cr), ptr(out), n, 1 if centred else 0)
    return out


def automorphism_coeff(a: np.ndarray, log_n: int, g: int, q: int) -> np.ndarray:
    a = u64(a)
    out = np.empty_like(a)
    lib().orc_automorphism_coeff(ptr(a), ptr(out), log_n, g, q)
    return out
