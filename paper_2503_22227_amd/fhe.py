"""Python binding of the C ABI: argument marshalling only.

Ciphertexts, keys and workspaces are torch int64 tensors on a HIP device that
hold uint64 residues; every operation runs in the library's kernels on the
current torch stream (torch supplies device memory and streams, nothing else).
Layouts: a ciphertext with l Q-limbs is [2, l, N]; a key is [dnum, 2, L + k, N].
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check, lib

SCHEMES = {"ckks": _lib.RF_CKKS, "bfv": _lib.RF_BFV, "bgv": _lib.RF_BGV}


def _ptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must be on a HIP device")
    if t.dtype not in (torch.int64, torch.uint64):
        raise ValueError("tensor must hold 64-bit residues")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _fptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must be on a HIP device")
    if t.dtype not in (torch.float64, torch.complex128):
        raise ValueError("tensor must hold doubles")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Context:
    """An RNS chain q_0..q_{L-1} | p_0..p_{k-1} at ring degree 2^log_n on one device."""

    def __init__(self, q: Sequence[int], p: Sequence[int], log_n: int, alpha: int,
                 log_nmax: Optional[int] = None, scheme: str = "ckks", t: int = 0,
                 device: int = 0, b: Sequence[int] = (), m_sk: int = 0):
        self.scheme = scheme
        self.t = int(t)
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.log_n = int(log_n)
        self.n = 1 << self.log_n
        self.log_nmax = int(log_nmax if log_nmax is not None else log_n)
        self.alpha = int(alpha)
        self.L = len(self.q)
        self.k = len(self.p)
        self.dnum = (self.L + self.alpha - 1) // self.alpha
        self.device = torch.device("cuda", device)
        qa = (ctypes.c_uint64 * self.L)(*self.q)
        pa = (ctypes.c_uint64 * self.k)(*self.p)
        self.b = [int(x) for x in b]
        ba = (ctypes.c_uint64 * max(1, len(self.b)))(*self.b)
        prm = _lib.rf_params(SCHEMES[scheme], self.log_n, self.log_nmax, self.L,
                             ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)), self.k,
                             ctypes.cast(pa, ctypes.POINTER(ctypes.c_uint64)), self.alpha, int(t),
                             len(self.b), ctypes.cast(ba, ctypes.POINTER(ctypes.c_uint64)), int(m_sk))
        h = ctypes.c_void_p()
        check(lib.rf_ctx_create(ctypes.byref(prm), device, ctypes.byref(h)), "rf_ctx_create")
        self._h = h
        self._ws = {}
        # kernel variants tuned on this device for this shape, when shipped
        from . import autotune
        self.shipped_levels = autotune.apply_shipped(self)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.rf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- memory
    def empty(self, *shape) -> torch.Tensor:
        return torch.empty(shape, dtype=torch.int64, device=self.device)

    def workspace_bytes(self, op: int, nlimbs: int) -> int:
        return int(lib.rf_workspace_bytes(self._h, op, nlimbs))

    def workspace(self, op: int, nlimbs: int, slot: int = 0) -> torch.Tensor:
        """The device workspace of ``slot``, grown to what (op, nlimbs) needs; every call
        on one slot reuses it.  Work enqueued on different streams at the same time must
        use different slots.  A buffer replaced by a larger one is released through torch's
        stream-ordered caching allocator, so queued kernels still see valid memory."""
        nbytes = self.workspace_bytes(op, nlimbs)
        if nbytes == 0:
            raise ValueError("no workspace size for op %d at %d limbs" % (op, nlimbs))
        ws = self._ws.get(slot)
        if ws is None or ws.numel() * 8 < nbytes:
            ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=self.device)
            self._ws[slot] = ws
        return ws

    # ---------------------------------------------------------------- kernel variants
    TUNING_FIELDS = ("ntt_small_below", "ntt_small_tile", "ntt_small_radix", "modup_chunk", "ntt_fused_small_below")

    def set_tuning(self, nlimbs: int, setting: dict) -> None:
        """Kernel variants of level ``nlimbs`` (0: every level); fields not given keep
        their current value (rf_tuning in include/rnsfhe.h)."""
        cur = self.get_tuning(max(1, min(nlimbs, self.L)))
        cur.update(setting)
        t = _lib.rf_tuning(*(int(cur[f]) for f in self.TUNING_FIELDS))
        check(lib.rf_ctx_set_tuning(self._h, nlimbs, ctypes.byref(t)), "rf_ctx_set_tuning")

    def get_tuning(self, nlimbs: int) -> dict:
        t = _lib.rf_tuning()
        check(lib.rf_ctx_get_tuning(self._h, nlimbs, ctypes.byref(t)), "rf_ctx_get_tuning")
        return {f: int(getattr(t, f)) for f in self.TUNING_FIELDS}

    # ---------------------------------------------------------------- operations
    def ntt(self, data: torch.Tensor, first_limb: int, n_limbs: int, n_polys: int = 1) -> torch.Tensor:
        check(lib.rf_ntt(self._h, _ptr(data), first_limb, n_limbs, n_polys, _stream()), "rf_ntt")
        return data

    def intt(self, data: torch.Tensor, first_limb: int, n_limbs: int, n_polys: int = 1) -> torch.Tensor:
        check(lib.rf_intt(self._h, _ptr(data), first_limb, n_limbs, n_polys, _stream()), "rf_intt")
        return data

    def tensor(self, a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        nl = a.shape[1]
        out = self.empty(3, nl, self.n) if out is None else out
        check(lib.rf_tensor(self._h, _ptr(a), _ptr(b), _ptr(out), nl, _stream()), "rf_tensor")
        return out

    def hmult_relin(self, a: torch.Tensor, b: torch.Tensor, rlk: torch.Tensor,
                    out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        nl = a.shape[1]
        out = self.empty(2, nl, self.n) if out is None else out
        ws = self.workspace(_lib.RF_OP_HMULT_RELIN, nl, slot)
        check(lib.rf_hmult_relin(self._h, _ptr(a), _ptr(b), _ptr(rlk), _ptr(out), nl, _ptr(ws),
                                 ws.numel() * 8, _stream()), "rf_hmult_relin")
        return out

    def rotate(self, ct: torch.Tensor, galois: int, gk: torch.Tensor,
               out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        nl = ct.shape[1]
        out = self.empty(2, nl, self.n) if out is None else out
        ws = self.workspace(_lib.RF_OP_ROTATE, nl, slot)
        check(lib.rf_rotate(self._h, _ptr(ct), galois, _ptr(gk), _ptr(out), nl, _ptr(ws),
                            ws.numel() * 8, _stream()), "rf_rotate")
        return out

    def keyswitch(self, d: torch.Tensor, evk: torch.Tensor, out: torch.Tensor,
                  accumulate: bool = False, slot: int = 0) -> torch.Tensor:
        nl = d.shape[-2]
        ws = self.workspace(_lib.RF_OP_KEYSWITCH, nl, slot)
        check(lib.rf_keyswitch(self._h, _ptr(d), _ptr(evk), _ptr(out), nl, 1 if accumulate else 0,
                               _ptr(ws), ws.numel() * 8, _stream()), "rf_keyswitch")
        return out

    def rescale(self, ct: torch.Tensor, out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        nl = ct.shape[1]
        out = self.empty(2, nl - 1, self.n) if out is None else out
        ws = self.workspace(_lib.RF_OP_RESCALE, nl, slot)
        check(lib.rf_rescale(self._h, _ptr(ct), _ptr(out), nl, _ptr(ws), ws.numel() * 8, _stream()),
              "rf_rescale")
        return out

    def modswitch(self, ct: torch.Tensor, out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        """CKKS: drop the last limb.  BGV: (c - delta)/q_l keeping the message mod t; the
        caller multiplies the ciphertext's correction factor by q_l^-1 mod t."""
        nl = ct.shape[1]
        out = self.empty(2, nl - 1, self.n) if out is None else out
        if self.scheme == "bgv":
            ws = self.workspace(_lib.RF_OP_MODSWITCH, nl, slot)
            wp, wb = _ptr(ws), ws.numel() * 8
        else:
            wp, wb = None, 0
        check(lib.rf_modswitch(self._h, _ptr(ct), _ptr(out), nl, wp, wb, _stream()), "rf_modswitch")
        return out

    def add(self, a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(a) if out is None else out
        check(lib.rf_add(self._h, _ptr(a), _ptr(b), _ptr(out), a.shape[1], a.shape[0], _stream()), "rf_add")
        return out

    def sub(self, a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(a) if out is None else out
        check(lib.rf_sub(self._h, _ptr(a), _ptr(b), _ptr(out), a.shape[1], a.shape[0], _stream()), "rf_sub")
        return out

    def mul_scalar(self, a: torch.Tensor, k: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(a) if out is None else out
        check(lib.rf_mul_scalar(self._h, _ptr(a), int(k), _ptr(out), a.shape[1], a.shape[0], _stream()),
              "rf_mul_scalar")
        return out

    def add_scalar(self, a: torch.Tensor, k: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(a) if out is None else out
        check(lib.rf_add_scalar(self._h, _ptr(a), int(k), _ptr(out), a.shape[1], _stream()), "rf_add_scalar")
        return out

    def mul_plain(self, a: torch.Tensor, pt: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(a) if out is None else out
        check(lib.rf_mul_plain(self._h, _ptr(a), _ptr(pt), _ptr(out), a.shape[1], a.shape[0], _stream()),
              "rf_mul_plain")
        return out

    def galois_element(self, rotation: int, conjugate: bool = False) -> int:
        """The Galois element rotating slots left by ``rotation`` (5^r mod 2N), times 2N - 1
        when ``conjugate``; computed by the library."""
        g = ctypes.c_uint32()
        check(lib.rf_galois_element(self._h, int(rotation), 1 if conjugate else 0, ctypes.byref(g)),
              "rf_galois_element")
        return int(g.value)

    # ---------------------------------------------------------------- client side
    def key_ntt(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """NTT-domain form over every prime of the chain ([L + k, N]) of an int64 [N] polynomial."""
        out = self.empty(self.L + self.k, self.n) if out is None else out
        check(lib.rf_key_ntt(self._h, _ptr(x), _ptr(out), _stream()), "rf_key_ntt")
        return out

    def keygen_switch(self, s_ntt: torch.Tensor, galois: int, a: torch.Tensor, e: torch.Tensor,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Switching key [dnum, 2, L + k, N] from s^2 (galois 0) or s(X^g) to s, with the masks
        a [dnum, L + k, N] and errors e [dnum, N] drawn by the caller."""
        out = self.empty(self.dnum, 2, self.L + self.k, self.n) if out is None else out
        check(lib.rf_keygen_switch(self._h, _ptr(s_ntt), int(galois), _ptr(a), _ptr(e), _ptr(out), _stream()),
              "rf_keygen_switch")
        return out

    def encrypt(self, m: torch.Tensor, e: torch.Tensor, a: torch.Tensor, s_ntt: torch.Tensor,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Secret-key encryption of the int64 [N] message coefficients m with error e and mask
        a [limbs, N]; returns [2, limbs, N]."""
        nl = a.shape[0]
        out = self.empty(2, nl, self.n) if out is None else out
        check(lib.rf_encrypt_sk(self._h, _ptr(m), _ptr(e), _ptr(a), _ptr(s_ntt), _ptr(out), nl, _stream()),
              "rf_encrypt_sk")
        return out

    def decrypt(self, ct: torch.Tensor, s_ntt: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Coefficient-domain residues [limbs, N] of the phase c0 + c1 s."""
        nl = ct.shape[1]
        out = self.empty(nl, self.n) if out is None else out
        check(lib.rf_decrypt(self._h, _ptr(ct), _ptr(s_ntt), _ptr(out), nl, _stream()), "rf_decrypt")
        return out

    def crt_centered(self, x: torch.Tensor, scale: float = 1.0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """float64 [N]: the centred integer of the residues x [limbs, N] divided by scale."""
        out = torch.empty(self.n, dtype=torch.float64, device=self.device) if out is None else out
        check(lib.rf_crt_centered(self._h, _ptr(x), _fptr(out), x.shape[0], float(scale), _stream()),
              "rf_crt_centered")
        return out

    def encode(self, z: torch.Tensor, scale: float, out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        """CKKS encode of complex128 [N/2] slots: int64 [N] coefficients."""
        out = self.empty(self.n) if out is None else out
        ws = self.workspace(_lib.RF_OP_ENCODE, 1, slot)
        check(lib.rf_encode_ckks(self._h, _fptr(z), float(scale), _ptr(out), _ptr(ws), ws.numel() * 8, _stream()),
              "rf_encode_ckks")
        return out

    def decode(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, slot: int = 0) -> torch.Tensor:
        """CKKS decode of float64 [N] coefficients (already divided by the scale): complex128 [N/2]."""
        out = torch.empty(self.n // 2, dtype=torch.complex128, device=self.device) if out is None else out
        ws = self.workspace(_lib.RF_OP_DECODE, 1, slot)
        check(lib.rf_decode_ckks(self._h, _fptr(x), _fptr(out), _ptr(ws), ws.numel() * 8, _stream()),
              "rf_decode_ckks")
        return out

    def automorphism(self, x: torch.Tensor, galois: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """sigma_g of a [polys, limbs, N] NTT-domain tensor."""
        npolys, nl = x.shape[0], x.shape[1]
        out = torch.empty_like(x) if out is None else out
        check(lib.rf_automorphism(self._h, _ptr(x), _ptr(out), galois, nl, npolys, _stream()),
              "rf_automorphism")
        return out


BATCH_STAGES = ("tensor", "intt_d2_rows", "intt_d2_cols", "modup_bconv", "ntt_ext_cols", "ntt_ext_rows",
                "inner_product", "intt_p_rows", "intt_p_cols", "moddown_bconv", "ntt_conv_cols",
                "ntt_conv_rows", "moddown_tail")


class BatchPlan:
    """A fixed list of independent HMult+Relin items (mixed ring degree and level)
    executed as one launch per step of the chain, optionally through a hipGraph.

    items: sequence of (ctx, a, b, rlk, out) with a, b, out of shape [2, limbs, N]."""

    def __init__(self, items):
        self._keep = list(items)
        arr = (_lib.rf_batch_item * len(items))()
        for i, (ctx, a, b, rlk, out) in enumerate(items):
            arr[i] = _lib.rf_batch_item(ctx._h, _ptr(a), _ptr(b), _ptr(rlk), _ptr(out), a.shape[1])
        nbytes = int(lib.rf_batch_workspace_bytes(arr, len(items)))
        if nbytes == 0:
            raise ValueError("invalid batch: %s" % lib.rf_last_error().decode())
        dev = items[0][1].device
        self.workspace = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=dev)
        h = ctypes.c_void_p()
        check(lib.rf_batch_create(arr, len(items), _ptr(self.workspace), nbytes, ctypes.byref(h)),
              "rf_batch_create")
        self._h = h
        self.n_items = len(items)

    def close(self):
        if getattr(self, "_h", None):
            lib.rf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, graph: bool = False) -> None:
        if graph:
            check(lib.rf_batch_graph_launch(self._h, _stream()), "rf_batch_graph_launch")
        else:
            check(lib.rf_batch_hmult_relin(self._h, _stream()), "rf_batch_hmult_relin")

    def set_grid(self, stage: int, workgroups: int) -> None:
        check(lib.rf_batch_set_grid(self._h, stage, workgroups), "rf_batch_set_grid")

    def set_modup_chunk(self, chunk: int) -> None:
        check(lib.rf_batch_set_modup_chunk(self._h, chunk), "rf_batch_set_modup_chunk")

    def stage_units(self, stage: int) -> int:
        n = lib.rf_batch_stage_units(self._h, stage)
        if n < 0:
            check(n, "rf_batch_stage_units")
        return n
