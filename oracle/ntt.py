"""The negacyclic NTT over R_q = Z_q[X]/(X^N + 1).  Test infrastructure only.

Definition (used for every pin): for a primitive 2N-th root psi of unity mod q,
    NTT(a)[i] = a(psi^(2*brv(i) + 1)) = sum_j a_j * psi^((2*brv(i)+1)*j)  mod q,
brv the log2(N)-bit reversal.  The points psi^(odd) are exactly the roots of
X^N + 1, so the transform turns negacyclic convolution into a slot-wise
product; the bit-reversed output order is the one the butterfly recursion
produces, so no separate bit-reversal pass is ever needed.

``ntt_definition``/``intt_definition`` evaluate the sums directly in O(N^2)
with Python integers; ``ntt``/``intt`` call the C core's radix-2 transform,
which the tests pin to the definition.
"""
from __future__ import annotations

import numpy as np

from . import _core
from .params import bitrev


def ntt_definition(a, q: int, psi: int) -> list:
    n = len(a)
    logn = n.bit_length() - 1
    a = [int(x) for x in a]
    out = []
    for i in range(n):
        w = pow(psi, 2 * bitrev(i, logn) + 1, q)
        acc, wj = 0, 1
        for j in range(n):
            acc += a[j] * wj
            wj = wj * w % q
        out.append(acc % q)
    return out


def intt_definition(ahat, q: int, psi: int) -> list:
    """Inverse by the inverse-DFT sum: a_j = N^-1 sum_i ahat_i * psi^(-(2 brv(i)+1) j)."""
    n = len(ahat)
    logn = n.bit_length() - 1
    ahat = [int(x) for x in ahat]
    n_inv = pow(n, -1, q)
    psi_inv = pow(psi, -1, q)
    out = [0] * n
    for i in range(n):
        w = pow(psi_inv, 2 * bitrev(i, logn) + 1, q)
        wj = 1
        for j in range(n):
            out[j] += ahat[i] * wj
            wj = wj * w % q
    return [x * n_inv % q for x in out]


def negacyclic_schoolbook(a, b, q: int) -> list:
    """a*b mod (X^N + 1, q) by the O(N^2) product with X^N = -1."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += ai * int(b[j])
            else:
                out[k - n] -= ai * int(b[j])
    return [x % q for x in out]


def ntt(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    n = a.shape[-1]
    return _core.ntt_fwd(a, n.bit_length() - 1, q, psi)


def intt(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    n = a.shape[-1]
    return _core.ntt_inv(a, n.bit_length() - 1, q, psi)


def ntt_limbs(poly: np.ndarray, moduli, params) -> np.ndarray:
    """Forward NTT of each limb of a [limbs][N] array; limb i is mod moduli[i]."""
    return np.stack([ntt(poly[i], q, params.psi(q)) for i, q in enumerate(moduli)])


def intt_limbs(poly: np.ndarray, moduli, params) -> np.ndarray:
    return np.stack([intt(poly[i], q, params.psi(q)) for i, q in enumerate(moduli)])
