"""RNS <-> big-integer conversion by the CRT (the paper's RNS section).  Test infrastructure only.

Z_Q = Z_{q_0} x ... x Z_{q_{l}} for pairwise coprime q_i, Q = prod q_i:
    X = sum_i x_i * (Q/q_i) * [(Q/q_i)^-1]_{q_i}  mod Q.
Polynomials are handled coefficient-wise (numpy object arrays of Python ints).
"""
from __future__ import annotations

from functools import reduce

import numpy as np


def product(moduli) -> int:
    return reduce(lambda x, y: x * y, [int(m) for m in moduli], 1)


def crt(limbs: np.ndarray, moduli) -> np.ndarray:
    """limbs [len(moduli)][n] of residues -> object array of n integers in [0, Q)."""
    moduli = [int(m) for m in moduli]
    Q = product(moduli)
    acc = np.zeros(limbs.shape[-1], dtype=object)
    for i, q in enumerate(moduli):
        qhat = Q // q
        coef = qhat * pow(qhat % q, -1, q)
        acc = acc + limbs[i].astype(object) * coef
    return acc % Q


def centered(x: np.ndarray, Q: int) -> np.ndarray:
    """Representatives in (-Q/2, Q/2]."""
    x = x % Q
    return np.where(x > Q // 2, x - Q, x)


def to_rns(x, moduli) -> np.ndarray:
    """Integers (any sign) -> [len(moduli)][n] uint64 residues."""
    x = np.asarray(x, dtype=object)
    return np.stack([(x % int(q)).astype(np.uint64) for q in moduli])
