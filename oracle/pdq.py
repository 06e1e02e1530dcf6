"""Private-table query circuit on the CPU: client encoding, an executor of op
lists with the oracle's CKKS operations, and the float64 evaluation of the
same circuit.  Test infrastructure only.

Search-and-average (section IV-C) adds the paper's two-party multiply-inverse
of the count: the server masks it by a random r, the client (``Client``)
decrypts, inverts and re-encrypts, the server unmasks by r and multiplies by
the sum.

The circuit (section IV of the paper: search-and-sum over an encrypted table;
its comparison method is only cited, so the composite sign polynomial stands
in): mask_r = ((F(x_a[r] - lo') + 1)/2) ((F(hi' - x_a[r]) + 1)/2) with
F = f7 o f7 o f7, f7(x) = sum_{i=0..7} C(2i, i)/4^i x (1 - x^2)^i; the result
is (sum_r mask_r x_b[r], sum_r mask_r) over the R_pad row slots of the table.
Values v in [0, 1000) are encoded as v/2000, padding rows as -0.5,
lo' = (lo - 1/2)/2000, hi' = (hi + 1/2)/2000.
"""
from __future__ import annotations

from math import comb

import numpy as np

from . import ckks as C

ROWS_SCALE = 2000.0
PAD_VALUE = -0.5


def f7(x):
    """The degree-15 sign approximation, summed term by term from its definition."""
    x = np.asarray(x, dtype=np.float64)
    return sum(comb(2 * i, i) / 4.0 ** i * x * (1.0 - x * x) ** i for i in range(8))


def sign01(x):
    return (f7(f7(f7(x))) + 1.0) / 2.0


def r_pad(rows: int) -> int:
    p = 1
    while p < rows:
        p <<= 1
    return p


def table_slots(values: np.ndarray, n_slots: int) -> np.ndarray:
    """values [R][4] ints in [0, 1000) -> slot vector: column c, row r at c * R_pad + r."""
    rows = values.shape[0]
    w = r_pad(rows)
    assert 4 * w <= n_slots
    z = np.zeros(n_slots, dtype=np.complex128)
    for c in range(4):
        z[c * w:(c + 1) * w] = PAD_VALUE
        z[c * w:c * w + rows] = values[:, c] / ROWS_SCALE
    return z


def bound_slots(lo: int, hi: int, n_slots: int):
    return (np.full(n_slots, (lo - 0.5) / ROWS_SCALE, dtype=np.complex128),
            np.full(n_slots, (hi + 0.5) / ROWS_SCALE, dtype=np.complex128))


def reference(values: np.ndarray, lo: int, hi: int, col_a: int, col_b: int):
    """float64 evaluation of the circuit: (sum, count) over the R_pad row slots."""
    rows = values.shape[0]
    w = r_pad(rows)
    xa = np.full(w, PAD_VALUE)
    xb = np.full(w, PAD_VALUE)
    xa[:rows] = values[:, col_a] / ROWS_SCALE
    xb[:rows] = values[:, col_b] / ROWS_SCALE
    lo_s, hi_s = (lo - 0.5) / ROWS_SCALE, (hi + 0.5) / ROWS_SCALE
    mask = sign01(xa - lo_s) * sign01(hi_s - xa)
    return float(np.sum(mask * xb)), float(np.sum(mask))


def exact_answer(values: np.ndarray, lo: int, hi: int, col_a: int, col_b: int):
    """The SQL answer the circuit approximates: (sum of v_b / 2000, count) over lo <= v_a <= hi."""
    sel = (values[:, col_a] >= lo) & (values[:, col_a] <= hi)
    return float(values[sel, col_b].sum() / ROWS_SCALE), float(sel.sum())


def reference_average(values: np.ndarray, lo: int, hi: int, col_a: int, col_b: int) -> float:
    """float64 evaluation of the search-and-average circuit: sum / count of ``reference``."""
    total, count = reference(values, lo, hi, col_a, col_b)
    return total / count


class Client:
    """The data holder in the two-party multiply-inverse (section IV-C, Algorithm
    "The Two-Party Multiply-Inverse Method"), on the oracle.  Given the server's
    C1 = Enc(r x) it decrypts x1 = Dec(C1) (slot 0), computes x2 = 1 / x1 and
    returns a fresh encryption of x2 in every slot: the constant polynomial
    round(x2 scale), secret-key encrypted with masks from ``rng_a`` and errors
    from ``rng_e``."""

    def __init__(self, params, s, rng_a, rng_e):
        self.p = params
        self.s = s
        self.rng_a = rng_a
        self.rng_e = rng_e

    def inverse(self, ct: C.Ciphertext, src_scale: float, limbs: int, scale: float) -> C.Ciphertext:
        p = self.p
        x1 = C.decode(C.decrypt(p, self.s, C.Ciphertext(ct.data, src_scale)), src_scale, p.n)[0].real
        x2 = 1.0 / x1
        m = np.zeros(p.n, dtype=object)
        m[0] = int(round(x2 * scale))
        return C.encrypt(p, self.s, m, limbs, scale, self.rng_a, self.rng_e)


def rotation_keys(params, s, amounts, rng) -> dict:
    """{r: Galois key rotating slots left by r}."""
    return {r: C.galois_key(params, s, C.galois_element(r, params.n), rng) for r in amounts}


class Executor:
    """Runs an op list with the oracle (registers are oracle Ciphertexts);
    ``client`` answers the multiply-inverse's client steps."""

    def __init__(self, params, rlk, gkeys: dict, client=None):
        self.p = params
        self.rlk = rlk
        self.gkeys = gkeys
        self.client = client

    def run(self, ops, regs: dict) -> dict:
        for op in ops:
            self.step(op, regs)
        return regs

    def step(self, op, regs: dict, slot: int = 0) -> None:
        p = self.p
        kind, dst = op[0], op[1]
        if kind == "add":
            regs[dst] = C.ct_add(regs[op[2]], regs[op[3]], p)
        elif kind == "sub":
            regs[dst] = C.ct_sub(regs[op[2]], regs[op[3]], p)
        elif kind == "hmult":
            regs[dst] = C.hmult_relin(regs[op[2]], regs[op[3]], self.rlk, p)
        elif kind == "rescale":
            regs[dst] = C.rescale(regs[op[2]], p)
        elif kind == "mul_int":
            regs[dst] = C.ct_mul_int(regs[op[2]], op[3], p)
        elif kind == "add_int":
            regs[dst] = C.ct_add_int(regs[op[2]], op[3], p)
        elif kind == "rot":
            r = op[3]
            regs[dst] = C.rotate(regs[op[2]], C.galois_element(r, p.n), self.gkeys[r], p)
        elif kind == "drop":
            src = regs[op[2]]
            regs[dst] = C.Ciphertext(src.data[:, :op[3]].copy(), src.scale)
        elif kind == "client_inv":
            regs[dst] = self.client.inverse(regs[op[2]], op[3], op[4], op[5])
        else:
            raise ValueError("unknown op %r" % (kind,))
