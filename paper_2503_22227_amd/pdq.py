"""Private dataset query (PDQ) circuit: planner and GPU executor.

The paper's application (section IV) answers search and search-and-sum
queries over an encrypted table on the server.  Its comparison method is not
described beyond a citation, so the circuit here is the composite sign
approximation: a range predicate lo <= x_a <= hi on column a becomes
    mask = ((F(x_a - lo') + 1)/2) * ((F(hi' - x_a) + 1)/2),   F = f7 o f7 o f7,
    f7(x) = sum_{i=0..7} C(2i, i) / 4^i * x (1 - x^2)^i
(a degree-15 odd polynomial), then sum = sum_r mask_r * x_b[r] and
count = sum_r mask_r by rotate-and-add.

Table layout (CKKS slots): column c, row r at slot c * R_pad + r, R_pad the
next power of two >= R rows; values v in [0, 1000) are encoded as v / 2000,
padding rows as -0.5 (so their predicate is false), lo' = (lo - 1/2) / 2000,
hi' = (hi + 1/2) / 2000 broadcast to every slot.

The planner turns a query shape into an op list: plain data (tuples of ints
and register names) with explicit levels, executed identically by the GPU
executor here and by any other executor.  Ops:
    ("rot", dst, src, r)        rotate slots left by a power of two r (one key switch)
    ("add"|"sub", dst, a, b)    a, b at the same level
    ("hmult", dst, a, b)        HMult+Relin (scale s_a * s_b)
    ("rescale", dst, src)       divide by the last prime
    ("mul_int", dst, src, k)    multiply by the integer k
    ("add_int", dst, src, k)    add the integer k to every slot value * scale
    ("drop", dst, src, limbs)   keep the first `limbs` limbs
    ("client_inv", dst, src, src_scale, limbs, scale)
                                the two-party multiply-inverse's client step
                                (section IV-C): the data holder decrypts src,
                                inverts its slot 0 and sends back a fresh
                                encryption of that constant at `limbs` limbs
                                and `scale`
"""
from __future__ import annotations

from fractions import Fraction
from math import comb
from typing import Dict, List, Tuple

def f7_coefficients() -> List[Fraction]:
    """Odd coefficients c_1, c_3, ..., c_15 of f7 (exact)."""
    coef = [Fraction(0)] * 16
    for i in range(8):
        a = Fraction(comb(2 * i, i), 4 ** i)
        # x (1 - x^2)^i = sum_j C(i, j) (-1)^j x^(2j+1)
        for j in range(i + 1):
            coef[2 * j + 1] += a * comb(i, j) * (-1) ** j
    return [coef[2 * k + 1] for k in range(8)]


F7 = f7_coefficients()


class Planner:
    """Builds an op list with level and scale bookkeeping (no arithmetic on data)."""

    def __init__(self, q: List[int]):
        self.q = list(q)
        self.ops: List[tuple] = []
        self.regs: Dict[str, Tuple[int, float]] = {}
        self._n = 0

    def _tmp(self) -> str:
        self._n += 1
        return "t%d" % self._n

    def input(self, name: str, limbs: int, scale: float) -> str:
        self.regs[name] = (limbs, scale)
        return name

    def limbs(self, r: str) -> int:
        return self.regs[r][0]

    def scale(self, r: str) -> float:
        return self.regs[r][1]

    def drop(self, r: str, limbs: int) -> str:
        if self.limbs(r) == limbs:
            return r
        assert self.limbs(r) > limbs
        d = self._tmp()
        self.ops.append(("drop", d, r, limbs))
        self.regs[d] = (limbs, self.scale(r))
        return d

    def _align(self, a: str, b: str):
        nl = min(self.limbs(a), self.limbs(b))
        return self.drop(a, nl), self.drop(b, nl)

    def add(self, a: str, b: str) -> str:
        a, b = self._align(a, b)
        d = self._tmp()
        self.ops.append(("add", d, a, b))
        self.regs[d] = (self.limbs(a), self.scale(a))
        return d

    def sub(self, a: str, b: str) -> str:
        a, b = self._align(a, b)
        d = self._tmp()
        self.ops.append(("sub", d, a, b))
        self.regs[d] = (self.limbs(a), self.scale(a))
        return d

    def mul(self, a: str, b: str) -> str:
        """HMult+Relin then rescale."""
        a, b = self._align(a, b)
        nl = self.limbs(a)
        assert nl >= 2, "out of levels"
        m = self._tmp()
        self.ops.append(("hmult", m, a, b))
        d = self._tmp()
        self.ops.append(("rescale", d, m))
        self.regs[d] = (nl - 1, self.scale(a) * self.scale(b) / self.q[nl - 1])
        return d

    def mulc(self, a: str, c) -> str:
        """Multiply by a real constant: k = round(c q_last), then rescale by q_last (scale kept)."""
        nl = self.limbs(a)
        assert nl >= 2, "out of levels"
        k = int(round(Fraction(c) * self.q[nl - 1]))
        m = self._tmp()
        self.ops.append(("mul_int", m, a, k))
        d = self._tmp()
        self.ops.append(("rescale", d, m))
        self.regs[d] = (nl - 1, self.scale(a))
        return d

    def addc(self, a: str, c) -> str:
        k = int(round(Fraction(c) * Fraction(self.scale(a))))
        d = self._tmp()
        self.ops.append(("add_int", d, a, k))
        self.regs[d] = (self.limbs(a), self.scale(a))
        return d

    def rot(self, a: str, r: int) -> str:
        """Rotate left by r >= 0: one key switch per set bit of r (keys for powers of two)."""
        cur = a
        bit = 0
        while r:
            if r & 1:
                d = self._tmp()
                self.ops.append(("rot", d, cur, 1 << bit))
                self.regs[d] = self.regs[cur]
                cur = d
            r >>= 1
            bit += 1
        return cur

    def client_inverse(self, a: str, limbs: int, scale: float) -> str:
        """Fresh encryption of 1 / slot0(a) in every slot, made by the client."""
        d = self._tmp()
        self.ops.append(("client_inv", d, a, self.scale(a), limbs, scale))
        self.regs[d] = (limbs, scale)
        return d

    def odd_poly15(self, x: str, coef) -> str:
        """sum_k coef[k] x^(2k+1): y = x^2, q(y) by baby-step giant-step, result x q(y)."""
        y = self.mul(x, x)
        y2 = self.mul(y, y)
        y3 = self.mul(y, y2)
        y4 = self.mul(y2, y2)

        def cubic(c0, c1, c2, c3):
            t = self.add(self.add(self.mulc(y, c1), self.mulc(y2, c2)), self.mulc(y3, c3))
            return self.addc(t, c0)

        lo = cubic(*coef[0:4])
        hi = cubic(*coef[4:8])
        q = self.add(lo, self.mul(y4, hi))
        return self.mul(x, q)

    def sign01(self, x: str) -> str:
        """(F(x) + 1) / 2 with F = f7 o f7 o f7; the affine map folded into the last round."""
        s = self.odd_poly15(x, F7)
        s = self.odd_poly15(s, F7)
        s = self.odd_poly15(s, [c / 2 for c in F7])
        return self.addc(s, Fraction(1, 2))

    def rotsum(self, a: str, width: int) -> str:
        """Slot 0 <- sum of slots [0, width): rotate-and-add with 1, 2, ..., width/2."""
        acc = a
        r = 1
        while r < width:
            acc = self.add(acc, self.rot(acc, r))
            r <<= 1
        return acc


def r_pad(rows: int) -> int:
    p = 1
    while p < rows:
        p <<= 1
    return p


def plan_query(q: List[int], limbs: int, scale: float, rows: int, col_a: int, col_b: int):
    """Op list of one range-sum query; inputs T (table), LO, HI; outputs (sum, count)."""
    pl = Planner(q)
    T = pl.input("T", limbs, scale)
    LO = pl.input("LO", limbs, scale)
    HI = pl.input("HI", limbs, scale)
    width = r_pad(rows)
    xa = pl.rot(T, col_a * width)
    xb = pl.rot(T, col_b * width)
    m1 = pl.sign01(pl.sub(xa, LO))
    m2 = pl.sign01(pl.sub(HI, xa))
    mask = pl.mul(m1, m2)
    prod = pl.mul(mask, xb)
    s = pl.rotsum(prod, width)
    c = pl.rotsum(mask, width)
    return pl.ops, (s, c), pl.regs


def plan_average_query(q: List[int], limbs: int, scale: float, rows: int, col_a: int, col_b: int, r: float):
    """Op list of one search-and-average query (section IV-C): the range-sum circuit,
    then the two-party multiply-inverse of the count (the paper's Algorithm "The
    Two-Party Multiply-Inverse Method"): the server masks the count by its random
    r, the client decrypts r count, inverts it and encrypts 1 / (r count) afresh,
    the server multiplies that by r (giving 1 / count) and by the sum.  Inputs T,
    LO, HI; outputs (average, sum, count), the average in slot 0."""
    pl = Planner(q)
    T = pl.input("T", limbs, scale)
    LO = pl.input("LO", limbs, scale)
    HI = pl.input("HI", limbs, scale)
    width = r_pad(rows)
    xa = pl.rot(T, col_a * width)
    xb = pl.rot(T, col_b * width)
    mask = pl.mul(pl.sign01(pl.sub(xa, LO)), pl.sign01(pl.sub(HI, xa)))
    s = pl.rotsum(pl.mul(mask, xb), width)
    c = pl.rotsum(mask, width)
    inv = pl.client_inverse(pl.mulc(c, r), limbs, scale)
    avg = pl.mul(s, pl.mulc(inv, r))
    return pl.ops, (avg, s, c), pl.regs


def rotation_amounts(ops) -> List[int]:
    return sorted({op[3] for op in ops if op[0] == "rot"})


def peak_live(ops, inputs=("T", "LO", "HI"), outputs=()) -> int:
    """Most registers alive at once while the op list runs."""
    last_use = {}
    for i, op in enumerate(ops):
        for r in op[2:]:
            if isinstance(r, str):
                last_use[r] = i
    for r in outputs:
        last_use[r] = len(ops)
    live = set(inputs)
    peak = len(live)
    for i, op in enumerate(ops):
        live.add(op[1])
        peak = max(peak, len(live))
        live = {r for r in live if last_use.get(r, -1) > i}
    return peak


class GpuClient:
    """The data holder's side of the multiply-inverse protocol on the GPU (the
    client runs the same framework, section IV-A): its secret key in the NTT
    domain and its own random streams for fresh encryptions (numpy Generators
    drawn in the order of the oracle's encryption: masks from ``rng_a``, errors
    from ``rng_e``)."""

    def __init__(self, ctx, s_ntt, rng_a, rng_e):
        self.ctx = ctx
        self.s_ntt = s_ntt
        self.rng_a = rng_a
        self.rng_e = rng_e

    def slot0(self, ct, scale: float) -> float:
        """Real part of slot 0 of the decryption of ct (waits for the stream)."""
        c = self.ctx
        z = c.decode(c.crt_centered(c.decrypt(ct, self.s_ntt), scale))
        return float(z[0].real.item())

    def _encrypt(self, m, limbs: int):
        import numpy as np
        import torch

        import synthetic
        c = self.ctx
        a = synthetic.uniform_residues(self.rng_a, c.q[:limbs], c.n)
        e = synthetic.gaussian(self.rng_e, c.n)
        return c.encrypt(m, torch.from_numpy(e).to(c.device), torch.from_numpy(a.view(np.int64)).to(c.device),
                         self.s_ntt)

    def encrypt_constant(self, v: float, limbs: int, scale: float):
        """Fresh encryption of v in every slot: the constant polynomial round(v scale)
        (0 for a value that is not finite or does not fit the coefficient)."""
        import math

        import torch
        c = self.ctx
        k = v * scale
        m = torch.zeros(c.n, dtype=torch.int64, device=c.device)
        m[0] = int(round(k)) if math.isfinite(k) and abs(k) < 2.0 ** 62 else 0
        return self._encrypt(m, limbs)

    def encrypt_slots(self, z, limbs: int, scale: float):
        """Fresh encryption of the complex128 slot vector z (N/2 values): GPU encode, then encrypt."""
        import torch
        return self._encrypt(self.ctx.encode(torch.as_tensor(z).to(self.ctx.device), scale), limbs)

    def encrypt_table(self, values, limbs: int, scale: float):
        """The table [rows][4] of integers in [0, 1000): column c, row r at slot c R_pad + r
        holding v / 2000, padding rows -0.5 (see the module docstring)."""
        import numpy as np
        rows = len(values)
        w = r_pad(rows)
        z = np.zeros(self.ctx.n // 2, dtype=np.complex128)
        for c in range(4):
            z[c * w:(c + 1) * w] = -0.5
            z[c * w:c * w + rows] = np.asarray(values)[:, c] / 2000.0
        return self.encrypt_slots(z, limbs, scale)

    def encrypt_bounds(self, lo: int, hi: int, limbs: int, scale: float):
        """(LO, HI): (lo - 1/2) / 2000 and (hi + 1/2) / 2000 in every slot."""
        return (self.encrypt_constant((lo - 0.5) / 2000.0, limbs, scale),
                self.encrypt_constant((hi + 0.5) / 2000.0, limbs, scale))

    def switch_keys(self, amounts, rng):
        """{"rlk": relinearisation key, r: Galois key of the rotation by r} made on the GPU
        from the secret key, with masks and errors drawn from ``rng``."""
        import numpy as np
        import torch

        import synthetic
        c = self.ctx
        qp = c.q + c.p

        def one(g):
            a = np.stack([synthetic.uniform_residues(rng, qp, c.n) for _ in range(c.dnum)])
            e = np.stack([synthetic.gaussian(rng, c.n) for _ in range(c.dnum)])
            return c.keygen_switch(self.s_ntt, g, torch.from_numpy(a.view(np.int64)).to(c.device),
                                   torch.from_numpy(e).to(c.device))

        keys = {"rlk": one(0)}
        for r in amounts:
            keys[r] = one(c.galois_element(r))
        return keys

    def inverse(self, ct, src_scale: float, limbs: int, scale: float):
        return self.encrypt_constant(1.0 / self.slot0(ct, src_scale), limbs, scale)


class GpuExecutor:
    """Runs op lists with the library on the current torch stream.

    keys: {"rlk": tensor, r: galois key tensor for rotation by r}.  ``slot``
    selects the workspace set, so op lists on different streams never share
    scratch memory.  ``client``: the GpuClient (or any object with its
    ``inverse``) that answers "client_inv" steps."""

    def __init__(self, ctx, keys: dict, client=None):
        self.ctx = ctx
        self.keys = keys
        self.client = client
        self.gal = {r: ctx.galois_element(r) for r in keys if r != "rlk"}

    def run(self, ops, regs: dict, slot: int = 0) -> dict:
        for op in ops:
            self.step(op, regs, slot)
        return regs

    def step(self, op, regs: dict, slot: int = 0) -> None:
        c = self.ctx
        kind, dst = op[0], op[1]
        if kind == "add":
            regs[dst] = c.add(regs[op[2]], regs[op[3]])
        elif kind == "sub":
            regs[dst] = c.sub(regs[op[2]], regs[op[3]])
        elif kind == "hmult":
            regs[dst] = c.hmult_relin(regs[op[2]], regs[op[3]], self.keys["rlk"], slot=slot)
        elif kind == "rescale":
            regs[dst] = c.rescale(regs[op[2]], slot=slot)
        elif kind == "mul_int":
            regs[dst] = c.mul_scalar(regs[op[2]], op[3])
        elif kind == "add_int":
            regs[dst] = c.add_scalar(regs[op[2]], op[3])
        elif kind == "rot":
            regs[dst] = c.rotate(regs[op[2]], self.gal[op[3]], self.keys[op[3]], slot=slot)
        elif kind == "drop":
            src = regs[op[2]]
            regs[dst] = src[:, :op[3]].contiguous()
        elif kind == "client_inv":
            if self.client is None:
                raise ValueError("a client_inv step needs a client")
            regs[dst] = self.client.inverse(regs[op[2]], op[3], op[4], op[5])
        else:
            raise ValueError("unknown op %r" % (kind,))


def last_uses(ops, outputs=()) -> Dict[str, int]:
    """Index of the last op reading each register (outputs live to the end)."""
    last = {}
    for i, op in enumerate(ops):
        for r in op[2:]:
            if isinstance(r, str):
                last[r] = i
    for r in outputs:
        last[r] = len(ops)
    return last
