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


class GpuExecutor:
    """Runs op lists with the library on the current torch stream.

    keys: {"rlk": tensor, r: galois key tensor for rotation by r}.  ``slot``
    selects the workspace set, so op lists on different streams never share
    scratch memory."""

    def __init__(self, ctx, keys: dict):
        self.ctx = ctx
        self.keys = keys
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
