"""Parameters of the RNS chains: primes, roots of unity, digit partition.

Test infrastructure only.

The paper fixes only the ring degree, the number of limbs and the total bit
count of its benchmark chain (evaluation setup, "N=32768, L=16, Q=881") and
represents Z_Q as a product of word-sized Z_{q_i} by the CRT (RNS section).
Everything else here is a reading, listed with the design notes:

* every prime is congruent to 1 mod 2*N_max so that Z_q holds a primitive
  2N-th root of unity for every N <= N_max;
* primes are taken largest first within their bit size, in the order the
  chain lists its sizes (Q primes, then special primes P, then auxiliary
  bases), and a prime is never used twice;
* psi_max = g^((q-1)/(2 N_max)) for the smallest integer g >= 2 whose power is
  a primitive 2N_max-th root (psi_max^N_max = -1), and psi_N = psi_max^(N_max/N);
* hybrid key-switching digits are consecutive runs of ``alpha`` Q-primes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (bases 2..37)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_primes_down(bits: int, modulus: int, count: int, used: set) -> List[int]:
    """The ``count`` largest unused primes q = 1 mod ``modulus`` with 2^(bits-1) <= q < 2^bits."""
    out = []
    c = ((1 << bits) - 2) // modulus * modulus + 1  # largest candidate below 2^bits
    while len(out) < count:
        if c < (1 << (bits - 1)):
            raise ValueError("not enough %d-bit primes = 1 mod %d" % (bits, modulus))
        if c not in used and is_prime(c):
            out.append(c)
            used.add(c)
        c -= modulus
    return out


def prime_chain(bit_groups, modulus: int) -> List[List[int]]:
    """One prime list per group of bit sizes, drawn in order from a shared pool."""
    used: set = set()
    groups = []
    for sizes in bit_groups:
        g = []
        for b in sizes:
            g += next_primes_down(b, modulus, 1, used)
        groups.append(g)
    return groups


def root_2n(q: int, nmax: int) -> int:
    """psi_max: g^((q-1)/(2 nmax)) for the smallest g >= 2 with psi_max^nmax = -1 mod q."""
    assert (q - 1) % (2 * nmax) == 0
    g = 2
    while True:
        psi = pow(g, (q - 1) // (2 * nmax), q)
        if pow(psi, nmax, q) == q - 1:
            return psi
        g += 1


def bitrev(x: int, bits: int) -> int:
    r = 0
    for i in range(bits):
        r |= ((x >> i) & 1) << (bits - 1 - i)
    return r


@dataclass
class Params:
    """One RNS parameter set at ring degree N = 2^log_n.

    q: the ciphertext primes q_0..q_{L-1} (rescale drops the last one first);
    p: the special primes of hybrid key switching; alpha: Q-primes per digit.
    """
    log_n: int
    log_nmax: int
    q: List[int]
    p: List[int]
    alpha: int
    scheme: str = "ckks"
    log_scale: int = 40
    t: int = 0
    b: List[int] = field(default_factory=list)
    msk: int = 0
    log_mtilde: int = 0

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def k(self) -> int:
        return len(self.p)

    def psi(self, prime: int) -> int:
        """Primitive 2N-th root of unity mod ``prime`` for this ring degree."""
        nmax = 1 << self.log_nmax
        return pow(root_2n(prime, nmax), nmax // self.n, prime)

    def digits(self, nlimbs: int) -> List[List[int]]:
        """Limb indices of each key-switching digit at a level with ``nlimbs`` Q-limbs."""
        return [list(range(j, min(j + self.alpha, nlimbs))) for j in range(0, nlimbs, self.alpha)]

    def dnum(self, nlimbs: int | None = None) -> int:
        nl = self.L if nlimbs is None else nlimbs
        return (nl + self.alpha - 1) // self.alpha

    def at_degree(self, log_n: int) -> "Params":
        """The same chain used at a smaller ring degree (roots are strided powers)."""
        assert log_n <= self.log_nmax
        return Params(log_n, self.log_nmax, self.q, self.p, self.alpha, self.scheme,
                      self.log_scale, self.t, self.b, self.msk, self.log_mtilde)


def make_params(w: dict) -> Params:
    """Build the parameter set of a workload description (see ``synthetic.WORKLOADS``)."""
    modulus = 2 << w["log_nmax"]
    groups = [w["q_bits"], w["p_bits"]]
    if w.get("b_bits"):
        groups += [w["b_bits"], [w["msk_bits"]]]
    chain = prime_chain(groups, modulus)
    q, p = chain[0], chain[1]
    b = chain[2] if len(chain) > 2 else []
    msk = chain[3][0] if len(chain) > 3 else 0
    return Params(log_n=w["log_n"], log_nmax=w["log_nmax"], q=q, p=p, alpha=w["alpha"],
                  scheme=w["scheme"], log_scale=w.get("log_scale", 40), t=w.get("t", 0),
                  b=b, msk=msk, log_mtilde=w.get("log_mtilde", 0))
