"""BGV over RNS limbs (the paper's BGV operator table; "similar to CKKS").  Test infrastructure only.

Plaintexts live in R_t, t prime with t = 1 mod 2N, so R_t splits into N slots:
slot i is the evaluation at psi_t^(2 brv(i) + 1) (the same order as the NTT
of the ciphertext primes), and slot-wise products of plaintexts are products
of polynomials.  Ciphertexts (c0, c1) rest in the NTT domain of Q_l and
decrypt to [c0 + c1 s]_Q = f m (mod t) for a correction factor f kept beside
the ciphertext:

* encryption (secret key): (-a s + t e + m, a), f = 1;
* HMult+Relin: the CKKS tensor, then key switching with keys of error t e_j
  and a ModDown that keeps the message mod t: out = (y - delta)/P with
  delta = t [y t^-1]_P (centred digits), delta = 0 mod t, delta = y mod P;
  f_out = f_a f_b;
* modulus switch: c' = (c - delta)/q_l, delta = t [c t^-1]_{q_l} (centred),
  f' = f q_l^-1 mod t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synthetic
from . import _core
from . import ckks as C
from .ntt import intt, intt_limbs, ntt, ntt_limbs
from .params import Params, root_2n
from .rns import centered, crt, product, to_rns


@dataclass
class Ciphertext:
    data: np.ndarray  # uint64 [2][limbs][N], NTT domain
    factor: int = 1   # correction factor f: decrypts to f m mod t

    @property
    def nlimbs(self) -> int:
        return self.data.shape[1]


def psi_t(params: Params) -> int:
    return root_2n(params.t, params.n)


def encode(z: np.ndarray, params: Params) -> np.ndarray:
    """Slots z (integers mod t) -> coefficients in [0, t): the inverse NTT mod t."""
    t = params.t
    return intt(np.asarray(z, dtype=np.int64).astype(np.uint64) % np.uint64(t), t, psi_t(params))


def decode(m: np.ndarray, params: Params) -> np.ndarray:
    t = params.t
    mm = np.array([int(x) % t for x in m], dtype=np.uint64)
    return ntt(mm, t, psi_t(params)).astype(np.int64)


def relin_key(params: Params, s: np.ndarray, rng) -> np.ndarray:
    return C.switch_key(params, s, C.negacyclic_square(s), rng, err_mult=params.t)


def galois_key(params: Params, s: np.ndarray, g: int, rng) -> np.ndarray:
    return C.switch_key(params, s, C.automorphism_coeffs(s, g), rng, err_mult=params.t)


def encrypt(params: Params, s: np.ndarray, m: np.ndarray, nlimbs: int, rng_a, rng_e) -> Ciphertext:
    moduli = params.q[:nlimbs]
    a = synthetic.uniform_residues(rng_a, moduli, params.n)
    e = C.small_to_ntt(synthetic.gaussian(rng_e, params.n) * params.t, moduli, params)
    mh = ntt_limbs(to_rns(np.array([int(x) for x in m], dtype=object), moduli), moduli, params)
    sh = C.small_to_ntt(s, moduli, params)
    c0 = C.poly_add(C.poly_add(C.poly_neg(C.poly_mul(a, sh, moduli), moduli), e, moduli), mh, moduli)
    return Ciphertext(np.stack([c0, a]), 1)


def decrypt(params: Params, s: np.ndarray, ct: Ciphertext) -> np.ndarray:
    """Slots of f^-1 [c0 + c1 s]_Q mod t."""
    moduli = params.q[:ct.nlimbs]
    sh = C.small_to_ntt(s, moduli, params)
    v = C.poly_add(ct.data[0], C.poly_mul(ct.data[1], sh, moduli), moduli)
    x = centered(crt(intt_limbs(v, moduli, params), moduli), product(moduli))
    t = params.t
    finv = pow(ct.factor, -1, t)
    m = np.array([int(c) % t * finv % t for c in x], dtype=object)
    return decode(m, params)


def noise_bits(params: Params, s: np.ndarray, ct: Ciphertext) -> float:
    """log2 of max |[c0 + c1 s]_Q| (centred): the budget left is log2(Q/2) minus this."""
    moduli = params.q[:ct.nlimbs]
    sh = C.small_to_ntt(s, moduli, params)
    v = C.poly_add(ct.data[0], C.poly_mul(ct.data[1], sh, moduli), moduli)
    x = centered(crt(intt_limbs(v, moduli, params), moduli), product(moduli))
    return float(np.log2(max(abs(int(c)) for c in x) + 1))


def moddown(y: np.ndarray, params: Params, nlimbs: int) -> np.ndarray:
    """(y - delta) / P on Q_l, delta = t * conv_P->Q( centred [y_P t^-1]_P )."""
    qs = params.q[:nlimbs]
    ps = params.p
    t = params.t
    P = product(ps)
    yp = intt_limbs(y[nlimbs:], ps, params)
    z = np.stack([_core.mul_scalar(yp[i], pow(t, -1, p), p) for i, p in enumerate(ps)])
    in_factor = [pow((P // p) % p, -1, p) for p in ps]
    cross = [[(P // p) % q for q in qs] for p in ps]
    conv = _core.bconv(z, ps, in_factor, qs, cross, centred=True)
    out = np.empty((nlimbs, params.n), dtype=np.uint64)
    for i, q in enumerate(qs):
        delta = _core.mul_scalar(conv[i], t % q, q)
        dh = ntt(delta, q, params.psi(q))
        out[i] = _core.mul_scalar(_core.sub(y[i], dh, q), pow(P % q, -1, q), q)
    return out


def hmult_relin(a: Ciphertext, b: Ciphertext, rlk: np.ndarray, params: Params) -> Ciphertext:
    assert a.nlimbs == b.nlimbs
    moduli = params.q[:a.nlimbs]
    d0, d1, d2 = C.tensor(C.Ciphertext(a.data, 1.0), C.Ciphertext(b.data, 1.0), params)
    k0, k1 = C.keyswitch(d2, rlk, params, moddown_fn=moddown)
    return Ciphertext(np.stack([C.poly_add(d0, k0, moduli), C.poly_add(d1, k1, moduli)]),
                      a.factor * b.factor % params.t)


def modswitch(ct: Ciphertext, params: Params) -> Ciphertext:
    """Drop q_l keeping the message mod t: c' = (c - delta)/q_l with delta = t [c t^-1]_{q_l}."""
    nl = ct.nlimbs
    assert nl >= 2
    t = params.t
    ql = params.q[nl - 1]
    out = np.empty((2, nl - 1, params.n), dtype=np.uint64)
    for c in range(2):
        last = intt(ct.data[c, nl - 1], ql, params.psi(ql))
        z = _core.mul_scalar(last, pow(t, -1, ql), ql).astype(object)
        r = np.where(z > ql // 2, z - ql, z)  # centred
        for i in range(nl - 1):
            q = params.q[i]
            delta = ((r * t) % q).astype(np.uint64)
            dh = ntt(delta, q, params.psi(q))
            out[c, i] = _core.mul_scalar(_core.sub(ct.data[c, i], dh, q), pow(ql % q, -1, q), q)
    return Ciphertext(out, ct.factor * pow(ql, -1, t) % t)


def rotate(ct: Ciphertext, g: int, gk: np.ndarray, params: Params) -> Ciphertext:
    """Galois automorphism then key switching back to s (BGV keys and ModDown)."""
    moduli = params.q[:ct.nlimbs]
    c0 = C.automorphism_ntt(ct.data[0], g, moduli, params)
    c1 = C.automorphism_ntt(ct.data[1], g, moduli, params)
    k0, k1 = C.keyswitch(c1, gk, params, moddown_fn=moddown)
    return Ciphertext(np.stack([C.poly_add(c0, k0, moduli), k1]), ct.factor)
