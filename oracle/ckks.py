"""CKKS client and server operations over RNS limbs.  Test infrastructure only.

Ciphertexts are (c0, c1) pairs of polynomials in R_Q (the paper's ciphertext
ring), stored as uint64 arrays [2][limbs][N] in the NTT domain, limb i mod
q_i.  The operations the paper times (multiply, relinearize, rescale,
rotate; CKKS operator table) are written from their textbook definitions:

* multiply (tensor): d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 -- the five
  products/sums the paper fuses in its kernel-fusion example;
* relinearize / rotate: hybrid key switching.  d is split into digits of
  ``alpha`` consecutive Q-primes; each digit is lifted to Q_l u P by fast base
  conversion (ModUp), multiplied by the key and summed (inner product), and
  brought back to Q_l by the floor form of division by P (ModDown);
* rescale: round(c / q_l) on the centred representative of c mod q_l (the
  level concept of the RNS section: one prime is dropped per level);
* rotate by r: the Galois automorphism a(X) -> a(X^g), g = 5^r mod 2N,
  followed by key switching from s(X^g) back to s.

Random values come from ``synthetic`` streams; nothing here draws its own.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synthetic
from . import _core
from .ntt import intt, intt_limbs, ntt, ntt_limbs
from .params import Params
from .rns import centered, crt, product, to_rns


@dataclass
class Ciphertext:
    data: np.ndarray  # uint64 [2][limbs][N], NTT domain
    scale: float

    @property
    def nlimbs(self) -> int:
        return self.data.shape[1]


# ---------------------------------------------------------------- limb helpers

def _map2(fn, a, b, moduli):
    return np.stack([fn(a[i], b[i], q) for i, q in enumerate(moduli)])


def poly_mul(a, b, moduli):
    return _map2(_core.mul, a, b, moduli)


def poly_add(a, b, moduli):
    return _map2(_core.add, a, b, moduli)


def poly_sub(a, b, moduli):
    return _map2(_core.sub, a, b, moduli)


def poly_neg(a, moduli):
    return poly_sub(np.zeros_like(a), a, moduli)


def small_to_ntt(coeffs: np.ndarray, moduli, params: Params) -> np.ndarray:
    """Signed small integer coefficients -> NTT-domain limbs."""
    return ntt_limbs(to_rns(coeffs, moduli), moduli, params)


# ---------------------------------------------------------------- encoding

def _slot_exponents(n: int) -> np.ndarray:
    """k_j = 5^j mod 2N for the N/2 slots."""
    e = np.empty(n // 2, dtype=np.int64)
    x = 1
    for j in range(n // 2):
        e[j] = x
        x = x * 5 % (2 * n)
    return e


def encode(z: np.ndarray, scale: float, n: int) -> np.ndarray:
    """m = round(scale * tau^-1(z)): integer coefficients whose evaluation at
    zeta^(5^j) (zeta = exp(i pi / N)) is scale * z_j.  Returns an object array of ints."""
    assert z.shape == (n // 2,)
    k = _slot_exponents(n)
    v = np.zeros(2 * n, dtype=np.complex128)
    v[k] = z
    v[2 * n - k] = np.conj(z)
    u = v[1::2]  # values at the odd exponents 2t+1
    i = np.arange(n)
    coeff = np.exp(-1j * np.pi * i / n) * np.fft.fft(u) / n
    m = np.rint(coeff.real * scale)
    return np.array([int(x) for x in m], dtype=object)


def decode(m: np.ndarray, scale: float, n: int) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) / scale from centred integer coefficients."""
    mf = np.array([float(int(x)) for x in m], dtype=np.float64) / scale
    i = np.arange(n)
    vals = np.fft.ifft(mf * np.exp(1j * np.pi * i / n)) * n  # value at zeta^(2t+1)
    k = _slot_exponents(n)
    return vals[(k - 1) // 2]


def encode_direct(z: np.ndarray, scale: float, n: int) -> np.ndarray:
    """O(N^2) encode by the inverse-DFT sum over the 2N-th roots (for pins)."""
    k = _slot_exponents(n)
    v = {}
    for j in range(n // 2):
        v[int(k[j])] = z[j]
        v[int(2 * n - k[j])] = np.conj(z[j])
    out = []
    for i in range(n):
        s = sum(v[e] * np.exp(-1j * np.pi * e * i / n) for e in v)
        out.append(int(np.rint(s.real / n * scale)))
    return np.array(out, dtype=object)


def decode_direct(m, scale: float, n: int) -> np.ndarray:
    k = _slot_exponents(n)
    mf = [float(int(x)) / scale for x in m]
    return np.array([sum(mf[i] * np.exp(1j * np.pi * int(e) * i / n) for i in range(n))
                     for e in k])


# ---------------------------------------------------------------- keys

def secret_key(params: Params, rng) -> np.ndarray:
    return synthetic.ternary(rng, params.n)


def automorphism_coeffs(s: np.ndarray, g: int) -> np.ndarray:
    """a(X) -> a(X^g) on signed integer coefficients."""
    n = len(s)
    out = np.zeros(n, dtype=np.int64)
    for j in range(n):
        k = j * g % (2 * n)
        if k < n:
            out[k] += s[j]
        else:
            out[k - n] -= s[j]
    return out


def switch_key(params: Params, s: np.ndarray, s_from: np.ndarray, rng, err_mult: int = 1) -> np.ndarray:
    """Key switching key from ``s_from`` to ``s`` over Q_L u P, NTT domain,
    shape [dnum][2][L+k][N]:  evk_j = (-a_j s + err_mult e_j + P [i in D_j] s_from, a_j)
    (err_mult = t for BGV, 1 otherwise).

    [i in D_j] is 1 on the limbs of digit j and 0 on every other Q-limb (and the
    P term vanishes on the P-limbs), so one key serves every level."""
    qp = params.q + params.p
    P = product(params.p)
    s_hat = small_to_ntt(s, qp, params)
    sf_hat = small_to_ntt(s_from, qp, params)
    digits = params.digits(params.L)
    out = np.empty((len(digits), 2, len(qp), params.n), dtype=np.uint64)
    for j, dj in enumerate(digits):
        a = synthetic.uniform_residues(rng, qp, params.n)
        e = small_to_ntt(synthetic.gaussian(rng, params.n) * err_mult, qp, params)
        b = poly_add(poly_neg(poly_mul(a, s_hat, qp), qp), e, qp)
        for i in dj:
            q = params.q[i]
            b[i] = _core.add(b[i], _core.mul_scalar(sf_hat[i], P % q, q), q)
        out[j, 0] = b
        out[j, 1] = a
    return out


def relin_key(params: Params, s: np.ndarray, rng) -> np.ndarray:
    """Key from s^2 to s (relinearisation)."""
    return switch_key(params, s, negacyclic_square(s), rng)


def negacyclic_square(s: np.ndarray) -> np.ndarray:
    """s^2 mod (X^N + 1) over the integers: the full product folded with X^N = -1."""
    n = len(s)
    full = np.convolve(np.asarray(s, dtype=np.int64), np.asarray(s, dtype=np.int64))
    out = full[:n].copy()
    out[:n - 1] -= full[n:]
    return out


def galois_element(r: int, n: int) -> int:
    """g = 5^r mod 2N: rotates slots left by r."""
    return pow(5, r, 2 * n)


def galois_key(params: Params, s: np.ndarray, g: int, rng) -> np.ndarray:
    return switch_key(params, s, automorphism_coeffs(s, g), rng)


# ---------------------------------------------------------------- encryption

def encrypt(params: Params, s: np.ndarray, m: np.ndarray, nlimbs: int, scale: float,
            rng_a, rng_e) -> Ciphertext:
    """Secret-key encryption (c0, c1) = (-a s + e + m, a) over the first ``nlimbs`` Q-primes."""
    moduli = params.q[:nlimbs]
    a = synthetic.uniform_residues(rng_a, moduli, params.n)
    e = small_to_ntt(synthetic.gaussian(rng_e, params.n), moduli, params)
    mh = ntt_limbs(to_rns(m, moduli), moduli, params)
    sh = small_to_ntt(s, moduli, params)
    c0 = poly_add(poly_add(poly_neg(poly_mul(a, sh, moduli), moduli), e, moduli), mh, moduli)
    return Ciphertext(np.stack([c0, a]), float(scale))


def decrypt(params: Params, s: np.ndarray, ct: Ciphertext) -> np.ndarray:
    """Centred integer coefficients of c0 + c1 s mod Q_l."""
    moduli = params.q[:ct.nlimbs]
    sh = small_to_ntt(s, moduli, params)
    mh = poly_add(ct.data[0], poly_mul(ct.data[1], sh, moduli), moduli)
    m = intt_limbs(mh, moduli, params)
    return centered(crt(m, moduli), product(moduli))


def decrypt_decode(params: Params, s: np.ndarray, ct: Ciphertext) -> np.ndarray:
    return decode(decrypt(params, s, ct), ct.scale, params.n)


# ---------------------------------------------------------------- server ops

def tensor(a: Ciphertext, b: Ciphertext, params: Params):
    moduli = params.q[:a.nlimbs]
    a0, a1 = a.data
    b0, b1 = b.data
    d0 = poly_mul(a0, b0, moduli)
    d1 = poly_add(poly_mul(a0, b1, moduli), poly_mul(a1, b0, moduli), moduli)
    d2 = poly_mul(a1, b1, moduli)
    return d0, d1, d2


def ext_moduli(params: Params, nlimbs: int):
    """The basis Q_l u P of key switching: q_0..q_{nlimbs-1}, then p_0..p_{k-1}."""
    return params.q[:nlimbs] + params.p


def modup(d_ntt: np.ndarray, params: Params):
    """ModUp of every digit: list over digits j of [nlimbs + k][N] NTT-domain limbs.

    Limbs of digit j are copied; every other limb m of Q_l u P holds
    NTT( sum_{i in D_j} [x_i (Q_j/q_i)^-1]_{q_i} * (Q_j/q_i)  mod m ),  x = INTT(d)."""
    nl = d_ntt.shape[0]
    basis = ext_moduli(params, nl)
    x = intt_limbs(d_ntt, params.q[:nl], params)
    out = []
    for dj in params.digits(nl):
        qj = [params.q[i] for i in dj]
        Qj = product(qj)
        in_factor = [pow((Qj // q) % q, -1, q) for q in qj]
        targets = [m for m in range(len(basis)) if m not in dj]
        tmod = [basis[m] for m in targets]
        cross = [[(Qj // q) % t for t in tmod] for q in qj]
        conv = _core.bconv(x[dj], qj, in_factor, tmod, cross)
        ext = np.empty((len(basis), params.n), dtype=np.uint64)
        for i in dj:
            ext[i] = d_ntt[i]
        for r, m in enumerate(targets):
            ext[m] = ntt(conv[r], basis[m], params.psi(basis[m]))
        out.append(ext)
    return out


def key_limb(params: Params, nlimbs: int, m: int) -> int:
    """Index into the key's L+k limbs of limb m of Q_l u P."""
    return m if m < nlimbs else params.L + (m - nlimbs)


def inner_product(ext, evk: np.ndarray, params: Params, nlimbs: int) -> np.ndarray:
    """(sum_j ext_j * evk_{j,0}, sum_j ext_j * evk_{j,1}) on every limb of Q_l u P."""
    basis = ext_moduli(params, nlimbs)
    out = np.zeros((2, len(basis), params.n), dtype=np.uint64)
    for c in range(2):
        for m, q in enumerate(basis):
            km = key_limb(params, nlimbs, m)
            acc = np.zeros(params.n, dtype=np.uint64)
            for j, e in enumerate(ext):
                acc = _core.add(acc, _core.mul(e[m], evk[j, c, km], q), q)
            out[c, m] = acc
    return out


def moddown(y: np.ndarray, params: Params, nlimbs: int) -> np.ndarray:
    """Division by P with rounding of a [limbs of Q_l u P][N] NTT-domain polynomial:
    out_i = (y_i - NTT(conv_P->q_i(INTT(y_P)))) * P^-1 mod q_i, where the
    conversion uses centred digits y'_j in (-p_j/2, p_j/2], so that
    conv = [y]_P (centred) + u P with u symmetric about 0 and the result is
    round(y/P) - u: an error of mean zero."""
    qs = params.q[:nlimbs]
    ps = params.p
    P = product(ps)
    yp = intt_limbs(y[nlimbs:], ps, params)
    in_factor = [pow((P // p) % p, -1, p) for p in ps]
    cross = [[(P // p) % q for q in qs] for p in ps]
    conv = _core.bconv(yp, ps, in_factor, qs, cross, centred=True)
    out = np.empty((nlimbs, params.n), dtype=np.uint64)
    for i, q in enumerate(qs):
        ch = ntt(conv[i], q, params.psi(q))
        out[i] = _core.mul_scalar(_core.sub(y[i], ch, q), pow(P % q, -1, q), q)
    return out


def keyswitch(d_ntt: np.ndarray, evk: np.ndarray, params: Params, moddown_fn=None):
    nl = d_ntt.shape[0]
    md = moddown if moddown_fn is None else moddown_fn
    ext = modup(d_ntt, params)
    ip = inner_product(ext, evk, params, nl)
    return md(ip[0], params, nl), md(ip[1], params, nl)


def hmult_relin(a: Ciphertext, b: Ciphertext, rlk: np.ndarray, params: Params) -> Ciphertext:
    assert a.nlimbs == b.nlimbs
    moduli = params.q[:a.nlimbs]
    d0, d1, d2 = tensor(a, b, params)
    k0, k1 = keyswitch(d2, rlk, params)
    return Ciphertext(np.stack([poly_add(d0, k0, moduli), poly_add(d1, k1, moduli)]),
                      a.scale * b.scale)


def rescale(ct: Ciphertext, params: Params) -> Ciphertext:
    """Divide by the last prime q_l with rounding: c' = (c - [c]_{q_l}) * q_l^-1,
    [c]_{q_l} the centred residue, taken to every remaining q_i."""
    nl = ct.nlimbs
    assert nl >= 2
    ql = params.q[nl - 1]
    out = np.empty((2, nl - 1, params.n), dtype=np.uint64)
    for c in range(2):
        last = intt(ct.data[c, nl - 1], ql, params.psi(ql)).astype(object)
        r = np.where(last > ql // 2, last - ql, last)  # centred, |r| < q_l/2
        for i in range(nl - 1):
            q = params.q[i]
            rh = ntt((r % q).astype(np.uint64), q, params.psi(q))
            out[c, i] = _core.mul_scalar(_core.sub(ct.data[c, i], rh, q), pow(ql % q, -1, q), q)
    return Ciphertext(out, ct.scale / ql)


def modswitch_drop(ct: Ciphertext) -> Ciphertext:
    """CKKS modulus switch: drop the last limb (c mod Q_{l-1}); scale unchanged."""
    return Ciphertext(ct.data[:, :-1].copy(), ct.scale)


def automorphism_ntt(poly: np.ndarray, g: int, moduli, params: Params) -> np.ndarray:
    """sigma_g on NTT-domain limbs, by its definition on coefficients."""
    out = np.empty_like(poly)
    for i, q in enumerate(moduli):
        psi = params.psi(q)
        a = intt(poly[i], q, psi)
        out[i] = ntt(_core.automorphism_coeff(a, params.log_n, g, q), q, psi)
    return out


def rotate(ct: Ciphertext, g: int, gk: np.ndarray, params: Params) -> Ciphertext:
    """(sigma_g(c0) + KS_0(sigma_g(c1)), KS_1(sigma_g(c1))) with the key from s(X^g) to s."""
    moduli = params.q[:ct.nlimbs]
    c0 = automorphism_ntt(ct.data[0], g, moduli, params)
    c1 = automorphism_ntt(ct.data[1], g, moduli, params)
    k0, k1 = keyswitch(c1, gk, params)
    return Ciphertext(np.stack([poly_add(c0, k0, moduli), k1]), ct.scale)


# ---------------------------------------------------------------- element-wise helpers

def ct_add(a: Ciphertext, b: Ciphertext, params: Params) -> Ciphertext:
    moduli = params.q[:a.nlimbs]
    return Ciphertext(np.stack([poly_add(a.data[c], b.data[c], moduli) for c in range(2)]), a.scale)


def ct_sub(a: Ciphertext, b: Ciphertext, params: Params) -> Ciphertext:
    moduli = params.q[:a.nlimbs]
    return Ciphertext(np.stack([poly_sub(a.data[c], b.data[c], moduli) for c in range(2)]), a.scale)


def ct_mul_int(a: Ciphertext, k: int, params: Params) -> Ciphertext:
    """k * (c0, c1) for a signed integer k."""
    moduli = params.q[:a.nlimbs]
    return Ciphertext(np.stack([np.stack([_core.mul_scalar(a.data[c, i], k % q, q)
                                          for i, q in enumerate(moduli)]) for c in range(2)]), a.scale)


def ct_add_int(a: Ciphertext, k: int, params: Params) -> Ciphertext:
    """(c0 + k, c1): adds the constant polynomial k (every NTT-domain residue of c0)."""
    moduli = params.q[:a.nlimbs]
    c0 = np.stack([_core.add(a.data[0, i], np.full(params.n, k % q, dtype=np.uint64), q)
                   for i, q in enumerate(moduli)])
    return Ciphertext(np.stack([c0, a.data[1].copy()]), a.scale)


def ct_mul_plain(a: Ciphertext, pt: np.ndarray, params: Params) -> Ciphertext:
    moduli = params.q[:a.nlimbs]
    return Ciphertext(np.stack([poly_mul(a.data[c], pt[:a.nlimbs], moduli) for c in range(2)]), a.scale)
