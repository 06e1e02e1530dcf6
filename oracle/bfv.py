"""BFV over RNS limbs with BEHZ multiplication.  Test infrastructure only.

The paper's BFV multiply uses "the BEHZ algorithm" (section III, middle tier,
citing the GPU implementation of Al Badawi et al.); this module follows the
full-RNS BFV multiplication of Bajard, Eynard, Hasan and Zucca step by step.
Ciphertexts rest in the COEFFICIENT domain of Q = q_0 ... q_{L-1}; plaintexts
are in R_t with the slot encoding of the BGV module (t = 1 mod 2N).

    encrypt   (-a s + e + Delta m, a),  Delta = floor(Q / t)
    decrypt   m = round(t [c0 + c1 s]_Q / Q) mod t

Multiplication of (c0, c1) by (c0', c1'), with the auxiliary base
B = {b_j}, B_sk = B u {m_sk} and m~ = 2^32:
  1. each input polynomial x: fast base conversion of [m~ x]_q to B_sk u {m~}
     (no overflow correction), then the small Montgomery reduction by m~:
     r = [-x~_{m~} q^-1]_{m~} taken in (-m~/2, m~/2],
     x'_m = (x~_m + q r) m~^-1 mod m for m in B_sk;
  2. tensor (d0, d1, d2) = (c0 c0', c0 c1' + c1 c0', c1 c1') on q u B_sk
     (negacyclic products through the NTT of each prime);
  3. fast floor: for each d, in B_sk,
     f_m = (t d_m - conv_{q->B_sk}([t d]_q)_m) q^-1 mod m;
  4. Shenoy-Kumaresan conversion B_sk -> q:
     w_j = [f_j (M/b_j)^-1]_{b_j},  alpha = [(sum_j w_j [M/b_j]_{m_sk} - f_{m_sk}) M^-1]_{m_sk}
     taken in (-m_sk/2, m_sk/2],  out_i = sum_j w_j [M/b_j]_{q_i} - alpha M  mod q_i;
  5. relinearisation of d2 with the hybrid key switch (CKKS ModDown), in the
     NTT domain, then back to the coefficient domain.
"""
from __future__ import annotations

import numpy as np

import synthetic
from . import _core
from . import ckks as C
from .bgv import decode, encode  # slot encoding mod t is shared with BGV
from .ntt import intt, intt_limbs, ntt, ntt_limbs
from .params import Params
from .rns import centered, crt, product, to_rns

MTILDE = 1 << 32

__all__ = ["encode", "decode", "encrypt", "decrypt", "hmult_relin", "behz_tensor", "relin_key", "galois_key",
           "rotate"]


def qb_moduli(params: Params):
    """The extended basis q u B_sk: q_0..q_{L-1}, b_0..b_{n-1}, m_sk."""
    return params.q + params.b + [params.msk]


def encrypt(params: Params, s: np.ndarray, m: np.ndarray, rng_a, rng_e) -> np.ndarray:
    """[2][L][N] coefficient-domain ciphertext of the plaintext coefficients m (in [0, t))."""
    q = params.q
    Q = product(q)
    delta = Q // params.t
    a = synthetic.uniform_residues(rng_a, q, params.n)
    e = synthetic.gaussian(rng_e, params.n)
    s_ntt = C.small_to_ntt(s, q, params)
    as_ = intt_limbs(C.poly_mul(ntt_limbs(a, q, params), s_ntt, q), q, params)
    dm = np.array([int(x) * delta for x in m], dtype=object)
    c0 = C.poly_add(C.poly_neg(as_, q), to_rns(np.asarray(e, dtype=object) + dm, q), q)
    return np.stack([c0, a])


def phase(params: Params, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """[c0 + c1 s]_Q, centred, as Python integers."""
    q = params.q
    s_ntt = C.small_to_ntt(s, q, params)
    c1s = intt_limbs(C.poly_mul(ntt_limbs(ct[1], q, params), s_ntt, q), q, params)
    v = C.poly_add(ct[0], c1s, q)
    return centered(crt(v, q), product(q))


def decrypt(params: Params, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """Slots of round(t [c0 + c1 s]_Q / Q) mod t."""
    Q = product(params.q)
    t = params.t
    x = phase(params, s, ct)
    m = np.array([((2 * t * int(v) + Q) // (2 * Q)) % t for v in x], dtype=object)
    return decode(m, params)


def noise_bits(params: Params, s: np.ndarray, ct: np.ndarray, m_coeffs) -> float:
    """log2 of max |[c0 + c1 s - Delta m]_Q| (centred)."""
    Q = product(params.q)
    delta = Q // params.t
    x = phase(params, s, ct)
    diff = np.array([int(v) - delta * int(mm) for v, mm in zip(x, m_coeffs)], dtype=object)
    worst = max(abs(int(v)) for v in centered(diff, Q))
    return float(np.log2(worst + 1))


def _extend(x: np.ndarray, params: Params) -> np.ndarray:
    """Step 1 for one polynomial x [L][N] (coefficient domain) -> its B_sk limbs [n_b + 1][N]."""
    q = params.q
    Q = product(q)
    bsk = params.b + [params.msk]
    targets = bsk + [MTILDE]
    in_factor = [MTILDE * pow((Q // qi) % qi, -1, qi) % qi for qi in q]
    cross = [[(Q // qi) % m for m in targets] for qi in q]
    conv = _core.bconv(x, q, in_factor, targets, cross)
    xm = conv[-1].astype(object)
    r = (-xm * pow(Q, -1, MTILDE)) % MTILDE
    r = np.where(r >= MTILDE // 2, r - MTILDE, r)  # centred
    out = np.empty((len(bsk), params.n), dtype=np.uint64)
    for k, m in enumerate(bsk):
        v = (conv[k].astype(object) + (Q % m) * r) % m
        out[k] = ((v * pow(MTILDE, -1, m)) % m).astype(np.uint64)
    return out


def _floor_sk(d: np.ndarray, params: Params) -> np.ndarray:
    """Steps 3 and 4 for one polynomial d [L + n_b + 1][N] on q u B_sk -> [L][N] on q."""
    q = params.q
    L = len(q)
    Q = product(q)
    t = params.t
    B = params.b
    bsk = B + [params.msk]
    M = product(B)
    dq = d[:L]
    dbsk = d[L:]
    # fast floor: f = (t d_Bsk - conv([t d]_q)) q^-1 in B_sk
    in_factor = [t * pow((Q // qi) % qi, -1, qi) % qi for qi in q]
    cross = [[(Q // qi) % m for m in bsk] for qi in q]
    conv = _core.bconv(dq, q, in_factor, bsk, cross)
    f = np.empty_like(dbsk)
    for k, m in enumerate(bsk):
        v = (t * dbsk[k].astype(object) - conv[k].astype(object)) % m
        f[k] = ((v * pow(Q % m, -1, m)) % m).astype(np.uint64)
    # Shenoy-Kumaresan: B_sk -> q
    in_b = [pow((M // b) % b, -1, b) for b in B]
    to = q + [params.msk]
    cross_b = [[(M // b) % m for m in to] for b in B]
    conv_b = _core.bconv(f[:len(B)], B, in_b, to, cross_b)
    msk = params.msk
    alpha = ((conv_b[-1].astype(object) - f[-1].astype(object)) * pow(M % msk, -1, msk)) % msk
    alpha = np.where(alpha > msk // 2, alpha - msk, alpha)
    out = np.empty((L, params.n), dtype=np.uint64)
    for i, qi in enumerate(q):
        out[i] = ((conv_b[i].astype(object) - alpha * (M % qi)) % qi).astype(np.uint64)
    return out


def behz_tensor(a: np.ndarray, b: np.ndarray, params: Params):
    """(d0, d1, d2) on q (coefficient domain) ~ round-down of t (a x b) / Q."""
    qb = qb_moduli(params)
    ext = []
    for x in (a[0], a[1], b[0], b[1]):
        full = np.concatenate([x, _extend(x, params)])
        ext.append(ntt_limbs(full, qb, params))
    a0, a1, b0, b1 = ext
    d0 = C.poly_mul(a0, b0, qb)
    d1 = C.poly_add(C.poly_mul(a0, b1, qb), C.poly_mul(a1, b0, qb), qb)
    d2 = C.poly_mul(a1, b1, qb)
    return tuple(_floor_sk(intt_limbs(d, qb, params), params) for d in (d0, d1, d2))


def relin_key(params: Params, s: np.ndarray, rng) -> np.ndarray:
    return C.switch_key(params, s, C.negacyclic_square(s), rng)


def hmult_relin(a: np.ndarray, b: np.ndarray, rlk: np.ndarray, params: Params) -> np.ndarray:
    q = params.q
    d0, d1, d2 = behz_tensor(a, b, params)
    k0, k1 = C.keyswitch(ntt_limbs(d2, q, params), rlk, params)
    return np.stack([C.poly_add(d0, intt_limbs(k0, q, params), q),
                     C.poly_add(d1, intt_limbs(k1, q, params), q)])


def galois_key(params: Params, s: np.ndarray, g: int, rng) -> np.ndarray:
    """Key switching key from s(X^g) to s (the hybrid key of the relinearisation)."""
    return C.galois_key(params, s, g, rng)


def rotate(ct: np.ndarray, g: int, gk: np.ndarray, params: Params) -> np.ndarray:
    """Galois automorphism sigma_g: a(X) -> a(X^g) of both coefficient-domain
    polynomials (X^(g j) reduced mod X^N + 1), then the key switch of
    sigma_g(c1) from s(X^g) back to s, in the NTT domain as in the
    relinearisation: (sigma_g(c0) + KS_0, KS_1).  Decrypts to m(X^g) mod t,
    which permutes the slots."""
    q = params.q
    c0 = np.stack([_core.automorphism_coeff(ct[0, i], params.log_n, g, q[i]) for i in range(len(q))])
    c1 = np.stack([_core.automorphism_coeff(ct[1, i], params.log_n, g, q[i]) for i in range(len(q))])
    k0, k1 = C.keyswitch(ntt_limbs(c1, q, params), gk, params)
    return np.stack([C.poly_add(c0, intt_limbs(k0, q, params), q), intt_limbs(k1, q, params)])
