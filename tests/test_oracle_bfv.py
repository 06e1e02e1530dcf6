"""Pins of the oracle's BFV with BEHZ multiplication.

* step 1 (extension to B_sk with the small Montgomery reduction) gives a
  representative of the input mod Q: CRT over B_sk (centred) is X or X - Q,
  X the CRT over q in [0, Q);
* steps 2-4 against big-integer arithmetic: on N=32 the BEHZ tensor equals
  floor(t (a' x b') / Q) mod Q, a' and b' those representatives and the
  products schoolbook over Z, up to an error in [-(L+1), 1] per coefficient;
* end to end: exact slot products through two multiplications;
* rotation: the rotated ciphertext decrypts to the plaintext polynomial with
  X -> X^g applied (mod X^N + 1, mod t), for rotation elements and the
  conjugation.
"""
import numpy as np
import pytest

import synthetic
from oracle import bfv as F
from oracle import ckks as C
from oracle import params as P
from oracle import rns


def small_bfv(log_n=5, nq=4, nb=5):
    w = dict(synthetic.WORKLOADS["bfv_n15"])
    w.update(q_bits=[55] * nq, b_bits=[60] * nb)
    return P.make_params(w).at_degree(log_n)


def test_extension_is_exact():
    p = small_bfv()
    rng = np.random.default_rng(2)
    x = synthetic.uniform_residues(rng, p.q, p.n)
    ext = F._extend(x, p)
    bsk = p.b + [p.msk]
    Q = rns.product(p.q)
    xs = rns.centered(rns.crt(ext, bsk), rns.product(bsk))
    for v, X in zip(xs, rns.crt(x, p.q)):
        assert int(v) in (int(X), int(X) - Q)


def test_behz_tensor_against_big_integers():
    p = small_bfv()
    rng = np.random.default_rng(3)
    a = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
    b = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
    Q = rns.product(p.q)
    bsk = p.b + [p.msk]
    Msk = rns.product(bsk)

    def rep(x):  # the representative the extension carries into B_sk
        return [int(v) for v in rns.centered(rns.crt(F._extend(x, p), bsk), Msk)]

    A = [rep(a[c]) for c in range(2)]
    Bv = [rep(b[c]) for c in range(2)]

    def conv(x, y):  # negacyclic product over Z
        n = len(x)
        out = [0] * n
        for i in range(n):
            for j in range(n):
                k = i + j
                if k < n:
                    out[k] += x[i] * y[j]
                else:
                    out[k - n] -= x[i] * y[j]
        return out

    exact = [conv(A[0], Bv[0]), [u + v for u, v in zip(conv(A[0], Bv[1]), conv(A[1], Bv[0]))],
             conv(A[1], Bv[1])]
    got = F.behz_tensor(a, b, p)
    for d, e in zip(got, exact):
        D = [int(v) for v in rns.crt(d, p.q)]
        for x, y in zip(D, e):
            diff = (x - (p.t * y) // Q) % Q
            diff = diff - Q if diff > Q // 2 else diff
            assert -(p.L + 1) <= diff <= 1


@pytest.mark.parametrize("log_n", [12, pytest.param(15, marks=pytest.mark.slow)])
def test_e2e_exact_slots(log_n):
    w = synthetic.WORKLOADS["bfv_n15"]
    p = P.make_params(w).at_degree(log_n)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    rlk = F.relin_key(p, s, st["rlk"])
    z1 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    z2 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    a = F.encrypt(p, s, F.encode(z1, p), st["ct_a"], st["ct_e"])
    b = F.encrypt(p, s, F.encode(z2, p), st["ct_a"], st["ct_e"])
    assert np.array_equal(F.decrypt(p, s, a), z1)
    c = F.hmult_relin(a, b, rlk, p)
    z12 = z1 * z2 % p.t
    assert np.array_equal(F.decrypt(p, s, c), z12)
    e = F.hmult_relin(c, c, rlk, p)
    assert np.array_equal(F.decrypt(p, s, e), z12 * z12 % p.t)


@pytest.mark.parametrize("g", [5, 25, 3, 63])
def test_rotation_decrypts_to_the_automorphism(g):
    p = small_bfv()
    assert g < 2 * p.n and g % 2 == 1
    rng = np.random.default_rng(40 + g)
    s = C.secret_key(p, rng)
    m = rng.integers(0, p.t, p.n)
    ct = F.encrypt(p, s, m, rng, rng)
    rot = F.rotate(ct, g, F.galois_key(p, s, g, rng), p)
    m_g = np.mod(C.automorphism_coeffs(np.asarray(m, dtype=np.int64), g), p.t)
    assert np.array_equal(F.decrypt(p, s, rot), F.decode(m_g, p))
    assert not np.array_equal(F.decrypt(p, s, rot), F.decrypt(p, s, ct))
