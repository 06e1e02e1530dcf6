"""Pins of the oracle's BGV operations.

* slots: encode/decode round trip, and the slot-wise product equals the
  schoolbook negacyclic product mod t (so slots are the evaluations);
* ModDown (t-preserving): out P = y - delta with delta = 0 mod t, delta = y mod P,
  |delta| <= t P (k/2 + 1), checked per coefficient with big integers;
* modulus switch: c' q_l = c - delta, delta = 0 mod t, delta = c mod q_l,
  |delta| <= t q_l / 2;
* end to end: decryptions equal the plaintext slot products exactly, across
  a modulus switch and a second multiplication, and rotations permute slots.
"""
import numpy as np
import pytest

import synthetic
from oracle import bgv as B
from oracle import ckks as C
from oracle import ntt as T
from oracle import params as P
from oracle import rns


def small_bgv(log_n=5, nq=4, nk=1):
    w = dict(synthetic.WORKLOADS["bgv_n15"])
    w.update(q_bits=[55] * nq, p_bits=[60] * nk)
    return P.make_params(w).at_degree(log_n)


def test_slots_are_evaluations():
    p = small_bgv(log_n=5)
    rng = np.random.default_rng(1)
    z1 = synthetic.integer_slots(rng, p.n, p.t)
    z2 = synthetic.integer_slots(rng, p.n, p.t)
    m1, m2 = B.encode(z1, p), B.encode(z2, p)
    assert np.array_equal(B.decode(m1, p), z1)
    prod = T.negacyclic_schoolbook(m1, m2, p.t)
    assert np.array_equal(B.decode(np.array(prod, dtype=object), p), z1 * z2 % p.t)


@pytest.mark.parametrize("nk", [1, 2])
def test_moddown_keeps_t(nk):
    p = small_bgv(nk=nk)
    nl = 3
    basis = C.ext_moduli(p, nl)
    rng = np.random.default_rng(nk)
    y = synthetic.uniform_residues(rng, basis, p.n)
    out = B.moddown(y, p, nl)
    Pm = rns.product(p.p)
    Ql = rns.product(p.q[:nl])
    Y = rns.crt(T.intt_limbs(y, basis, p), basis)
    O = rns.crt(T.intt_limbs(out, p.q[:nl], p), p.q[:nl])
    for c in range(p.n):
        delta = (int(Y[c]) - int(O[c]) * Pm) % (Ql * Pm)
        if delta > Ql * Pm // 2:
            delta -= Ql * Pm
        assert delta % p.t == 0
        assert (delta - int(Y[c])) % Pm == 0
        assert abs(delta) <= p.t * Pm * (nk / 2 + 1)


def test_modswitch_keeps_t():
    p = small_bgv()
    nl = 4
    rng = np.random.default_rng(3)
    data = np.stack([synthetic.uniform_residues(rng, p.q[:nl], p.n) for _ in range(2)])
    out = B.modswitch(B.Ciphertext(data, 1), p)
    ql = p.q[nl - 1]
    Qn = rns.product(p.q[:nl - 1])
    assert out.factor == pow(ql, -1, p.t)
    for c in range(2):
        X = rns.crt(T.intt_limbs(data[c], p.q[:nl], p), p.q[:nl])
        Y = rns.crt(T.intt_limbs(out.data[c], p.q[:nl - 1], p), p.q[:nl - 1])
        for x, y in zip(X, Y):
            delta = (int(x) - int(y) * ql) % (Qn * ql)
            if delta > Qn * ql // 2:
                delta -= Qn * ql
            assert delta % p.t == 0 and (int(x) - delta) % ql == 0
            assert abs(delta) <= p.t * ql // 2


def _client(log_n):
    w = dict(synthetic.WORKLOADS["bgv_n15"])
    w["log_n"] = log_n
    p = P.make_params(w)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    z1 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    z2 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    a = B.encrypt(p, s, B.encode(z1, p), p.L, st["ct_a"], st["ct_e"])
    b = B.encrypt(p, s, B.encode(z2, p), p.L, st["ct_a"], st["ct_e"])
    return p, st, s, z1, z2, a, b


@pytest.mark.parametrize("log_n", [12, pytest.param(15, marks=pytest.mark.slow)])
def test_e2e_exact_slots(log_n):
    p, st, s, z1, z2, a, b = _client(log_n)
    rlk = B.relin_key(p, s, st["rlk"])
    assert np.array_equal(B.decrypt(p, s, a), z1)
    c = B.hmult_relin(a, b, rlk, p)
    z12 = z1 * z2 % p.t
    assert np.array_equal(B.decrypt(p, s, c), z12)
    d = B.modswitch(c, p)
    assert np.array_equal(B.decrypt(p, s, d), z12)
    e = B.hmult_relin(d, d, rlk, p)
    assert np.array_equal(B.decrypt(p, s, e), z12 * z12 % p.t)
    g = C.galois_element(3, p.n)
    gk = B.galois_key(p, s, g, st["galois"])
    r = B.rotate(a, g, gk, p)
    perm = [P.bitrev(((2 * P.bitrev(k, p.log_n) + 1) * g % (2 * p.n) - 1) // 2, p.log_n) for k in range(p.n)]
    assert np.array_equal(B.decrypt(p, s, r), z1[perm])
