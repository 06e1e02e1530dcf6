"""Pins of the oracle's parameters, NTT and CRT against independent mathematics.

* primes: sympy's primality test (an implementation other than the oracle's
  Miller-Rabin), the congruence q = 1 mod 2N, bit sizes and distinctness;
* roots: psi has multiplicative order exactly 2N;
* NTT: the fast transform equals the O(N^2) evaluation at psi^(2 brv(i) + 1),
  and INTT(NTT(a) * NTT(b)) equals the schoolbook negacyclic product;
* CRT: big-integer round trips.
"""
import math

import numpy as np
import pytest
import sympy

import synthetic
from oracle import ntt as T
from oracle import params as P
from oracle import rns


@pytest.mark.parametrize("name", list(synthetic.WORKLOADS))
def test_prime_chains(name):
    w = synthetic.WORKLOADS[name]
    p = P.make_params(w)
    modulus = 2 << w["log_nmax"]
    allp = p.q + p.p + p.b + ([p.msk] if p.msk else [])
    assert len(set(allp)) == len(allp)
    for q in allp:
        assert sympy.isprime(q)
        assert q % modulus == 1
    for q, b in zip(p.q, w["q_bits"]):
        assert q.bit_length() == b
    for q, b in zip(p.p, w["p_bits"]):
        assert q.bit_length() == b
    # no larger unused prime of the same size class is skipped in a group
    same = [q for q, b in zip(p.q, w["q_bits"]) if b == w["q_bits"][-1]]
    assert same == sorted(same, reverse=True)


def test_chain_sizes_n16():
    p = P.make_params(synthetic.WORKLOADS["ckks_n16_l24"])
    assert round(sum(math.log2(q) for q in p.q), 1) == 1095.0
    assert round(sum(math.log2(q) for q in p.q + p.p), 1) == 1335.0
    assert p.dnum() == 3 and p.L == 24 and p.k == 4


def test_paper_setup_ciphertext_size():
    """The paper's setup: N=32768, L=16 limbs, 64-bit words -> about 8 MB per ciphertext."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_setup.json")))
    size = 2 * g["L"] * g["N"] * 8
    assert size == g["ciphertext_bytes"]


@pytest.mark.parametrize("name", ["ckks_n12", "ckks_n16_l24", "bfv_n15"])
def test_root_order(name):
    p = P.make_params(synthetic.WORKLOADS[name])
    for q in (p.q + p.p)[:6]:
        psi = p.psi(q)
        n = p.n
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1
        # order exactly 2N: psi^(2N/r) != 1 for the only prime factor r = 2
        assert pow(psi, n, q) != 1


def test_root_strided_across_degrees():
    p16 = P.make_params(synthetic.WORKLOADS["ckks_batch"])
    for log_n in (14, 15):
        pn = p16.at_degree(log_n)
        for q in p16.q[:3]:
            assert pn.psi(q) == pow(p16.psi(q), 1 << (16 - log_n), q)


def _small_params(log_n):
    w = dict(synthetic.WORKLOADS["ckks_n16_l24"])
    return P.make_params(w).at_degree(log_n)


@pytest.mark.parametrize("log_n", [2, 3, 5, 7, 8])
def test_ntt_equals_definition(log_n):
    p = _small_params(log_n)
    rng = np.random.default_rng(log_n)
    for q in (p.q[0], p.q[5], p.p[1]):
        psi = p.psi(q)
        a = rng.integers(0, q, p.n, dtype=np.uint64)
        fast = T.ntt(a, q, psi)
        assert [int(x) for x in fast] == T.ntt_definition(a, q, psi)
        assert [int(x) for x in T.intt(fast, q, psi)] == [int(x) for x in a]
        assert T.intt_definition(T.ntt_definition(a, q, psi), q, psi) == [int(x) for x in a]


def test_ntt_equals_definition_1024():
    p = _small_params(10)
    q = p.q[1]
    psi = p.psi(q)
    a = np.random.default_rng(7).integers(0, q, p.n, dtype=np.uint64)
    assert [int(x) for x in T.ntt(a, q, psi)] == T.ntt_definition(a, q, psi)


@pytest.mark.parametrize("log_n", [2, 4, 6, 8])
def test_ntt_negacyclic_product(log_n):
    p = _small_params(log_n)
    rng = np.random.default_rng(100 + log_n)
    for q in (p.q[0], p.q[3], p.p[0]):
        psi = p.psi(q)
        a = rng.integers(0, q, p.n, dtype=np.uint64)
        b = rng.integers(0, q, p.n, dtype=np.uint64)
        from oracle import _core
        prod = T.intt(_core.mul(T.ntt(a, q, psi), T.ntt(b, q, psi), q), q, psi)
        assert [int(x) for x in prod] == T.negacyclic_schoolbook(a, b, q)


def test_ntt_linearity_and_inverse_large():
    p = P.make_params(synthetic.WORKLOADS["ckks_n16_l24"])
    q = p.q[7]
    psi = p.psi(q)
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, p.n, dtype=np.uint64)
    b = rng.integers(0, q, p.n, dtype=np.uint64)
    from oracle import _core
    lhs = T.ntt(_core.add(a, b, q), q, psi)
    rhs = _core.add(T.ntt(a, q, psi), T.ntt(b, q, psi), q)
    assert np.array_equal(lhs, rhs)
    assert np.array_equal(T.intt(T.ntt(a, q, psi), q, psi), a)
    # a few outputs by the direct sum at N = 2^16
    ah = T.ntt(a, q, psi)
    for i in (0, 1, 12345, p.n - 1):
        w = pow(psi, 2 * P.bitrev(i, p.log_n) + 1, q)
        acc = 0
        wj = 1
        for j in range(p.n):
            acc += int(a[j]) * wj
            wj = wj * w % q
        assert acc % q == int(ah[i])


def test_crt_round_trip():
    p = P.make_params(synthetic.WORKLOADS["ckks_n16_l24"])
    moduli = p.q + p.p
    Q = rns.product(moduli)
    rng = np.random.default_rng(11)
    xs = [int(rng.integers(0, 2**62)) * int(rng.integers(0, 2**62)) ** 20 % Q for _ in range(16)]
    xs += [0, 1, Q - 1, Q // 2, Q // 2 + 1]
    limbs = rns.to_rns(np.array(xs, dtype=object), moduli)
    back = rns.crt(limbs, moduli)
    assert [int(v) for v in back] == xs
    c = rns.centered(np.array(xs, dtype=object), Q)
    for x, y in zip(xs, c):
        assert -Q // 2 < y <= Q // 2 and (x - y) % Q == 0
