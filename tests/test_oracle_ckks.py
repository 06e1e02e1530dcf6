"""Pins of the oracle's CKKS operations against big-integer arithmetic and closed forms.

Each pin is chosen so a plausible slip (a dropped product, a wrong sign, a
transposed index, a wrong digit boundary) fails it:

* encode/decode: the FFT form equals the O(N^2) sums over the roots;
* tensor: coefficient-domain schoolbook products of the two ciphertexts;
* ModUp: over Q_l u P, CRT(out) = X + u Q_j with X = CRT of the digit, 0 <= u < alpha;
* ModDown: out = (Y - [Y]_P - u P) / P exactly, |u| <= k/2 + 1;
* rescale: CRT(out) = round(CRT_centred(c) / q_l) for every coefficient;
* keys: evk_j0 + evk_j1 s - P [i in D_j] s' is a small error on every limb;
* automorphism: group law, and the NTT-domain permutation derived from the
  evaluation points;
* end to end: decryptions agree with the plaintext computation.
"""
import numpy as np
import pytest

import synthetic
from oracle import _core
from oracle import ckks as C
from oracle import ntt as T
from oracle import params as P
from oracle import rns


def small_ckks(log_n=6, alpha=2, nq=5, nk=2):
    w = dict(synthetic.WORKLOADS["ckks_n16_l24"])
    w.update(q_bits=[60] + [45] * (nq - 1), p_bits=[60] * nk, alpha=alpha)
    return P.make_params(w).at_degree(log_n)


def coeff(poly, moduli, params):
    return T.intt_limbs(poly, moduli, params)


@pytest.mark.parametrize("log_n", [3, 5, 7])
def test_encode_decode_against_direct_sums(log_n):
    n = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = synthetic.complex_slots(rng, n // 2)
    scale = 2.0 ** 30
    m = C.encode(z, scale, n)
    md = C.encode_direct(z, scale, n)
    assert max(abs(int(a) - int(b)) for a, b in zip(m, md)) <= 1
    zd = C.decode_direct(m, scale, n)
    assert np.abs(C.decode(m, scale, n) - zd).max() < 1e-9
    assert np.abs(zd - z).max() < 2.0 ** -20


def test_encode_decode_round_trip_n16():
    n = 1 << 16
    z = synthetic.complex_slots(np.random.default_rng(5), n // 2)
    m = C.encode(z, 2.0 ** 40, n)
    assert np.abs(C.decode(m, 2.0 ** 40, n) - z).max() < 2.0 ** -30


def test_tensor_schoolbook():
    p = small_ckks(log_n=5)
    st = synthetic.streams(1)
    moduli = p.q
    a = C.Ciphertext(synthetic.uniform_residues(st["ct_a"], moduli, p.n)[None].repeat(2, 0), 1.0)
    a.data[1] = synthetic.uniform_residues(st["ct_a"], moduli, p.n)
    b = C.Ciphertext(synthetic.uniform_residues(st["ct_e"], moduli, p.n)[None].repeat(2, 0), 1.0)
    b.data[1] = synthetic.uniform_residues(st["ct_e"], moduli, p.n)
    d0, d1, d2 = C.tensor(a, b, p)
    for i, q in enumerate(moduli):
        ac = [coeff(a.data[c], moduli, p)[i] for c in range(2)]
        bc = [coeff(b.data[c], moduli, p)[i] for c in range(2)]
        sb = T.negacyclic_schoolbook
        assert [int(x) for x in coeff(d0, moduli, p)[i]] == sb(ac[0], bc[0], q)
        s01 = [(x + y) % q for x, y in zip(sb(ac[0], bc[1], q), sb(ac[1], bc[0], q))]
        assert [int(x) for x in coeff(d1, moduli, p)[i]] == s01
        assert [int(x) for x in coeff(d2, moduli, p)[i]] == sb(ac[1], bc[1], q)


def test_mul_plain_schoolbook():
    """ct_mul_plain: each polynomial of the ciphertext times the plaintext, checked in the
    coefficient domain against the schoolbook negacyclic product (on a truncated level,
    so the plaintext's extra limbs must be ignored); ct_mul_int and ct_add_int against
    their integer definitions."""
    p = small_ckks(log_n=5)
    st = synthetic.streams(2)
    nl = 3
    moduli = p.q[:nl]
    ct = C.Ciphertext(np.stack([synthetic.uniform_residues(st["ct_a"], moduli, p.n) for _ in range(2)]), 1.0)
    pt = synthetic.uniform_residues(st["ct_e"], p.q, p.n)
    out = C.ct_mul_plain(ct, pt, p)
    assert out.data.shape == ct.data.shape
    for c in range(2):
        for i, q in enumerate(moduli):
            want = T.negacyclic_schoolbook(coeff(ct.data[c], moduli, p)[i], coeff(pt[:nl], moduli, p)[i], q)
            assert [int(x) for x in coeff(out.data[c], moduli, p)[i]] == want, (c, i)
    k = -(1 << 61) - 3
    mi = C.ct_mul_int(ct, k, p)
    ai = C.ct_add_int(ct, k, p)
    for c in range(2):
        for i, q in enumerate(moduli):
            assert [int(x) for x in mi.data[c, i]] == [int(x) * k % q for x in ct.data[c, i]]
            # adding the constant polynomial k: k on the constant coefficient only
            want = [int(x) for x in coeff(ct.data[c], moduli, p)[i]]
            if c == 0:
                want[0] = (want[0] + k) % q
            assert [int(x) for x in coeff(ai.data[c], moduli, p)[i]] == want


@pytest.mark.parametrize("alpha,nlimbs", [(2, 5), (2, 4), (3, 5), (1, 3), (5, 5)])
def test_modup_invariant(alpha, nlimbs):
    p = small_ckks(log_n=5, alpha=alpha)
    rng = np.random.default_rng(alpha * 10 + nlimbs)
    d = synthetic.uniform_residues(rng, p.q[:nlimbs], p.n)
    ext = C.modup(d, p)
    basis = C.ext_moduli(p, nlimbs)
    xc = rns.crt(coeff(d, p.q[:nlimbs], p), p.q[:nlimbs])
    digits = p.digits(nlimbs)
    assert len(ext) == len(digits)
    for dj, e in zip(digits, ext):
        qj = [p.q[i] for i in dj]
        Qj = rns.product(qj)
        # the digit's limbs are copies of the input
        for i in dj:
            assert np.array_equal(e[i], d[i])
        X = rns.crt(coeff(d[dj], qj, p), qj)
        full = rns.crt(coeff(e, basis, p), basis)
        for c in range(p.n):
            diff = int(full[c]) - int(X[c])
            assert diff % Qj == 0
            u = diff // Qj
            assert 0 <= u < len(dj)
            assert X[c] % p.q[dj[0]] == xc[c] % p.q[dj[0]]


@pytest.mark.parametrize("nk", [1, 2, 4])
def test_moddown_invariant(nk):
    p = small_ckks(log_n=5, nk=nk)
    nl = 4
    basis = C.ext_moduli(p, nl)
    rng = np.random.default_rng(nk)
    y = synthetic.uniform_residues(rng, basis, p.n)
    out = C.moddown(y, p, nl)
    Pm = rns.product(p.p)
    Ql = rns.product(p.q[:nl])
    Y = rns.crt(coeff(y, basis, p), basis)
    O = rns.crt(coeff(out, p.q[:nl], p), p.q[:nl])
    for c in range(p.n):
        yc = int(Y[c])
        yp = yc % Pm
        if yp > Pm // 2:
            yp -= Pm  # centred residue mod P
        # out * P = Y - [Y]_P - u P  (mod Q_l P), u small and symmetric
        r = (int(O[c]) * Pm - (yc - yp)) % (Ql * Pm)
        if r > Ql * Pm // 2:
            r -= Ql * Pm
        assert r % Pm == 0
        u = -r // Pm
        assert abs(u) <= nk // 2 + 1


@pytest.mark.parametrize("nl", [2, 3, 5])
def test_rescale_exact(nl):
    p = small_ckks(log_n=5)
    rng = np.random.default_rng(nl)
    data = np.stack([synthetic.uniform_residues(rng, p.q[:nl], p.n) for _ in range(2)])
    ct = C.Ciphertext(data, 2.0 ** 40)
    out = C.rescale(ct, p)
    ql = p.q[nl - 1]
    assert out.nlimbs == nl - 1
    assert out.scale == 2.0 ** 40 / ql
    for c in range(2):
        X = rns.centered(rns.crt(coeff(data[c], p.q[:nl], p), p.q[:nl]), rns.product(p.q[:nl]))
        Y = rns.crt(coeff(out.data[c], p.q[:nl - 1], p), p.q[:nl - 1])
        Qn = rns.product(p.q[:nl - 1])
        for x, y in zip(X, Y):
            x = int(x)
            # round to nearest (q_l odd: no ties)
            rounded = (2 * x + ql) // (2 * ql)
            assert rounded % Qn == int(y)


def test_switch_key_identity():
    p = small_ckks(log_n=5, alpha=2)
    st = synthetic.streams(3)
    s = C.secret_key(p, st["sk"])
    s2 = C.negacyclic_square(s)
    big = 2 ** 127 - 1  # prime, far above any coefficient of s^2
    sl = [int(x) % big for x in s]
    sb = T.negacyclic_schoolbook(sl, sl, big)
    assert [int(x) for x in s2] == [x if x <= big // 2 else x - big for x in sb]
    evk = C.relin_key(p, s, st["rlk"])
    qp = p.q + p.p
    Pm = rns.product(p.p)
    sh = C.small_to_ntt(s, qp, p)
    s2h = C.small_to_ntt(s2, qp, p)
    for j, dj in enumerate(p.digits(p.L)):
        for i, q in enumerate(qp):
            v = _core.add(evk[j, 0, i], _core.mul(evk[j, 1, i], sh[i], q), q)
            if i in dj:
                v = _core.sub(v, _core.mul_scalar(s2h[i], Pm % q, q), q)
            e = T.intt(v, q, p.psi(q))
            ec = [int(x) if int(x) <= q // 2 else int(x) - q for x in e]
            assert max(abs(x) for x in ec) <= synthetic.ERROR_BOUND


def test_automorphism_group_law_and_permutation():
    p = small_ckks(log_n=6)
    n = p.n
    q = p.q[2]
    psi = p.psi(q)
    rng = np.random.default_rng(9)
    a = synthetic.uniform_residues(rng, [q], n)
    g1, g2 = C.galois_element(3, n), C.galois_element(7, n)
    s1 = C.automorphism_ntt(C.automorphism_ntt(a, g2, [q], p), g1, [q], p)
    s12 = C.automorphism_ntt(a, g1 * g2 % (2 * n), [q], p)
    assert np.array_equal(s1, s12)
    # NTT-domain permutation: out[k] = in[k'] with 2 brv(k') + 1 = (2 brv(k) + 1) g mod 2N
    for g in (g1, 2 * n - 1):
        out = C.automorphism_ntt(a, g, [q], p)[0]
        for k in range(n):
            e = (2 * P.bitrev(k, p.log_n) + 1) * g % (2 * n)
            kp = P.bitrev((e - 1) // 2, p.log_n)
            assert out[k] == a[0, kp]
    del psi


def _e2e(name, alpha=None, rot=None):
    w = dict(synthetic.WORKLOADS[name])
    if alpha:
        w["alpha"] = alpha
    p = P.make_params(w)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    rlk = C.relin_key(p, s, st["rlk"])
    n = p.n
    D = 2.0 ** w["log_scale"]
    z1 = synthetic.complex_slots(st["msgs"], n // 2)
    z2 = synthetic.complex_slots(st["msgs"], n // 2)
    a = C.encrypt(p, s, C.encode(z1, D, n), p.L, D, st["ct_a"], st["ct_e"])
    b = C.encrypt(p, s, C.encode(z2, D, n), p.L, D, st["ct_a"], st["ct_e"])
    out = {}
    out["fresh"] = np.abs(C.decrypt_decode(p, s, a) - z1).max()
    c = C.hmult_relin(a, b, rlk, p)
    out["mult"] = np.abs(C.decrypt_decode(p, s, c) - z1 * z2).max()
    r = C.rescale(c, p)
    out["rescale"] = np.abs(C.decrypt_decode(p, s, r) - z1 * z2).max()
    out["rescale_scale"] = r.scale
    rot = rot if rot is not None else synthetic.rotation_index(st["rot"], n)
    g = C.galois_element(rot, n)
    gk = C.galois_key(p, s, g, st["galois"])
    rr = C.rotate(a, g, gk, p)
    out["rotate"] = np.abs(C.decrypt_decode(p, s, rr) - np.roll(z1, -rot)).max()
    conj = C.rotate(a, 2 * n - 1, C.galois_key(p, s, 2 * n - 1, st["galois"]), p)
    out["conjugate"] = np.abs(C.decrypt_decode(p, s, conj) - np.conj(z1)).max()
    return out


def test_e2e_n12():
    """The N=2^12 chain (q0 60-bit, q1 40-bit, one 60-bit special prime, dnum=2)."""
    e = _e2e("ckks_n12")
    tol = 2.0 ** -20
    assert e["fresh"] < tol and e["mult"] < tol and e["rotate"] < tol and e["conjugate"] < tol
    # q1 is 40-bit so the scale stays about 2^40 after rescale
    assert abs(np.log2(e["rescale_scale"]) - 40) < 0.01
    assert e["rescale"] < tol


@pytest.mark.slow
def test_e2e_n16_alpha4():
    """N=2^16, 24 Q-primes, 4 special primes, alpha=4: the shape whose P covers a digit."""
    e = _e2e("ckks_n16_l24_a4")
    tol = 2.0 ** -20
    assert e["fresh"] < tol and e["mult"] < tol and e["rotate"] < tol and e["conjugate"] < tol
    # after rescale by a 45-bit prime the scale is 2^35; the rounding error is
    # bounded in absolute units of 2^20 at scale 2^40
    assert e["rescale"] < 2.0 ** -15
