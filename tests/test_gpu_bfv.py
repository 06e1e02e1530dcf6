"""GPU parity for BFV HMult+Relin (BEHZ tensor + relinearisation) and HRotate
(Galois automorphism + key switch of coefficient-domain ciphertexts) against
the oracle, bit for bit, and exact decryption of GPU results with oracle keys."""
import numpy as np
import pytest

import synthetic
from oracle import bfv as F
from oracle import ckks as C
from oracle import params as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
_CTX = {}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def context(log_n):
    from paper_2503_22227_amd import Context
    if log_n not in _CTX:
        w = synthetic.WORKLOADS["bfv_n15"]
        p = P.make_params(w).at_degree(log_n)
        _CTX[log_n] = (p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax, scheme="bfv", t=p.t,
                                  b=p.b, m_sk=p.msk))
    return _CTX[log_n]


@pytest.mark.parametrize("log_n", [12, 15])
def test_bfv_hmult_relin_parity(log_n):
    p, ctx = context(log_n)
    print("bfv hmult log_n=%d" % log_n, flush=True)
    rng = np.random.default_rng(log_n)
    a = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
    b = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
    qp = p.q + p.p
    rlk = np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                    for _ in range(p.dnum())])
    got = host(ctx.hmult_relin(dev(a), dev(b), dev(rlk)))
    want = F.hmult_relin(a, b, rlk, p)
    assert np.array_equal(got, want)


def test_bfv_exact_slots_through_gpu():
    p, ctx = context(15)
    w = synthetic.WORKLOADS["bfv_n15"]
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    rlk = dev(F.relin_key(p, s, st["rlk"]))
    z1 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    z2 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    a = F.encrypt(p, s, F.encode(z1, p), st["ct_a"], st["ct_e"])
    b = F.encrypt(p, s, F.encode(z2, p), st["ct_a"], st["ct_e"])
    m = ctx.hmult_relin(dev(a), dev(b), rlk)
    z12 = z1 * z2 % p.t
    assert np.array_equal(F.decrypt(p, s, host(m)), z12)
    m2 = ctx.hmult_relin(m, m, rlk)
    assert np.array_equal(F.decrypt(p, s, host(m2)), z12 * z12 % p.t)


@pytest.mark.parametrize("log_n", [12, 15])
def test_bfv_rotate_parity(log_n):
    p, ctx = context(log_n)
    rng = np.random.default_rng(200 + log_n)
    ct = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
    qp = p.q + p.p
    gk = np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                   for _ in range(p.dnum())])
    for g in (C.galois_element(synthetic.rotation_index(rng, p.n), p.n), 2 * p.n - 1):
        print("bfv rotate log_n=%d g=%d" % (log_n, g), flush=True)
        got = host(ctx.rotate(dev(ct), g, dev(gk)))
        assert np.array_equal(got, F.rotate(ct, g, gk, p)), g


def test_bfv_rotate_permutes_slots_through_gpu():
    p, ctx = context(15)
    st = synthetic.streams(synthetic.WORKLOADS["bfv_n15"]["seed"] + 7)
    s = C.secret_key(p, st["sk"])
    m = F.encode(synthetic.integer_slots(st["msgs"], p.n, p.t), p)
    ct = dev(F.encrypt(p, s, m, st["ct_a"], st["ct_e"]))
    for g in (5, 2 * p.n - 1):
        gk = dev(F.galois_key(p, s, g, st["galois"]))
        m_g = np.mod(C.automorphism_coeffs(np.asarray(m, dtype=np.int64), g), p.t)
        assert np.array_equal(F.decrypt(p, s, host(ctx.rotate(ct, g, gk))), F.decode(m_g, p)), g


def test_bfv_rejects_other_levels():
    from paper_2503_22227_amd import RFError
    p, ctx = context(12)
    x = dev(np.zeros((2, p.L - 1, p.n), dtype=np.uint64))
    k = dev(np.zeros((p.dnum(), 2, p.L + p.k, p.n), dtype=np.uint64))
    with pytest.raises((RFError, ValueError)):
        ctx.hmult_relin(x, x, k)
    with pytest.raises(RFError):
        ctx.rotate(x, 5, k)
