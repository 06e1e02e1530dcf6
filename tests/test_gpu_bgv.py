"""GPU parity for BGV (t-preserving ModDown and modulus switch) against the oracle,
bit for bit, plus exact decryption of GPU results with oracle-made keys."""
import numpy as np
import pytest

import synthetic
from oracle import bgv as B
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


def context(log_n=15):
    from paper_2503_22227_amd import Context
    if log_n not in _CTX:
        w = dict(synthetic.WORKLOADS["bgv_n15"])
        w["log_n"] = log_n
        p = P.make_params(w)
        _CTX[log_n] = (p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax, scheme="bgv", t=p.t))
    return _CTX[log_n]


def rand_ct(p, nl, rng):
    return np.stack([synthetic.uniform_residues(rng, p.q[:nl], p.n) for _ in range(2)])


def rand_key(p, rng):
    qp = p.q + p.p
    return np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                     for _ in range(p.dnum())])


@pytest.mark.parametrize("log_n,nl", [(15, 14), (15, 5), (12, 14)])
def test_bgv_hmult_relin_parity(log_n, nl):
    p, ctx = context(log_n)
    print("bgv hmult log_n=%d nl=%d" % (log_n, nl), flush=True)
    rng = np.random.default_rng(nl + log_n)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    rlk = rand_key(p, rng)
    got = host(ctx.hmult_relin(dev(a), dev(b), dev(rlk)))
    want = B.hmult_relin(B.Ciphertext(a), B.Ciphertext(b), rlk, p)
    assert np.array_equal(got, want.data)


@pytest.mark.parametrize("nl", [14, 2])
def test_bgv_modswitch_parity(nl):
    p, ctx = context(15)
    rng = np.random.default_rng(50 + nl)
    ct = rand_ct(p, nl, rng)
    want = B.modswitch(B.Ciphertext(ct), p).data
    assert np.array_equal(host(ctx.modswitch(dev(ct))), want)
    d = dev(ct)
    ctx.modswitch(d, out=d)
    assert np.array_equal(host(d.view(-1)[: 2 * (nl - 1) * p.n].reshape(2, nl - 1, p.n)), want)


@pytest.mark.parametrize("conj,nl", [(False, 14), (True, 14), (True, 6)])
def test_bgv_rotate_parity(conj, nl):
    """Column rotation (g = 5) and the row swap (g = 2N - 1)."""
    p, ctx = context(15)
    rng = np.random.default_rng(77 + nl)
    ct = rand_ct(p, nl, rng)
    gk = rand_key(p, rng)
    g = 2 * p.n - 1 if conj else C.galois_element(5, p.n)
    got = host(ctx.rotate(dev(ct), g, dev(gk)))
    want = B.rotate(B.Ciphertext(ct), g, gk, p)
    assert np.array_equal(got, want.data)


def test_bgv_rescale_is_rejected():
    from paper_2503_22227_amd import RFError
    p, ctx = context(12)
    with pytest.raises(RFError):
        ctx.rescale(dev(np.zeros((2, 3, p.n), dtype=np.uint64)))


def test_bgv_exact_slots_through_gpu():
    """Oracle keys and ciphertexts; HMult+Relin, modulus switch and a second HMult+Relin on
    the GPU; the oracle decrypts the exact slot products."""
    p, ctx = context(15)
    w = synthetic.WORKLOADS["bgv_n15"]
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    z1 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    z2 = synthetic.integer_slots(st["msgs"], p.n, p.t)
    a = B.encrypt(p, s, B.encode(z1, p), p.L, st["ct_a"], st["ct_e"])
    b = B.encrypt(p, s, B.encode(z2, p), p.L, st["ct_a"], st["ct_e"])
    rlk = B.relin_key(p, s, st["rlk"])
    r = dev(rlk)
    m = ctx.hmult_relin(dev(a.data), dev(b.data), r)
    z12 = z1 * z2 % p.t
    assert np.array_equal(B.decrypt(p, s, B.Ciphertext(host(m), 1)), z12)
    ms = ctx.modswitch(m)
    f = pow(p.q[p.L - 1], -1, p.t)
    assert np.array_equal(B.decrypt(p, s, B.Ciphertext(host(ms), f)), z12)
    m2 = ctx.hmult_relin(ms, ms, r)
    assert np.array_equal(B.decrypt(p, s, B.Ciphertext(host(m2), f * f % p.t)), z12 * z12 % p.t)
