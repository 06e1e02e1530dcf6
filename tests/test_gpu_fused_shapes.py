"""GPU parity of the fused two-pass paths at ring degrees and special-prime
counts the workload tests do not reach.

HMult+Relin, HRotate and rescale at N = 2^13, 2^14, 2^15 run their element-wise
steps inside the NTT passes (tensor and automorphism in the first inverse
pass, ModDown conversion and rescale lift in the first forward pass, the tails
in the last), with a kernel variant per two-pass split and per number K of
special primes (1 to 4, and one for any K up to 8).  Each case here is
compared limb for limb with the oracle on seeded uniform residues.
"""
import numpy as np
import pytest

import synthetic
from oracle import ckks as C
from oracle import params as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (log_n, K): every two-pass split with special-prime counts 2, 3, 5 (the
# runtime-K variant) and 8 (its largest)
SHAPES = [(13, 2), (14, 3), (15, 5), (14, 8)]

_CTX = {}


def context(log_n, k):
    from paper_2503_22227_amd import Context
    if (log_n, k) not in _CTX:
        w = dict(scheme="ckks", log_n=log_n, log_nmax=15, q_bits=[50] + [40] * 5, p_bits=[50] * k, alpha=2,
                 log_scale=40, seed=2503222275 + 16 * log_n + k)
        p = P.make_params(w)
        _CTX[(log_n, k)] = (p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax))
    return _CTX[(log_n, k)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def rand_ct(p, nl, rng):
    return np.stack([synthetic.uniform_residues(rng, p.q[:nl], p.n) for _ in range(2)])


def rand_key(p, rng):
    qp = p.q + p.p
    return np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                     for _ in range(p.dnum())])


@pytest.mark.parametrize("log_n,k", SHAPES)
@pytest.mark.parametrize("nl", [6, 3])
def test_hmult_relin_fused(log_n, k, nl):
    p, ctx = context(log_n, k)
    print("hmult_relin log_n=%d K=%d nl=%d" % (log_n, k, nl), flush=True)
    rng = np.random.default_rng(1000 * log_n + 10 * k + nl)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    rlk = rand_key(p, rng)
    got = host(ctx.hmult_relin(dev(a), dev(b), dev(rlk)))
    want = C.hmult_relin(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), rlk, p).data
    for c in range(2):
        for i in range(nl):
            assert np.array_equal(got[c, i], want[c, i]), (c, i)


@pytest.mark.parametrize("log_n,k", SHAPES)
def test_rotate_fused(log_n, k):
    p, ctx = context(log_n, k)
    nl = 5
    print("rotate log_n=%d K=%d nl=%d" % (log_n, k, nl), flush=True)
    rng = np.random.default_rng(2000 * log_n + k)
    ct = rand_ct(p, nl, rng)
    gk = rand_key(p, rng)
    for g in (C.galois_element(synthetic.rotation_index(rng, p.n), p.n), 2 * p.n - 1):
        got = host(ctx.rotate(dev(ct), g, dev(gk)))
        want = C.rotate(C.Ciphertext(ct, 1.0), g, gk, p).data
        for c in range(2):
            for i in range(nl):
                assert np.array_equal(got[c, i], want[c, i]), (g, c, i)


@pytest.mark.parametrize("log_n,k", SHAPES)
def test_rescale_fused(log_n, k):
    p, ctx = context(log_n, k)
    nl = 6
    print("rescale log_n=%d K=%d nl=%d" % (log_n, k, nl), flush=True)
    rng = np.random.default_rng(3000 * log_n + k)
    ct = rand_ct(p, nl, rng)
    want = C.rescale(C.Ciphertext(ct, 2.0 ** 40), p).data
    assert np.array_equal(host(ctx.rescale(dev(ct))), want)


# Primes just below 2^50 (the largest 50-bit primes) run the fused ModDown and
# rescale passes' butterflies without sum corrections at the edge of their
# range; 51-bit primes run the strict butterflies.  N = 2^16 gives the longest
# chains of uncorrected stages.
EDGE = dict(scheme="ckks", log_n=16, log_nmax=16, q_bits=[51, 50, 50, 51, 50], p_bits=[50, 51], alpha=2,
            log_scale=40, seed=2503222290)


def test_lazy_bound_edges():
    from paper_2503_22227_amd import Context
    p = P.make_params(EDGE)
    assert max(q for q in p.q + p.p if q < 2 ** 50) > 2 ** 50 - 2 ** 24
    assert any(q > 2 ** 50 for q in p.q + p.p)
    ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
    nl = len(p.q)
    print("lazy-bound edges log_n=16 nl=%d" % nl, flush=True)
    rng = np.random.default_rng(77)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    rlk, gk = rand_key(p, rng), rand_key(p, rng)
    m = ctx.hmult_relin(dev(a), dev(b), dev(rlk))
    want_m = C.hmult_relin(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), rlk, p)
    assert np.array_equal(host(m), want_m.data)
    want_r = C.rescale(C.Ciphertext(want_m.data, 2.0 ** 40), p).data
    assert np.array_equal(host(ctx.rescale(m)), want_r)
    g = C.galois_element(synthetic.rotation_index(rng, p.n), p.n)
    assert np.array_equal(host(ctx.rotate(dev(a), g, dev(gk))), C.rotate(C.Ciphertext(a, 1.0), g, gk, p).data)
