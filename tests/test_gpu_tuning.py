"""Kernel variants a context or a batch plan can be tuned to (rf_tuning:
small-tile threshold, small tile size, radix of the small-tile rounds, ModUp
limb grouping; rf_batch_set_modup_chunk): every variant is bit-exact with the
oracle at sizes it finishes in seconds, and with the default variant at the
full N=2^16, L=24 shape, so a tuned setting changes speed only."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as C
from oracle import ntt as T
from oracle import params as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# every value of every knob at least once; small_below 4096 sends every plain
# (I)NTT launch of these shapes to the small tiles, fused_small_below 4096 every
# launch with a fused step
VARIANTS = [
    dict(ntt_small_below=0),
    dict(ntt_small_below=4096, ntt_small_tile=1024, ntt_small_radix=4),
    dict(ntt_small_below=4096, ntt_small_tile=2048, ntt_small_radix=4),
    dict(ntt_small_below=4096, ntt_small_tile=1024, ntt_small_radix=8),
    dict(ntt_small_below=4096, ntt_small_tile=2048, ntt_small_radix=8),
    dict(ntt_small_below=512, ntt_small_tile=0, ntt_small_radix=8),
    dict(modup_chunk=4),
    dict(modup_chunk=16),
    dict(ntt_small_below=64, modup_chunk=16),
    dict(ntt_fused_small_below=4096, ntt_small_tile=1024),
    dict(ntt_fused_small_below=4096, ntt_small_tile=2048),
    dict(ntt_small_below=4096, ntt_fused_small_below=512, ntt_small_tile=0, modup_chunk=4),
]
DEFAULT = dict(ntt_small_below=256, ntt_small_tile=0, ntt_small_radix=4, modup_chunk=8, ntt_fused_small_below=0)


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


_CTX = {}


def small_context(log_n):
    """Six Q-primes, three special primes, digits of two: every two-pass split."""
    from paper_2503_22227_amd import Context
    if log_n not in _CTX:
        w = dict(scheme="ckks", log_n=log_n, log_nmax=16, q_bits=[50] + [40] * 5, p_bits=[50] * 3, alpha=2,
                 log_scale=40, seed=2503222400 + log_n)
        p = P.make_params(w)
        _CTX[log_n] = (p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax))
    return _CTX[log_n]


@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
@pytest.mark.parametrize("vi", range(len(VARIANTS)))
def test_variant_ops_match_oracle(log_n, vi):
    p, ctx = small_context(log_n)
    nl = 5
    v = VARIANTS[vi]
    print("variant %s log_n=%d nl=%d" % (v, log_n, nl), flush=True)
    ctx.set_tuning(0, DEFAULT)
    ctx.set_tuning(nl, v)
    try:
        assert ctx.get_tuning(nl) == dict(DEFAULT, **v)
        rng = np.random.default_rng(100 * log_n + vi)
        a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
        rlk, gk = rand_key(p, rng), rand_key(p, rng)
        m = ctx.hmult_relin(dev(a), dev(b), dev(rlk))
        want_m = C.hmult_relin(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), rlk, p).data
        assert np.array_equal(host(m), want_m)
        assert np.array_equal(host(ctx.rescale(m)), C.rescale(C.Ciphertext(want_m, 2.0 ** 40), p).data)
        g = C.galois_element(synthetic.rotation_index(rng, p.n), p.n)
        assert np.array_equal(host(ctx.rotate(dev(a), g, dev(gk))), C.rotate(C.Ciphertext(a, 1.0), g, gk, p).data)
        # standalone transforms over a ragged window of Q- and P-limbs
        first, cnt = 3, 4
        moduli = (p.q + p.p)[first:first + cnt]
        x = np.stack([synthetic.uniform_residues(rng, moduli, p.n) for _ in range(2)])
        ctx.set_tuning(cnt, v)
        d = dev(x)
        ctx.ntt(d, first, cnt, 2)
        got = host(d)
        for c in range(2):
            for i, q in enumerate(moduli):
                assert np.array_equal(got[c, i], T.ntt(x[c, i], q, p.psi(q))), (c, i)
        ctx.intt(d, first, cnt, 2)
        assert np.array_equal(host(d), x)
    finally:
        ctx.set_tuning(0, DEFAULT)


def test_variants_full_shape_match_default():
    """N = 2^16, 24 limbs, alpha = 8: the benched shape under every variant."""
    from paper_2503_22227_amd import Context
    p = P.make_params(synthetic.WORKLOADS["ckks_n16_l24"])
    ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
    nl = p.L
    ctx.set_tuning(0, DEFAULT)
    rng = np.random.default_rng(2416)
    a, b = dev(rand_ct(p, nl, rng)), dev(rand_ct(p, nl, rng))
    rlk, gk = dev(rand_key(p, rng)), dev(rand_key(p, rng))
    g = C.galois_element(synthetic.rotation_index(rng, p.n), p.n)

    def run():
        m = ctx.hmult_relin(a, b, rlk)
        return host(m), host(ctx.rescale(m)), host(ctx.rotate(a, g, gk))

    want = run()
    for v in VARIANTS:
        print("full-shape variant %s" % v, flush=True)
        ctx.set_tuning(nl, v)
        got = run()
        for w_, g_ in zip(want, got):
            assert np.array_equal(w_, g_), v
        ctx.set_tuning(nl, DEFAULT)
    ctx.close()


def test_tuning_rejects_unsupported_values():
    from paper_2503_22227_amd import Context
    from paper_2503_22227_amd._lib import RFError
    p, ctx = small_context(14)
    ctx.set_tuning(0, DEFAULT)
    for bad in (dict(ntt_small_tile=4096), dict(ntt_small_radix=16), dict(modup_chunk=5)):
        with pytest.raises(RFError):
            ctx.set_tuning(3, bad)
    assert ctx.get_tuning(3) == DEFAULT
    with pytest.raises(RFError):
        ctx.get_tuning(p.L + 1)
    assert isinstance(ctx, Context)


def test_batch_modup_chunks_bit_identical():
    """A mixed batch under each ModUp limb grouping and two persistent grids equals
    the single-operation path, item by item."""
    from paper_2503_22227_amd import BatchPlan, Context
    w = synthetic.WORKLOADS["ckks_batch"]
    pbase = P.make_params(w)
    rng = np.random.default_rng(4242)
    shapes = [(14, 4), (14, 23), (15, 9), (15, 24), (16, 13), (16, 1)]
    ctxs, keys = {}, {}
    for ln in sorted({s[0] for s in shapes}):
        p = pbase.at_degree(ln)
        ctxs[ln] = (p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax))
        keys[ln] = dev(rand_key(p, rng))
    items, want = [], []
    for ln, nl in shapes:
        p, ctx = ctxs[ln]
        a, b = dev(rand_ct(p, nl, rng)), dev(rand_ct(p, nl, rng))
        items.append((ctx, a, b, keys[ln], torch.zeros_like(a)))
        want.append(host(ctx.hmult_relin(a, b, keys[ln])))
    plan = BatchPlan(items)
    for chunk, grid in ((4, 0), (16, 0), (8, 512), (4, 2048)):
        print("batch modup_chunk=%d grid=%d" % (chunk, grid), flush=True)
        plan.set_modup_chunk(chunk)
        for st in range(13):
            plan.set_grid(st, grid)
        for graph in (False, True):
            for it in items:
                it[4].zero_()
            plan.run(graph=graph)
            for i, it in enumerate(items):
                assert np.array_equal(host(it[4]), want[i]), (chunk, grid, graph, shapes[i])
    plan.close()


@pytest.mark.parametrize("scheme", ["bfv", "bgv"])
def test_variants_exact_schemes_match_default(scheme):
    """BFV (whose NTTs of q u B_sk and of the 14-digit ModUp run through the tuned
    launches) and BGV at N = 2^15, 14 limbs: HMult+Relin and HRotate under every
    variant equal the default."""
    from paper_2503_22227_amd import Context
    w = synthetic.WORKLOADS["%s_n15" % scheme]
    p = P.make_params(w)
    kw = dict(scheme=scheme, t=p.t)
    if scheme == "bfv":
        kw.update(b=p.b, m_sk=p.msk)
    ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax, **kw)
    nl = p.L
    rng = np.random.default_rng(1515)
    a, b = dev(rand_ct(p, nl, rng)), dev(rand_ct(p, nl, rng))
    rlk, gk = dev(rand_key(p, rng)), dev(rand_key(p, rng))
    g = C.galois_element(3, p.n)

    def run():
        return host(ctx.hmult_relin(a, b, rlk)), host(ctx.rotate(a, g, gk))

    want = run()
    for v in VARIANTS:
        print("%s variant %s" % (scheme, v), flush=True)
        ctx.set_tuning(nl, v)
        got = run()
        for w_, g_ in zip(want, got):
            assert np.array_equal(w_, g_), v
        ctx.set_tuning(nl, DEFAULT)
    ctx.close()
