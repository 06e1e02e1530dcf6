"""GPU parity: every C-ABI operation against the CPU oracle, limb for limb.

All arithmetic is exact modular integer arithmetic, so the bar is bit
equality on every residue.  Inputs are seeded uniform residues (any residues
are valid inputs of these maps) and, for the accuracy checks, keys and
ciphertexts made by the oracle's client side.
"""
import numpy as np
import pytest

import synthetic
from oracle import ckks as C
from oracle import ntt as T
from oracle import params as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


_CTX = {}


def context(name, alpha=None, log_n=None):
    from paper_2503_22227_amd import Context
    key = (name, alpha, log_n)
    if key not in _CTX:
        w = dict(synthetic.WORKLOADS[name])
        if alpha:
            w["alpha"] = alpha
        p = P.make_params(w)
        if log_n is not None:
            p = p.at_degree(log_n)
        ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
        _CTX[key] = (p, ctx)
    return _CTX[key]


def rand_ct(p, nl, rng):
    return np.stack([synthetic.uniform_residues(rng, p.q[:nl], p.n) for _ in range(2)])


def rand_key(p, rng):
    qp = p.q + p.p
    return np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                     for _ in range(p.dnum())])


def show(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_ntt_intt_parity(log_n):
    p, ctx = context("ckks_batch" if log_n > 12 else "ckks_n12",
                     log_n=log_n if log_n > 12 else None)
    show("ntt log_n=%d" % log_n)
    rng = np.random.default_rng(log_n)
    # two polynomials over the limbs q_1, q_2 and the special primes (a ragged range)
    first = 1
    nl = min(3, p.L + p.k - first)
    moduli = (p.q + p.p)[first:first + nl]
    x = np.stack([synthetic.uniform_residues(rng, moduli, p.n) for _ in range(2)])
    x[0, 0, :4] = [m - 1 for m in moduli[:1]] * 4  # top of the range
    x[1, -1, -3:] = 0
    d = dev(x)
    ctx.ntt(d, first, nl, 2)
    got = host(d)
    for c in range(2):
        for i, q in enumerate(moduli):
            assert np.array_equal(got[c, i], T.ntt(x[c, i], q, p.psi(q))), (c, i)
    ctx.intt(d, first, nl, 2)
    assert np.array_equal(host(d), x)


def test_ntt_many_limbs_n16():
    p, ctx = context("ckks_n16_l24")
    rng = np.random.default_rng(5)
    moduli = p.q + p.p
    x = synthetic.uniform_residues(rng, moduli, p.n)
    d = dev(x)
    ctx.ntt(d, 0, len(moduli), 1)
    got = host(d)
    for i in (0, 1, 12, 23, 24, 27):
        q = moduli[i]
        assert np.array_equal(got[i], T.ntt(x[i], q, p.psi(q))), i
    ctx.intt(d, 0, len(moduli), 1)
    assert np.array_equal(host(d), x)


@pytest.mark.parametrize("name,nl", [("ckks_n12", 2), ("ckks_n16_l24", 24), ("ckks_n16_l24", 7)])
def test_tensor_parity(name, nl):
    p, ctx = context(name)
    rng = np.random.default_rng(nl)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    got = host(ctx.tensor(dev(a), dev(b)))
    d0, d1, d2 = C.tensor(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), p)
    assert np.array_equal(got[0], d0) and np.array_equal(got[1], d1) and np.array_equal(got[2], d2)


HMULT_CASES = [
    ("ckks_n12", None, 2),
    ("ckks_n12", None, 1),
    ("ckks_n16_l24", None, 24),   # alpha = 8, dnum = 3
    ("ckks_n16_l24", None, 13),   # a truncated last digit
    ("ckks_n16_l24", None, 1),    # one digit of one prime (nl + k < alpha)
    ("ckks_n16_l24_a4", None, 24),  # alpha = 4, dnum = 6
    ("ckks_n16_l24_a4", None, 5),  # alpha = 4, digits of 4 and 1
]


@pytest.mark.parametrize("name,alpha,nl", HMULT_CASES)
def test_hmult_relin_parity(name, alpha, nl):
    p, ctx = context(name, alpha)
    show("hmult_relin %s alpha=%s nl=%d" % (name, alpha, nl))
    rng = np.random.default_rng(100 + nl)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    rlk = rand_key(p, rng)
    got = host(ctx.hmult_relin(dev(a), dev(b), dev(rlk)))
    want = C.hmult_relin(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), rlk, p)
    assert got.shape == want.data.shape
    for c in range(2):
        for i in range(nl):
            assert np.array_equal(got[c, i], want.data[c, i]), (c, i)


@pytest.mark.parametrize("name,alpha,nl", [("ckks_n12", None, 2), ("ckks_n16_l24", None, 24),
                                           ("ckks_n16_l24", None, 10), ("ckks_n16_l24_a4", None, 24),
                                           ("ckks_n16_l24_a4", None, 10)])
def test_rotate_parity(name, alpha, nl):
    p, ctx = context(name, alpha)
    show("rotate %s nl=%d" % (name, nl))
    rng = np.random.default_rng(200 + nl)
    ct = rand_ct(p, nl, rng)
    gk = rand_key(p, rng)
    r = synthetic.rotation_index(rng, p.n)
    g = C.galois_element(r, p.n)
    got = host(ctx.rotate(dev(ct), g, dev(gk)))
    want = C.rotate(C.Ciphertext(ct, 1.0), g, gk, p)
    for c in range(2):
        for i in range(nl):
            assert np.array_equal(got[c, i], want.data[c, i]), (c, i)


@pytest.mark.parametrize("name", ["ckks_n12", "ckks_n16_l24"])
def test_automorphism_parity(name):
    p, ctx = context(name)
    rng = np.random.default_rng(7)
    nl = 3
    x = rand_ct(p, nl, rng)
    for g in (C.galois_element(1, p.n), C.galois_element(p.n // 2 - 1, p.n), 2 * p.n - 1, 1):
        got = host(ctx.automorphism(dev(x), g))
        for c in range(2):
            want = C.automorphism_ntt(x[c], g, p.q[:nl], p)
            assert np.array_equal(got[c], want), g


@pytest.mark.parametrize("name,nl", [("ckks_n12", 2), ("ckks_n16_l24", 24), ("ckks_n16_l24", 2),
                                     ("ckks_n16_l24", 9)])
def test_rescale_parity(name, nl):
    p, ctx = context(name)
    show("rescale %s nl=%d" % (name, nl))
    rng = np.random.default_rng(300 + nl)
    ct = rand_ct(p, nl, rng)
    want = C.rescale(C.Ciphertext(ct, 2.0 ** 40), p).data
    got = host(ctx.rescale(dev(ct)))
    assert np.array_equal(got, want)
    # in place: out equals in
    d = dev(ct)
    ctx.rescale(d, out=d)
    torch.cuda.synchronize()
    inplace = d.view(-1)[: 2 * (nl - 1) * p.n].reshape(2, nl - 1, p.n)
    assert np.array_equal(host(inplace), want)


@pytest.mark.parametrize("name,nl", [("ckks_n12", 2), ("ckks_n16_l24", 24), ("ckks_n16_l24", 5)])
def test_elementwise_parity(name, nl):
    """rf_add, rf_sub, rf_mul_scalar, rf_add_scalar, rf_mul_plain against the oracle."""
    p, ctx = context(name)
    rng = np.random.default_rng(400 + nl)
    a, b = rand_ct(p, nl, rng), rand_ct(p, nl, rng)
    pt = synthetic.uniform_residues(rng, p.q[:nl], p.n)
    A, B = C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0)
    assert np.array_equal(host(ctx.mul_plain(dev(a), dev(pt))), C.ct_mul_plain(A, pt, p).data)
    assert np.array_equal(host(ctx.add(dev(a), dev(b))), C.ct_add(A, B, p).data)
    assert np.array_equal(host(ctx.sub(dev(a), dev(b))), C.ct_sub(A, B, p).data)
    for k in (3, -7, (1 << 62) + 5, -(1 << 61)):
        assert np.array_equal(host(ctx.mul_scalar(dev(a), k)), C.ct_mul_int(A, k, p).data), k
        assert np.array_equal(host(ctx.add_scalar(dev(a), k)), C.ct_add_int(A, k, p).data), k
    # out aliasing an input
    d = dev(a)
    ctx.mul_plain(d, dev(pt), out=d)
    assert np.array_equal(host(d), C.ct_mul_plain(A, pt, p).data)


def test_modswitch_parity():
    p, ctx = context("ckks_n16_l24")
    rng = np.random.default_rng(4)
    nl = 6
    ct = rand_ct(p, nl, rng)
    want = C.modswitch_drop(C.Ciphertext(ct, 1.0)).data
    assert np.array_equal(host(ctx.modswitch(dev(ct))), want)
    d = dev(ct)
    ctx.modswitch(d, out=d)
    assert np.array_equal(host(d.view(-1)[: 2 * (nl - 1) * p.n].reshape(2, nl - 1, p.n)), want)


def test_keyswitch_accumulate():
    p, ctx = context("ckks_n16_l24")
    rng = np.random.default_rng(8)
    nl = 24
    dpoly = synthetic.uniform_residues(rng, p.q[:nl], p.n)
    evk = rand_key(p, rng)
    base = rand_ct(p, nl, rng)
    k0, k1 = C.keyswitch(dpoly, evk, p)
    out = dev(np.zeros_like(base))
    ctx.keyswitch(dev(dpoly), dev(evk), out, accumulate=False)
    got = host(out)
    assert np.array_equal(got[0], k0) and np.array_equal(got[1], k1)
    out = dev(base)
    ctx.keyswitch(dev(dpoly), dev(evk), out, accumulate=True)
    got = host(out)
    assert np.array_equal(got[0], C.poly_add(base[0], k0, p.q[:nl]))
    assert np.array_equal(got[1], C.poly_add(base[1], k1, p.q[:nl]))


def _client(name):
    w = synthetic.WORKLOADS[name]
    p = P.make_params(w)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    D = 2.0 ** w["log_scale"]
    z1 = synthetic.complex_slots(st["msgs"], p.n // 2)
    z2 = synthetic.complex_slots(st["msgs"], p.n // 2)
    a = C.encrypt(p, s, C.encode(z1, D, p.n), p.L, D, st["ct_a"], st["ct_e"])
    b = C.encrypt(p, s, C.encode(z2, D, p.n), p.L, D, st["ct_a"], st["ct_e"])
    return p, st, s, z1, z2, a, b


@pytest.mark.parametrize("name", ["ckks_n12", "ckks_n16_l24_a4"])
def test_decrypt_accuracy(name):
    """GPU results decrypt (oracle client) to the plaintext computation within 2^-20."""
    show("accuracy %s" % name)
    p, st, s, z1, z2, a, b = _client(name)
    _, ctx = context(name)
    rlk = C.relin_key(p, s, st["rlk"])
    r = synthetic.rotation_index(st["rot"], p.n)
    g = C.galois_element(r, p.n)
    gk = C.galois_key(p, s, g, st["galois"])
    tol = 2.0 ** -20
    m = host(ctx.hmult_relin(dev(a.data), dev(b.data), dev(rlk)))
    cm = C.Ciphertext(m, a.scale * b.scale)
    assert np.abs(C.decrypt_decode(p, s, cm) - z1 * z2).max() < tol
    rs = host(ctx.rescale(dev(m)))
    crs = C.Ciphertext(rs, cm.scale / p.q[p.L - 1])
    err = np.abs(C.decrypt_decode(p, s, crs) - z1 * z2).max()
    assert err < (tol if name == "ckks_n12" else 2.0 ** -15)
    ro = host(ctx.rotate(dev(a.data), g, dev(gk)))
    assert np.abs(C.decrypt_decode(p, s, C.Ciphertext(ro, a.scale)) - np.roll(z1, -r)).max() < tol


def test_error_codes():
    from paper_2503_22227_amd import RFError
    from paper_2503_22227_amd import _lib
    p, ctx = context("ckks_n12")
    a = dev(np.zeros((2, 2, p.n), dtype=np.uint64))
    rlk = dev(np.zeros((p.dnum(), 2, p.L + p.k, p.n), dtype=np.uint64))
    out = dev(np.zeros((2, 2, p.n), dtype=np.uint64))
    small = dev(np.zeros(16, dtype=np.uint64))
    code = _lib.lib.rf_hmult_relin(ctx._h, a.data_ptr(), a.data_ptr(), rlk.data_ptr(), out.data_ptr(), 2,
                                   small.data_ptr(), 128, None)
    assert code == _lib.RF_EWORKSPACE
    with pytest.raises(RFError):
        ctx.rotate(a, 4, rlk)  # even Galois element
    code = _lib.lib.rf_rescale(ctx._h, a.data_ptr(), out.data_ptr(), 1, small.data_ptr(), 128, None)
    assert code == _lib.RF_ELEVEL
    code = _lib.lib.rf_hmult_relin(ctx._h, a.data_ptr(), a.data_ptr(), rlk.data_ptr(), out.data_ptr(), 3,
                                   small.data_ptr(), 128, None)
    assert code == _lib.RF_ELEVEL
    # outputs overlapping inputs, Galois elements out of range, empty or
    # out-of-range limb windows: rejected on the host before any launch
    ws = ctx.workspace(_lib.RF_OP_HMULT_RELIN, 2)
    code = _lib.lib.rf_hmult_relin(ctx._h, a.data_ptr(), out.data_ptr(), rlk.data_ptr(), a.data_ptr(), 2,
                                   ws.data_ptr(), ws.numel() * 8, None)
    assert code == _lib.RF_EINVAL
    code = _lib.lib.rf_rotate(ctx._h, a.data_ptr(), 5, rlk.data_ptr(), a.data_ptr(), 2, ws.data_ptr(),
                              ws.numel() * 8, None)
    assert code == _lib.RF_EINVAL
    code = _lib.lib.rf_rotate(ctx._h, a.data_ptr(), 2 * p.n + 1, rlk.data_ptr(), out.data_ptr(), 2, ws.data_ptr(),
                              ws.numel() * 8, None)
    assert code == _lib.RF_EINVAL
    for first, nl in ((0, 0), (p.L + p.k - 1, 2)):
        assert _lib.lib.rf_ntt(ctx._h, a.data_ptr(), first, nl, 1, None) == _lib.RF_ELEVEL
        assert _lib.lib.rf_intt(ctx._h, a.data_ptr(), first, nl, 1, None) == _lib.RF_ELEVEL
    assert _lib.lib.rf_ntt(ctx._h, None, 0, 1, 1, None) == _lib.RF_EINVAL
