"""rf_hmult_relin_noalloc (workspace in a static device array) against
rf_hmult_relin with a caller workspace, through the C ABI: two calls in a row
with the second on a smaller input, bit for bit, and the size limit.  Named to
run after every other test."""
import numpy as np
import pytest

import synthetic
from oracle import params as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    from paper_2503_22227_amd import _lib as L
    return L


def context(name, alpha=None):
    from paper_2503_22227_amd import Context
    w = dict(synthetic.WORKLOADS[name])
    if alpha:
        w["alpha"] = alpha
    p = P.make_params(w)
    return p, Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)


def operands(p, nl, gen):
    qp = p.q + p.p
    a = torch.stack([synthetic.device_uniform_residues(p.q[:nl], p.n, gen, "cuda") for _ in range(2)])
    b = torch.stack([synthetic.device_uniform_residues(p.q[:nl], p.n, gen, "cuda") for _ in range(2)])
    rlk = torch.stack([torch.stack([synthetic.device_uniform_residues(qp, p.n, gen, "cuda") for _ in range(2)])
                       for _ in range(p.dnum())])
    return a, b, rlk


def noalloc(L, ctx, a, b, rlk, out, nl):
    stream = torch.cuda.current_stream().cuda_stream
    return L.lib.rf_hmult_relin_noalloc(ctx._h, a.data_ptr(), b.data_ptr(), rlk.data_ptr(), out.data_ptr(), nl,
                                        stream)


def test_noalloc_equals_workspace_path():
    L = _lib()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    for name, alpha, sizes in (("ckks_n16_l24", None, (24, 13)), ("ckks_n16_l24", 4, (24, 5)),
                               ("ckks_n12", None, (2, 1))):
        p, ctx = context(name, alpha)
        for nl in sizes:  # the second call on a smaller input
            print("noalloc %s alpha=%d nl=%d" % (name, p.alpha, nl), flush=True)
            a, b, rlk = operands(p, nl, gen)
            want = ctx.hmult_relin(a, b, rlk)
            out = torch.zeros_like(a)
            assert noalloc(L, ctx, a, b, rlk, out, nl) == L.RF_OK, L.lib.rf_last_error()
            torch.cuda.synchronize()
            assert torch.equal(out, want), (name, nl)


def test_noalloc_rejects_what_does_not_fit():
    L = _lib()
    p, ctx = context("ckks_n16_l24", 1)  # alpha = 1: 24 digits, 400 MiB of workspace
    a = ctx.empty(2, p.L, p.n)
    out = ctx.empty(2, p.L, p.n)
    assert noalloc(L, ctx, a, a, a, out, p.L) == L.RF_EUNSUPPORTED
    assert b"static array" in L.lib.rf_last_error()
    assert noalloc(L, ctx, a, a, a, out, p.L + 1) == L.RF_ELEVEL
    assert L.lib.rf_hmult_relin_noalloc(None, None, None, None, None, 1, None) == L.RF_EINVAL
