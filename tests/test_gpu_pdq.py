"""Private-table queries on the GPU: the op list run by the library is bit-identical
to the oracle's run, and every query's result is the same alone and in a mix of
concurrent queries served by the continuous-batching server."""
import numpy as np
import pytest

from oracle import ckks as C
from oracle import pdq as OQ
from pdq_client import client_query

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def setup():
    from paper_2503_22227_amd import Context, pdq
    q = client_query(12, 60)
    p, s = q["p"], q["s"]
    ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
    rlk = C.relin_key(p, s, q["st"]["rlk"])
    amounts = [1 << i for i in range(11)]
    gk = OQ.rotation_keys(p, s, amounts, q["st"]["galois"])
    keys = {"rlk": dev(rlk)}
    keys.update({r: dev(k) for r, k in gk.items()})
    return dict(q=q, p=p, s=s, ctx=ctx, rlk=rlk, gk=gk, opx=pdq.GpuExecutor(ctx, keys))


def gpu_inputs(inputs):
    return {k: dev(v.data) for k, v in inputs.items()}


def test_pdq_gpu_equals_oracle(setup):
    from paper_2503_22227_amd import pdq
    q, p = setup["q"], setup["p"]
    ops, outs, regs = pdq.plan_query(p.q, p.L, q["D"], 60, q["a"], q["b"])
    print("pdq op list of %d ops" % len(ops), flush=True)
    got = setup["opx"].run(ops, gpu_inputs(q["inputs"]))
    want = OQ.Executor(p, setup["rlk"], setup["gk"]).run(ops, dict(q["inputs"]))
    for r in outs:
        assert np.array_equal(host(got[r]), want[r].data), r
    ref = OQ.reference(q["vals"], q["lo"], q["hi"], q["a"], q["b"])
    dec = [C.decode(C.decrypt(p, setup["s"], C.Ciphertext(host(got[r]), 1.0)), regs[r][1], p.n)[0].real
           for r in outs]
    assert abs(dec[0] - ref[0]) < 0.05 and abs(dec[1] - ref[1]) < 0.05


def test_server_alone_equals_mixed(setup):
    from paper_2503_22227_amd import pdq
    from paper_2503_22227_amd.serve import GpuQueryExecutor, Request, Server
    p = setup["p"]
    queries = []
    for i, rows in enumerate((10, 33, 60, 128, 200, 256)):
        q = client_query(12, rows, seed=100 + i)
        ops, outs, regs = pdq.plan_query(p.q, p.L, q["D"], rows, q["a"], q["b"])
        queries.append((q, ops, outs, regs))

    def requests(spacing):
        return [Request(rid=i, arrival=i * spacing, ops=ops, inputs=gpu_inputs(q["inputs"]), outputs=outs,
                        footprint=1) for i, (q, ops, outs, regs) in enumerate(queries)]

    alone = requests(0.0)
    st1 = Server(GpuQueryExecutor(setup["opx"], 1), budget_bytes=10, slots=1).run(alone)
    mixed = requests(0.0)
    st2 = Server(GpuQueryExecutor(setup["opx"], 4), budget_bytes=10, slots=4, ops_per_chunk=8).run(mixed)
    assert st1.completed == st2.completed == len(queries)
    assert st1.peak_inflight == 1 and st2.peak_inflight > 1
    for (q, ops, outs, regs), ra, rm in zip(queries, alone, mixed):
        for r in outs:
            a = ra.result[r].numpy().view(np.uint64)
            m = rm.result[r].numpy().view(np.uint64)
            assert np.array_equal(a, m), (ra.rid, r)
        ref = OQ.reference(q["vals"], q["lo"], q["hi"], q["a"], q["b"])
        got = C.decode(C.decrypt(p, q["s"], C.Ciphertext(rm.result[outs[0]].numpy().view(np.uint64), 1.0)),
                       regs[outs[0]][1], p.n)[0].real
        assert abs(got - ref[0]) < 0.05
