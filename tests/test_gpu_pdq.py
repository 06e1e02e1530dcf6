"""Private-table queries on the GPU: the op list run by the library is bit-identical
to the oracle's run, and every query's result is the same alone and in a mix of
concurrent queries served by the continuous-batching server.

N = 2^12 runs every operation on the single-pass kernels; N = 2^14 (alpha = 4,
4 special primes, the query chain) runs the fused two-pass kernels of the
benchmarked N = 2^16 workload; the alone-versus-mixed check is also made at
N = 2^16 itself (GPU against GPU, on seeded uniform residues)."""
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


_SETUP = {}


def make_setup(log_n, rows):
    from paper_2503_22227_amd import Context, pdq
    if log_n in _SETUP:
        return _SETUP[log_n]
    print("pdq keys at log_n=%d" % log_n, flush=True)
    q = client_query(log_n, rows)
    p, s = q["p"], q["s"]
    ctx = Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
    rlk = C.relin_key(p, s, q["st"]["rlk"])
    amounts = [1 << i for i in range(11)]
    gk = OQ.rotation_keys(p, s, amounts, q["st"]["galois"])
    keys = {"rlk": dev(rlk)}
    keys.update({r: dev(k) for r, k in gk.items()})
    _SETUP[log_n] = dict(q=q, p=p, s=s, ctx=ctx, rlk=rlk, gk=gk, opx=pdq.GpuExecutor(ctx, keys), rows=rows)
    return _SETUP[log_n]


@pytest.fixture(scope="module")
def setup():
    return make_setup(12, 60)


def gpu_inputs(inputs):
    return {k: dev(v.data) for k, v in inputs.items()}


@pytest.mark.parametrize("log_n,rows", [(12, 60), (14, 40)])
def test_pdq_gpu_equals_oracle(log_n, rows):
    from paper_2503_22227_amd import pdq
    setup = make_setup(log_n, rows)
    q, p = setup["q"], setup["p"]
    ops, outs, regs = pdq.plan_query(p.q, p.L, q["D"], rows, q["a"], q["b"])
    print("pdq op list of %d ops at log_n=%d (alpha=%d, k=%d)" % (len(ops), log_n, p.alpha, p.k), flush=True)
    got = setup["opx"].run(ops, gpu_inputs(q["inputs"]))
    want = OQ.Executor(p, setup["rlk"], setup["gk"]).run(ops, dict(q["inputs"]))
    # every register the op list wrote (the executors keep them all), outputs included
    assert set(got) == set(want)
    for r in sorted(got):
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


def test_server_alone_equals_mixed_n16():
    """The benchmarked serving shape (N = 2^16, 24 limbs, alpha = 4, 4 special primes):
    queries of different sizes served alone (one slot) and concurrently (four slots,
    each on its own stream and workspace) give bit-identical results."""
    import synthetic
    from paper_2503_22227_amd import Context, pdq
    from paper_2503_22227_amd.params import chain_for
    from paper_2503_22227_amd.serve import GpuQueryExecutor, Request, Server
    w = synthetic.WORKLOADS["pdq"]
    ch = chain_for(w)
    n = 1 << w["log_n"]
    L = len(ch["q"])
    ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w["seed"] + 1)
    qp = ch["q"] + ch["p"]

    def key():
        return torch.stack([torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda") for _ in range(2)])
                            for _ in range(ctx.dnum)])

    keys = {"rlk": key()}
    for i in range(9):
        keys[1 << i] = key()
    opx = pdq.GpuExecutor(ctx, keys)
    plans, inputs = [], []
    for i, rows in enumerate((10, 33, 64, 100, 128)):
        a, b = i % 4, (i + 1) % 4
        plans.append(pdq.plan_query(ch["q"], L, 2.0 ** w["log_scale"], rows, a, b))
        inputs.append({k: torch.stack([synthetic.device_uniform_residues(ch["q"], n, gen, "cuda")
                                       for _ in range(2)]) for k in ("T", "LO", "HI")})
    torch.cuda.synchronize()

    def requests():
        return [Request(rid=i, arrival=0.0, ops=ops, inputs={k: v.clone() for k, v in inputs[i].items()},
                        outputs=outs, footprint=1) for i, (ops, outs, regs) in enumerate(plans)]

    print("n16 serving: %d queries alone" % len(plans), flush=True)
    alone = requests()
    torch.cuda.synchronize()
    st1 = Server(GpuQueryExecutor(opx, 1), budget_bytes=10, slots=1).run(alone)
    print("n16 serving: mixed", flush=True)
    mixed = requests()
    torch.cuda.synchronize()
    st2 = Server(GpuQueryExecutor(opx, 4), budget_bytes=10, slots=4, ops_per_chunk=8).run(mixed)
    assert st1.completed == st2.completed == len(plans)
    assert st1.peak_inflight == 1 and st2.peak_inflight > 1
    for (ops, outs, regs), ra, rm in zip(plans, alone, mixed):
        for r in outs:
            assert torch.equal(ra.result[r], rm.result[r]), (ra.rid, r)


class _Recorder:
    """Oracle client that keeps every fresh ciphertext it sends, for replay."""

    def __init__(self, inner):
        self.inner = inner
        self.sent = []

    def inverse(self, *args):
        ct = self.inner.inverse(*args)
        self.sent.append(ct)
        return ct


class _Replay:
    def __init__(self, sent):
        self.sent = list(sent)

    def inverse(self, *args):
        return dev(self.sent.pop(0).data)


def test_search_and_average_gpu_equals_oracle(setup):
    """Search-and-average (the two-party multiply-inverse of the count): the server's
    steps on the GPU are bit-identical to the oracle's, every register, given the
    client's fresh ciphertext; then the whole protocol with the client on the GPU too
    (decrypt, CRT, decode, invert, encrypt: the client-side kernels) decrypts to the
    float64 evaluation of sum / count."""
    import synthetic
    from paper_2503_22227_amd import pdq
    q, p = setup["q"], setup["p"]
    ops, outs, regs = pdq.plan_average_query(p.q, p.L, q["D"], setup["rows"], q["a"], q["b"], 37.25)
    print("search-and-average op list of %d ops" % len(ops), flush=True)
    st = synthetic.streams(99)
    rec = _Recorder(OQ.Client(p, setup["s"], st["ct_a"], st["ct_e"]))
    want = OQ.Executor(p, setup["rlk"], setup["gk"], rec).run(ops, dict(q["inputs"]))
    opx = pdq.GpuExecutor(setup["ctx"], setup["opx"].keys, _Replay(rec.sent))
    got = opx.run(ops, gpu_inputs(q["inputs"]))
    assert set(got) == set(want)
    for r in sorted(got):
        assert np.array_equal(host(got[r]), want[r].data), r
    ref = OQ.reference_average(q["vals"], q["lo"], q["hi"], q["a"], q["b"])
    ctx = setup["ctx"]
    s_ntt = ctx.key_ntt(torch.from_numpy(np.asarray(setup["s"], dtype=np.int64)).cuda())
    st = synthetic.streams(99)
    client = pdq.GpuClient(ctx, s_ntt, st["ct_a"], st["ct_e"])
    got = pdq.GpuExecutor(ctx, setup["opx"].keys, client).run(ops, gpu_inputs(q["inputs"]))
    avg = client.slot0(got[outs[0]], regs[outs[0]][1])
    assert abs(avg - ref) < 5e-3
    # the GPU client reads the masked count as the oracle client does
    inv = [op for op in ops if op[0] == "client_inv"][0]
    x1_gpu = client.slot0(got[inv[2]], inv[3])
    x1 = C.decode(C.decrypt(p, setup["s"], C.Ciphertext(host(got[inv[2]]), inv[3])), inv[3], p.n)[0].real
    assert abs(x1_gpu - x1) <= 1e-9 * abs(x1)
