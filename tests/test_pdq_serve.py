"""CPU tests of the private-query circuit planner and the continuous-batching
scheduler (fake executor, synthetic clock), and of the circuit on the oracle
against its float64 evaluation."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as C
from oracle import params as P
from oracle import pdq as OQ
from paper_2503_22227_amd import pdq
from paper_2503_22227_amd.params import chain_for
from paper_2503_22227_amd.serve import Request, Server

from pdq_client import client_query


def test_f7_coefficients_match_definition():
    xs = np.linspace(-1, 1, 41)
    poly = sum(float(c) * xs ** (2 * k + 1) for k, c in enumerate(pdq.F7))
    assert np.allclose(poly, OQ.f7(xs), atol=1e-12)
    # the composite is a sign approximation on [-1, 1]
    assert abs(OQ.f7(OQ.f7(OQ.f7(0.1))) - 1) < 1e-3 and abs(OQ.f7(OQ.f7(OQ.f7(-0.5))) + 1) < 1e-6


@pytest.mark.parametrize("rows", [10, 100, 1000])
def test_plan_levels_and_scales(rows):
    ch = chain_for(synthetic.WORKLOADS["pdq"])
    ops, (s, c), regs = pdq.plan_query(ch["q"], 24, 2.0 ** 45, rows, 3, 0)
    assert all(regs[r][0] >= 1 for r in regs)
    for r in (s, c):
        assert abs(regs[r][1] / 2.0 ** 45 - 1) < 1e-4
    for op in ops:
        if op[0] == "rot":
            assert op[3] & (op[3] - 1) == 0 and op[3] < 4096
        if op[0] in ("add", "sub", "hmult"):
            assert regs[op[2]][0] == regs[op[3]][0]
    assert pdq.peak_live(ops, outputs=(s, c)) <= 16


class FakeExecutor:
    """Each op costs `cost` simulated seconds of device time on its slot; results are
    the request id (so ordering mistakes are visible)."""

    def __init__(self, clock, cost=1e-3, fail_rid=None):
        self.clock = clock
        self.cost = cost
        self.fail_rid = fail_rid
        self.busy_until = {}
        self.inflight_bytes = []

    def start(self, req, slot):
        if req.rid == self.fail_rid:
            raise RuntimeError("injected failure")
        return {"req": req, "slot": slot, "chunks": []}

    def issue(self, h, begin, end):
        t = max(self.clock.t, self.busy_until.get(h["slot"], 0.0)) + (end - begin) * self.cost
        self.busy_until[h["slot"]] = t
        h["chunks"].append(t)

    def poll(self, h):
        return sum(1 for t in h["chunks"] if t <= self.clock.t)

    def finish(self, h):
        return {"rid": h["req"].rid}


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


def make_requests(n, footprint, ops=20, spacing=0.002):
    return [Request(rid=i, arrival=i * spacing, ops=[("nop",)] * ops, inputs={}, outputs=(),
                    footprint=footprint) for i in range(n)]


def test_server_admission_and_latency():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=3 * 100, slots=4, ops_per_chunk=5, clock=clk, sleep=clk.sleep)
    reqs = make_requests(12, footprint=100)
    st = srv.run(reqs)
    assert st.completed == 12 and st.failed == 0
    assert st.peak_bytes <= 300 and st.peak_inflight == 3
    for r in reqs:
        assert r.result == {"rid": r.rid}
        assert r.admitted >= r.arrival - 1e-12
        assert r.latency >= len(r.ops) * ex.cost - 1e-9
    # FIFO admission
    adm = [r.admitted for r in sorted(reqs, key=lambda r: r.rid)]
    assert adm == sorted(adm)


def test_server_overlaps_requests_on_slots():
    clk = Clock()
    ex = FakeExecutor(clk)
    reqs = [Request(rid=i, arrival=0.0, ops=[("nop",)] * 40, inputs={}, outputs=(), footprint=1) for i in range(4)]
    st = Server(ex, budget_bytes=10, slots=4, ops_per_chunk=8, clock=clk, sleep=clk.sleep).run(reqs)
    serial = 4 * 40 * ex.cost
    assert st.makespan < serial / 2  # four slots run side by side


def test_server_failure_isolation_and_oversize():
    clk = Clock()
    ex = FakeExecutor(clk, fail_rid=2)
    reqs = make_requests(5, footprint=10)
    reqs.append(Request(rid=99, arrival=0.001, ops=[("nop",)], inputs={}, outputs=(), footprint=10 ** 9))
    st = Server(ex, budget_bytes=100, slots=2, clock=clk, sleep=clk.sleep).run(reqs)
    assert st.completed == 4 and st.failed == 2
    by = {r.rid: r for r in reqs}
    assert by[2].error and by[99].error and by[0].result == {"rid": 0}


@pytest.mark.slow
def test_circuit_on_oracle_matches_float_evaluation():
    q = client_query(12, 60)
    p, s = q["p"], q["s"]
    ops, (so, co), regs = pdq.plan_query(p.q, p.L, q["D"], 60, q["a"], q["b"])
    rlk = C.relin_key(p, s, q["st"]["rlk"])
    gk = OQ.rotation_keys(p, s, pdq.rotation_amounts(ops), q["st"]["galois"])
    out = OQ.Executor(p, rlk, gk).run(ops, dict(q["inputs"]))
    ref = OQ.reference(q["vals"], q["lo"], q["hi"], q["a"], q["b"])
    got_s = C.decode(C.decrypt(p, s, out[so]), regs[so][1], p.n)[0].real
    got_c = C.decode(C.decrypt(p, s, out[co]), regs[co][1], p.n)[0].real
    assert abs(got_s - ref[0]) < 0.05 and abs(got_c - ref[1]) < 0.05


def _oracle_keys(q):
    p, s = q["p"], q["s"]
    return C.relin_key(p, s, q["st"]["rlk"]), OQ.rotation_keys(p, s, [1 << i for i in range(11)], q["st"]["galois"])


@pytest.mark.parametrize("x", [1.0, 3.0, 117.0, 1000.0, 0.125])
def test_multiply_inverse_protocol_on_oracle(x):
    """The paper's two-party multiply-inverse on a fresh encryption of x in every slot:
    the server masks by r, the client inverts slot 0 of the decryption and re-encrypts,
    the server unmasks by r.  Pin: the result decrypts to 1/x within 2^-30 (the paper
    reports 32 fractional bits; here the noise of the rescales after the masking
    products bounds it)."""
    w = synthetic.WORKLOADS["pdq"]
    p = P.make_params(w).at_degree(12)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    rlk = C.relin_key(p, s, st["rlk"])
    D = 2.0 ** w["log_scale"]
    ct = C.encrypt(p, s, C.encode(np.full(p.n // 2, x, dtype=np.complex128), D, p.n), p.L, D, st["ct_a"], st["ct_e"])
    r = 13.75
    pl = pdq.Planner(p.q)
    X = pl.input("X", p.L, D)
    y = pl.mulc(pl.client_inverse(pl.mulc(X, r), p.L, D), r)
    cl = OQ.Client(p, s, st["ct_a"], st["ct_e"])
    res = OQ.Executor(p, rlk, {}, cl).run(pl.ops, {"X": ct})
    got = C.decode(C.decrypt(p, s, res[y]), pl.scale(y), p.n)
    assert [op[0] for op in pl.ops] == ["mul_int", "rescale", "client_inv", "mul_int", "rescale"]
    assert np.abs(got - 1.0 / x).max() < 2.0 ** -30


def test_search_and_average_on_oracle_matches_float_evaluation():
    """Search-and-average: the whole op list (range-sum circuit, masking, client
    inversion, unmasking, product with the sum) on the oracle decrypts to the float64
    evaluation of the same circuit's sum / count."""
    q = client_query(12, 60)
    p, s = q["p"], q["s"]
    rlk, gk = _oracle_keys(q)
    ops, outs, regs = pdq.plan_average_query(p.q, p.L, q["D"], 60, q["a"], q["b"], 37.25)
    assert sum(op[0] == "client_inv" for op in ops) == 1
    st = synthetic.streams(99)
    res = OQ.Executor(p, rlk, gk, OQ.Client(p, s, st["ct_a"], st["ct_e"])).run(ops, dict(q["inputs"]))
    avg = C.decode(C.decrypt(p, s, res[outs[0]]), regs[outs[0]][1], p.n)[0].real
    ref = OQ.reference_average(q["vals"], q["lo"], q["hi"], q["a"], q["b"])
    assert abs(avg - ref) < 5e-3
