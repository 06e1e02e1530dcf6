"""Client side of the private-table query tests: oracle keys, encrypted table and bounds."""
import numpy as np

import synthetic
from oracle import ckks as C
from oracle import params as P
from oracle import pdq as OQ


def client_query(log_n, rows, seed=5):
    w = synthetic.WORKLOADS["pdq"]
    p = P.make_params(w).at_degree(log_n)
    st = synthetic.streams(w["seed"])
    s = C.secret_key(p, st["sk"])
    rng = np.random.default_rng(seed)
    vals = rng.integers(0, 1000, size=(rows, 4))
    lo, hi = sorted(int(x) for x in rng.integers(0, 1000, 2))
    a, b = (int(x) for x in rng.choice(4, 2, replace=False))
    D = 2.0 ** w["log_scale"]
    ns = p.n // 2

    def enc(z):
        return C.encrypt(p, s, C.encode(z, D, p.n), p.L, D, st["ct_a"], st["ct_e"])

    T = enc(OQ.table_slots(vals, ns))
    los, his = OQ.bound_slots(lo, hi, ns)
    return dict(p=p, st=st, s=s, vals=vals, lo=lo, hi=hi, a=a, b=b, D=D,
                inputs={"T": T, "LO": enc(los), "HI": enc(his)})
