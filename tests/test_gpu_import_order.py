"""The package imported before torch still leaves torch (and the library) on
torch's HIP runtime: a fresh process imports the package first, then checks
that torch sees the GPU and that a library call runs."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import paper_2503_22227_amd as pkg
import torch
assert torch.cuda.is_available(), "torch sees no GPU after the package was imported first"
from oracle import params as P
import synthetic
p = P.make_params(synthetic.WORKLOADS["ckks_n12"])
ctx = pkg.Context(p.q, p.p, p.log_n, p.alpha, log_nmax=p.log_nmax)
x = torch.zeros((1, 1, p.n), dtype=torch.int64, device="cuda")
ctx.ntt(x, 0, 1, 1)
torch.cuda.synchronize()
assert int(x.abs().sum()) == 0
print("ok")
"""


def test_package_first_then_torch():
    print("import order: package before torch, in a fresh process", flush=True)
    res = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok")
