"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds random draws and workload descriptions only: no modular
arithmetic, no NTT, no key or ciphertext construction.  Both the CPU oracle
and the GPU path consume the arrays drawn here, so that for one seed they see
the same secret, errors, masks and messages.

Random streams are numpy ``Generator(PCG64)`` objects spawned from
``SeedSequence(seed)`` in a fixed order (``STREAM_NAMES``); each consumer asks
for its stream by name, so adding a draw to one stream never shifts another.

Distributions (the paper fixes none of them; these are the usual RLWE choices):
  * secret: ternary, each of {-1, 0, 1} with probability 1/3;
  * error: rounded normal with sigma = 3.2, redrawn when |e| > 19 (about 6 sigma);
  * mask polynomials ``a``: uniform residues in [0, q) per RNS limb;
  * CKKS messages: complex slots with real and imaginary parts uniform in [-1, 1].
"""
from __future__ import annotations

import numpy as np

STREAM_NAMES = (
    "sk", "rlk", "galois", "ct_a", "ct_e", "msgs", "rot", "batch_shape", "arrivals",
)

ERROR_SIGMA = 3.2
ERROR_BOUND = 19


def streams(seed: int) -> dict:
    """One independent Generator per name of ``STREAM_NAMES``, spawned from ``seed``."""
    children = np.random.SeedSequence(int(seed)).spawn(len(STREAM_NAMES))
    return {name: np.random.Generator(np.random.PCG64(c)) for name, c in zip(STREAM_NAMES, children)}


def ternary(rng: np.random.Generator, n: int) -> np.ndarray:
    """n coefficients uniform over {-1, 0, 1}, as int64."""
    return rng.integers(-1, 2, size=n, dtype=np.int64)


def gaussian(rng: np.random.Generator, n: int, sigma: float = ERROR_SIGMA,
             bound: int = ERROR_BOUND) -> np.ndarray:
    """n rounded-normal integers with standard deviation ``sigma``; draws with |e| > bound are redrawn."""
    out = np.rint(rng.normal(0.0, sigma, size=n)).astype(np.int64)
    bad = np.abs(out) > bound
    while bad.any():
        out[bad] = np.rint(rng.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(out) > bound
    return out


def uniform_residues(rng: np.random.Generator, moduli, n: int) -> np.ndarray:
    """Array [len(moduli), n] of uint64; row i is uniform in [0, moduli[i])."""
    moduli = [int(m) for m in moduli]
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, m in enumerate(moduli):
        out[i] = rng.integers(0, m, size=n, dtype=np.uint64)
    return out


def complex_slots(rng: np.random.Generator, count: int) -> np.ndarray:
    """``count`` complex128 values with real and imaginary parts uniform in [-1, 1]."""
    re = rng.uniform(-1.0, 1.0, size=count)
    im = rng.uniform(-1.0, 1.0, size=count)
    return re + 1j * im


def integer_slots(rng: np.random.Generator, count: int, t: int) -> np.ndarray:
    """``count`` integers uniform in [0, t), as int64 (BFV/BGV plaintext slots)."""
    return rng.integers(0, int(t), size=count, dtype=np.int64)


def rotation_index(rng: np.random.Generator, n: int) -> int:
    """A rotation amount uniform in [1, n/2)."""
    return int(rng.integers(1, n // 2))


# Workload descriptions: ring degree, prime bit sizes and counts, digit size
# (alpha = primes per key-switching digit), and the CKKS scale.  The prime
# values themselves are derived from these by each side independently.
WORKLOADS = {
    # one ciphertext pair, HMult+Relin then rescale
    "ckks_n12": dict(scheme="ckks", log_n=12, log_nmax=12, q_bits=[60, 40], p_bits=[60],
                     alpha=1, log_scale=40, seed=2503222270),
    # single-ciphertext HMult+Relin, HRotate, rescale at N=2^16 with 24 Q-primes
    # and 4 special primes; dnum=3 gives alpha=8
    "ckks_n16_l24": dict(scheme="ckks", log_n=16, log_nmax=16, q_bits=[60] + [45] * 23,
                         p_bits=[60] * 4, alpha=8, log_scale=40, seed=2503222271),
    # same chain with alpha=4 (dnum=6), the shape whose special modulus covers a digit
    "ckks_n16_l24_a4": dict(scheme="ckks", log_n=16, log_nmax=16, q_bits=[60] + [45] * 23,
                            p_bits=[60] * 4, alpha=4, log_scale=40, seed=2503222271),
    # mixed-N batches share one prime chain congruent to 1 mod 2^17
    "ckks_batch": dict(scheme="ckks", log_n=16, log_nmax=16, q_bits=[60] + [45] * 23,
                       p_bits=[60] * 4, alpha=8, log_scale=40, seed=2503222272,
                       items=256, log_n_choices=[14, 15, 16], limbs_range=[4, 24]),
    # BFV / BGV exact integer slots
    "bfv_n15": dict(scheme="bfv", log_n=15, log_nmax=15, q_bits=[55] * 14, p_bits=[60],
                    alpha=1, t=65537, b_bits=[60] * 14, msk_bits=60, log_mtilde=32,
                    seed=2503222273),
    "bgv_n15": dict(scheme="bgv", log_n=15, log_nmax=15, q_bits=[55] * 14, p_bits=[60],
                    alpha=1, t=65537, seed=2503222273),
    # private-table queries
    "pdq": dict(scheme="ckks", log_n=16, log_nmax=16, q_bits=[60] + [45] * 23,
                p_bits=[60] * 4, alpha=4, log_scale=45, seed=2503222274),
}


def batch_shapes(rng: np.random.Generator, items: int, log_n_choices, limbs_range):
    """(log_n, limbs) of each batch item: ring degree uniform over the choices,
    limb count uniform in [lo, hi]."""
    lns = rng.choice(np.asarray(log_n_choices), size=items)
    nls = rng.integers(limbs_range[0], limbs_range[1] + 1, size=items)
    return [(int(a), int(b)) for a, b in zip(lns, nls)]


def device_uniform_residues(moduli, n: int, generator, device):
    """Like ``uniform_residues`` but drawn on a torch device with a seeded torch
    Generator (for inputs too large to draw on the host); int64 tensor [len(moduli), n]."""
    import torch
    out = torch.empty((len(moduli), n), dtype=torch.int64, device=device)
    for i, m in enumerate(moduli):
        out[i] = torch.randint(0, int(m), (n,), generator=generator, device=device, dtype=torch.int64)
    return out
