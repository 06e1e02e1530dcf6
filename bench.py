"""Throughput benchmark of the CKKS key-switching hot path on one MI355X.

Workload (CKKS, N = 2^16, 24 Q-primes: one of 60 bits and 23 of 45 bits, 4
special 60-bit primes, hybrid key switching with dnum = 3 digits of alpha = 8
primes, uint64 limbs): seeded uniform residues for the ciphertexts and keys
(throughput does not depend on the values), resident in HBM before timing.

One step = HMult+Relin of two 24-limb ciphertexts, rescale of the product,
and HRotate of a 24-limb ciphertext by a random amount in [1, N/2); the
HMult+Relin -> rescale chain and the independent HRotate are issued on two
streams.  ``value`` counts the two key-switching operations of each step per
second; the same step on one stream and each operation alone (latency) are
reported beside it.

Also reported: per-operation rates from their own timed loops, per-kernel
durations from HIP events recorded on the launch stream (rf_profile_*), the
roofline of the dominant kernel, and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Integer VALU issue slots of the whole chip: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-N batch section")
    ap.add_argument("--no-pdq", action="store_true", help="skip the private-query serving section")
    ap.add_argument("--pdq-queries", type=int, default=1000, help="queries per arrival-rate point")
    ap.add_argument("--pdq-warmup", type=int, default=200, help="queries served before the measured points")
    ap.add_argument("--latency-reps", type=int, default=50, help="individually timed reps per op and cache state (0: skip)")
    ap.add_argument("--no-bfv-bgv", action="store_true", help="skip the BFV/BGV section")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the alpha=4 and N=2^12 shapes (profiling runs of the headline workload alone)")
    ap.add_argument("--variants", choices=("tuned", "shipped", "default"), default="tuned",
                    help="tuned: the shipped per-device settings, and the headline level searched again with "
                         "the two-stream step as the objective; shipped: the shipped settings, no search; "
                         "default: the library's default kernel variants everywhere")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotune section (searches against the defaults at six shapes) and the "
                         "batch autotune")
    ap.add_argument("--ntt-microbench", action="store_true",
                    help="only time forward and inverse NTTs of 60 limbs at N=2^16 (kernel profiling)")
    ap.add_argument("--workload", default="ckks_n16_l24")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (HBM counter calibration)")
    ap.add_argument("--section", choices=("batch", "bfv-bgv"),
                    help="only run this section with --steps repetitions and print its JSON (kernel profiling)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy kernel of known size, to scale FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 256 << 20
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": nbytes, "launches": 3}), flush=True)


def ntt_microbench(reps: int):
    """Forward then inverse NTT of 28, 56, 112 and 224 limbs (1, 2, 4, 8 polynomials over the
    28-prime chain) at N=2^16, ``reps`` times each; per-kernel HIP-event averages, the
    VALU fraction at 24 ops per butterfly and the HBM fraction of the pass's algorithmic
    bytes (every residue read and written once, plus a row pass's twiddle table of N
    16-byte pairs per prime)."""
    import torch

    import synthetic
    from paper_2503_22227_amd import Context
    from paper_2503_22227_amd import _lib
    from paper_2503_22227_amd.params import chain_for

    w = synthetic.WORKLOADS["ckks_n16_l24"]
    ch = chain_for(w)
    n = 1 << w["log_n"]
    ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    qp = ch["q"] + ch["p"]
    res = {}
    for polys in (1, 2, 4, 8):
        x = torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda") for _ in range(polys)])
        ctx.ntt(x, 0, 28, polys)
        ctx.intt(x, 0, 28, polys)
        torch.cuda.synchronize()
        _lib.profile_read()
        _lib.profile_enable(True)
        for _ in range(reps):
            ctx.ntt(x, 0, 28, polys)
            ctx.intt(x, 0, 28, polys)
        torch.cuda.synchronize()
        prof = _lib.profile_read()
        _lib.profile_enable(False)
        bfly = 28 * polys * (n // 2) * (w["log_n"] // 2)

        def pass_bytes(kernel):
            return 2 * 8.0 * n * 28 * polys + (16.0 * n * 28 if "rows" in kernel else 0.0)

        res[28 * polys] = {k: {"avg_us": round(ms / c * 1e3, 3),
                               "us_per_limb": round(ms / c * 1e3 / (28 * polys), 4),
                               "valu_frac_24ops": round(bfly * BFLY_OPS / (ms / c * 1e-3) / VALU_SLOTS_PER_S, 4),
                               "mb": round(pass_bytes(k) / 1e6, 1),
                               "hbm_frac": round(pass_bytes(k) / (ms / c * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
                           for k, (c, ms) in prof.items()}
        del x
    print(json.dumps({"ntt_microbench": "limbs per launch -> kernel stats at N=2^16", "limbs": res}), flush=True)


def algorithmic_bytes(kernel: str, nl: int, K: int, alpha: int, n: int, op: str) -> float:
    """Bytes one launch must move (read + write, 8 B per residue) in the HMult+Relin /
    HRotate chain at nl Q-limbs; NTT passes read and write every limb once."""
    dn = (nl + alpha - 1) // alpha
    ext = sum(nl - min(alpha, nl - j * alpha) + K for j in range(dn))
    limb = 8.0 * n
    # inner product: dn sources and 2 dn key limbs per limb of Q_l u P, 2 outputs;
    # on the fused path it also reads a, b (HMult: 4 nl limbs, its own-digit
    # residues and addends computed from them) or gathers c0, c1 (HRotate: 2 nl)
    # in place of the nl own-digit source limbs
    ip_base = dn * (nl + K) + 2 * dn * (nl + K) + 2 * (nl + K) - nl
    table = {
        "tensor": 7 * nl,
        "modup_bconv": nl + ext,
        "inner_product": ip_base + (4 * nl if op == "hmult" else 2 * nl),
        "moddown_bconv": 2 * K + 2 * nl,
        "moddown_tail": 8 * nl if op == "hmult" else 7 * nl,
        "rescale_lift": 2 + 2 * (nl - 1),
        "automorphism": 2 * nl,
    }
    return table[kernel] * limb if kernel in table else float("nan")


def latency_section(stream, ops, reps: int):
    """Per-operation latency distributions: every rep timed on its own with HIP
    events on the launch stream; median, p10, p90 and the mean of the first 10
    reps (the paper's protocol).  warm: reps back to back; cold: a 1 GiB buffer
    is rewritten on the same stream before each rep, which evicts the 256 MiB
    Infinity Cache and the L2s, so the op starts from HBM."""
    import numpy as np
    import torch

    flush = torch.empty(1 << 27, dtype=torch.int64, device="cuda")  # 1 GiB
    out = {"reps": reps, "flush_bytes": flush.numel() * 8}
    for mode in ("warm", "cold"):
        res = {}
        for name, fn in ops.items():
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            torch.cuda.synchronize()
            for e0, e1 in ev:
                if mode == "cold":
                    flush.fill_(1)
                e0.record(stream)
                fn()
                e1.record(stream)
            torch.cuda.synchronize()
            us = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])
            res[name] = {"median_us": round(float(np.median(us)), 2),
                         "p10_us": round(float(np.percentile(us, 10)), 2),
                         "p90_us": round(float(np.percentile(us, 90)), 2),
                         "mean10_us": round(float(us[:10].mean()), 2)}
        out[mode] = res
    del flush
    return out


def _copy_bandwidth(stream, nbytes: int = 256 << 20, reps: int = 5) -> float:
    """GB/s (bytes read + written) of a plain device-to-device copy of ``nbytes``,
    the best of ``reps`` event-timed copies on the launch stream."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2 * nbytes / best / 1e9


def _progress(msg: str) -> None:
    """One line per finished section on stderr (stdout carries only the result line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X; "
              "--gpus %d is not supported (the multi-GPU design is described, not built)" % args.gpus)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.ntt_microbench:
        ntt_microbench(args.steps)
        return
    if args.section:
        fn = batch_section if args.section == "batch" else bfv_bgv_section
        print(json.dumps({"section": args.section, "reps": args.steps, "result": fn(args.steps)}), flush=True)
        return

    if args.variants == "default":
        os.environ["RF_NO_SHIPPED_TUNING"] = "1"
    import synthetic

    w = synthetic.WORKLOADS[args.workload]
    cpu = None
    if not args.no_cpu_baseline:
        # first, before this process touches the GPU: the all-cores leg runs in
        # child processes
        cpu = cpu_baseline(w)
        _progress("CPU oracle baseline done")

    import numpy as np
    import torch

    from paper_2503_22227_amd import Context
    from paper_2503_22227_amd import _lib
    from paper_2503_22227_amd.params import chain_for

    ch = chain_for(w)
    n = 1 << w["log_n"]
    ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"])
    L, K, alpha = len(ch["q"]), len(ch["p"]), w["alpha"]
    dnum = (L + alpha - 1) // alpha
    st = synthetic.streams(w["seed"])
    qp = ch["q"] + ch["p"]

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()

    a = dev(np.stack([synthetic.uniform_residues(st["ct_a"], ch["q"], n) for _ in range(2)]))
    b = dev(np.stack([synthetic.uniform_residues(st["ct_a"], ch["q"], n) for _ in range(2)]))
    rlk = dev(np.stack([np.stack([synthetic.uniform_residues(st["rlk"], qp, n) for _ in range(2)])
                        for _ in range(dnum)]))
    gk = dev(np.stack([np.stack([synthetic.uniform_residues(st["galois"], qp, n) for _ in range(2)])
                       for _ in range(dnum)]))
    r = synthetic.rotation_index(st["rot"], n)
    g = ctx.galois_element(r)
    m_out = ctx.empty(2, L, n)
    r_out = ctx.empty(2, L - 1, n)
    ro_out = ctx.empty(2, L, n)

    def step():
        ctx.hmult_relin(a, b, rlk, out=m_out)
        ctx.rescale(m_out, out=r_out)
        ctx.rotate(a, g, gk, out=ro_out)

    # the timed step: the HMult+Relin -> rescale chain and the independent HRotate
    # run on two streams (own workspace slots), so their small launches overlap
    s_mul, s_rot = torch.cuda.Stream(), torch.cuda.Stream()

    def step_concurrent():
        cur = torch.cuda.current_stream()
        s_mul.wait_stream(cur)
        s_rot.wait_stream(cur)
        with torch.cuda.stream(s_mul):
            ctx.hmult_relin(a, b, rlk, out=m_out, slot=0)
            ctx.rescale(m_out, out=r_out, slot=0)
        with torch.cuda.stream(s_rot):
            ctx.rotate(a, g, gk, out=ro_out, slot=1)
        cur.wait_stream(s_mul)
        cur.wait_stream(s_rot)

    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # kernel variants of this level: the shipped settings are tuned for one
    # operation at a time (latency); the timed step runs two streams at once, so
    # the level is searched again with that step as the objective (every variant
    # gives the same residues)
    from paper_2503_22227_amd import autotune
    if args.variants in ("default", "shipped"):
        tuning = {"source": args.variants, "setting": ctx.get_tuning(L)}
    else:
        shipped = ctx.get_tuning(L)
        tuning = dict(autotune.tune_level(ctx, L, step_concurrent, reps=10, use_cache=False),
                      source="search (two-stream step)", shipped=shipped)
        _progress("autotune of the headline level done")
    for _ in range(args.warmup):
        step_concurrent()
    torch.cuda.synchronize()
    t_steps = timed(step_concurrent, args.steps)
    t_serial = timed(step, args.steps)
    ms_per_step = t_steps / args.steps * 1e3
    value = 2 * args.steps / t_steps

    # per-operation rates, each in its own loop
    reps = max(args.steps, 10)
    t_hm = timed(lambda: ctx.hmult_relin(a, b, rlk, out=m_out), reps)
    t_ro = timed(lambda: ctx.rotate(a, g, gk, out=ro_out), reps)
    t_rs = timed(lambda: ctx.rescale(m_out, out=r_out), reps)
    latency = None
    if args.latency_reps > 0:
        latency = latency_section(stream, {"hmult_relin": lambda: ctx.hmult_relin(a, b, rlk, out=m_out),
                                           "hrotate": lambda: ctx.rotate(a, g, gk, out=ro_out),
                                           "rescale": lambda: ctx.rescale(m_out, out=r_out)}, args.latency_reps)
        _progress("per-op latency distributions done")

    # per-kernel durations from HIP events on the launch stream
    _lib.profile_read()
    _lib.profile_enable(True)
    prof_steps = min(args.steps, 20)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    kernels = {k: {"launches_per_step": c / prof_steps, "avg_us": ms / c * 1e3,
                   "us_per_step": ms / prof_steps * 1e3} for k, (c, ms) in prof.items()}
    dominant = max(kernels, key=lambda k: kernels[k]["us_per_step"])
    # the same step with the Infinity Cache and the L2s flushed before every
    # operation (a 1 GiB buffer rewritten on the launch stream): each kernel's
    # inputs that the operation did not produce itself (keys, ciphertexts) come
    # from HBM
    flush = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    cold_steps = min(args.steps, 10)
    _lib.profile_read()
    for _ in range(cold_steps):
        for fn in (lambda: ctx.hmult_relin(a, b, rlk, out=m_out), lambda: ctx.rescale(m_out, out=r_out),
                   lambda: ctx.rotate(a, g, gk, out=ro_out)):
            flush.fill_(1)
            _lib.profile_enable(True)
            fn()
            _lib.profile_enable(False)
    torch.cuda.synchronize()
    cold = {k: ms / c * 1e3 for k, (c, ms) in _lib.profile_read().items()}
    del flush

    # roofline of the dominant kernel: its integer-ALU and HBM fractions, and
    # the larger of the two is the bound it is closest to
    kd = kernels[dominant]
    traffic = _counter_traffic(dominant)
    secs = kd["avg_us"] * 1e-6
    if dominant.startswith("ntt"):
        limbs, by = _ntt_launch_model(dominant, L, K, alpha, n)
        bfly = limbs * (n // 2) * (w["log_n"] // 2)
        alu = bfly * BFLY_OPS / secs / 1e12
        alu_peak = VALU_SLOTS_PER_S / 1e12
        work = "%.0f butterflies x %d int32 VALU ops; %.1f MB algorithmic HBM bytes" % (bfly, BFLY_OPS, by / 1e6)
    else:
        if dominant == "inner_product":  # one HMult+Relin and one HRotate launch per step
            by = (algorithmic_bytes(dominant, L, K, alpha, n, "hmult") +
                  algorithmic_bytes(dominant, L, K, alpha, n, "rotate")) / 2
        else:
            by = algorithmic_bytes(dominant, L, K, alpha, n, "rotate" if dominant == "automorphism" else "hmult")
        alu, alu_peak = 0.0, VALU_SLOTS_PER_S / 1e12
        work = "%.1f MB algorithmic HBM bytes" % (by / 1e6)
    hbm = by / secs / 1e9
    alu_frac, hbm_frac = alu / alu_peak, hbm / HBM_PEAK_GBS
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(alu, 3), "peak": round(alu_peak, 3), "unit": "Tops/s",
                "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    copy_gbs = _copy_bandwidth(stream)
    cold_us = cold.get(dominant)
    roof.update({"cold_avg_us": round(cold_us, 3) if cold_us else None,
                 "cold_hbm_frac": round(by / (cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if cold_us else None})
    roof.update({"passes": _pass_fractions(kernels, cold, L, K, alpha, n, w["log_n"])})
    roof.update({"traffic": traffic, "kernel": dominant, "avg_us": round(kd["avg_us"], 3),
                 "alu_frac": round(alu_frac, 4), "hbm_frac": round(hbm_frac, 4),
                 "algorithmic_bytes": round(by), "work_per_launch": work,
                 # what a plain device copy reaches on this GPU, measured here: the
                 # practical ceiling a streaming kernel is compared with
                 "copy_gbs": round(copy_gbs, 1), "hbm_frac_of_copy": round(hbm / copy_gbs, 4)})

    _progress("timed steps and kernel roofline done")
    del m_out, r_out, ro_out
    shapes = None
    if not args.no_shapes:
        shapes = other_shapes_section(max(args.steps, 20))
        _progress("alpha=4 and N=2^12 shapes done")
    tuned_shapes = None
    if not args.no_autotune:
        tuned_shapes = autotune_section()
        _progress("autotune section done")
    batch = None
    if not args.no_batch:
        batch = batch_section(max(3, min(args.steps, 10)), tune=not args.no_autotune)
        _progress("batched section done")

    exact = None
    if not args.no_bfv_bgv:
        exact = bfv_bgv_section(max(args.steps, 10))
        _progress("BFV/BGV section done")

    serving = None
    if not args.no_pdq:
        serving = pdq_section(args.pdq_queries, args.pdq_warmup)
        _progress("serving section done")

    line = {
        "metric": "CKKS HMult+Relin/HRotate per sec @N=2^16 L=24",
        "value": round(value, 2),
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "CKKS N=2^16 L=24 k=4 dnum=3 (alpha=8): HMult+Relin, rescale, HRotate "
                               "on single ciphertexts", "log_n": w["log_n"], "limbs": L,
                   "special_primes": K, "alpha": alpha, "rotation": r},
        "ops": {"step_ms_one_stream": round(t_serial / args.steps * 1e3, 4),
                "hmult_relin_per_s": round(reps / t_hm, 2), "hrotate_per_s": round(reps / t_ro, 2),
                "rescale_per_s": round(reps / t_rs, 2),
                "hmult_relin_us": round(t_hm / reps * 1e6, 2), "hrotate_us": round(t_ro / reps * 1e6, 2),
                "rescale_us": round(t_rs / reps * 1e6, 2)},
        "latency": latency,
        "tuning": tuning,
        "shapes": shapes,
        "autotune": tuned_shapes,
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in sorted(kernels.items())},
        "roofline": roof,
        "batch": batch,
        "bfv_bgv": exact,
        "pdq": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _pass_fractions(kernels, cold, L, K, alpha, n, log_n):
    """HBM (and, for NTT passes, integer-ALU) fraction of every kernel of the step,
    warm and cold, from its byte and butterfly model."""
    out = {}
    for k, v in sorted(kernels.items()):
        if k.startswith("ntt"):
            limbs, by = _ntt_launch_model(k, L, K, alpha, n)
            bfly = limbs * (n // 2) * (log_n // 2) if limbs == limbs else 0
        else:
            op = "rotate" if k == "automorphism" else "hmult"
            by = algorithmic_bytes(k, L, K, alpha, n, op)
            if k == "inner_product":
                by = (by + algorithmic_bytes(k, L, K, alpha, n, "rotate")) / 2
            bfly = 0
        if by != by:  # no byte model for this kernel
            continue
        row = {"avg_us": round(v["avg_us"], 2), "mb": round(by / 1e6, 1),
               "hbm_frac": round(by / (v["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)}
        if bfly:
            row["alu_frac"] = round(bfly * BFLY_OPS / (v["avg_us"] * 1e-6) / VALU_SLOTS_PER_S, 3)
        if k in cold:
            row["cold_us"] = round(cold[k], 2)
            row["cold_hbm_frac"] = round(by / (cold[k] * 1e-6) / 1e9 / HBM_PEAK_GBS, 3)
        out[k] = row
    return out


# Algorithmic integer work of one Harvey butterfly with a Shoup product on
# 64-bit words, counted as the fewest gfx950 VALU instructions that compute it:
# 64x64 high product 6, two 64-bit low products 4 + 4, their difference 2,
# the lazy [0, 2q) correction 4, the two outputs 1 + 3.
BFLY_OPS = 24


def _counter_traffic(kernel: str):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter table,
    or None when the table is missing or was taken on different kernel sources."""
    from paper_2503_22227_amd.profsum import source_digest
    path = os.path.join(ROOT, "profiles", "hbm_traffic_ckks_n16_l24.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if ("source-sha1: %s" % source_digest()) not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0].startswith(_kernel_symbol(kernel)):
            return round(float(cells[6]) * 1e6)
    return None


def _kernel_symbol(name: str) -> str:
    """Profiler name of a kernel as it appears in rocprofv3 tables."""
    table = {"ntt_fwd_cols": "ntt_cols_kernel<8, 8, true>", "ntt_fwd_rows": "ntt_rows_kernel<8, 8, true>",
             "ntt_inv_cols": "ntt_cols_kernel<8, 8, false>", "ntt_inv_rows": "ntt_rows_kernel<8, 8, false>",
             "ntt_fwd_rows_moddown": "ntt_rows_moddown_kernel<8, 8>",
             "ntt_fwd_rows_rescale": "ntt_rows_rescale_kernel<8, 8>",
             "ntt_fwd_cols_moddown": "ntt_cols_moddown_kernel<8, 8, 4>",
             "ntt_fwd_cols_lift": "ntt_cols_lift_kernel<8, 8, false>",
             "ntt_inv_rows_tensor": "ntt_inv_rows_tensor_kernel<8, 8>",
             "ntt_inv_rows_gather": "ntt_inv_rows_gather_kernel<8, 8>",
             "modup_bconv": "modup_bconv_kernel<true, 8>", "inner_product": "inner_product_kernel<1>"}
    return table.get(name, name + "_kernel")


def _ntt_launch_model(name: str, L: int, K: int, alpha: int, n: int):
    """(mean limbs, mean algorithmic HBM bytes) per launch of an NTT pass kernel in
    one step (HMult+Relin, rescale of its result, HRotate, at L limbs).  Bytes: every
    residue the pass and its fused prologue / epilogue must read or write once
    (8 B), plus, for row passes, each distinct prime's twiddle table once
    (N pairs of 16 B; column passes use 2^A - 1 pairs per prime, negligible)."""
    dn = (L + alpha - 1) // alpha
    ext = sum(L - min(alpha, L - j * alpha) + K for j in range(dn))
    limb, tw = 8.0 * n, 16.0 * n
    # per launch: (limbs transformed, residues-limbs moved, distinct primes with a row twiddle table)
    launches = {
        "ntt_inv_rows_tensor": [(L, 2 * L + L, L)],                   # a1, b1 in; row pass of d2 = a1 b1 out
        "ntt_inv_rows_gather": [(L, L + L, L)],                       # c1 gathered in; row pass out
        # few-limb launches (fewer tiles than CUs) run the small-tile passes:
        # the P-limbs of both key switches and rescale's last limb
        "ntt_inv_rows_small": [(2 * K, 4 * K, K)] * 2 + [(2, 4, 1)],
        "ntt_inv_cols_small": [(2 * K, 4 * K, 0)] * 2 + [(2, 4, 0)],
        "ntt_inv_cols": [(L, 2 * L, 0)] * 2,                          # d2 / sigma(c1)
        "ntt_fwd_cols": [(ext, 2 * ext, 0)] * 2,                      # ModUp NTT
        "ntt_fwd_rows": [(ext, 2 * ext, L + K)] * 2,
        "ntt_fwd_cols_moddown": [(2 * L, 2 * K + 2 * L, 0)] * 2,      # P-limbs in, conv out
        "ntt_fwd_rows_moddown": [(2 * L, 6 * L, L)] * 2,              # conv, folded ip in; out
        "ntt_fwd_cols_lift": [(2 * (L - 1), 2 + 2 * (L - 1), 0)],     # last limb in, lift out
        "ntt_fwd_rows_rescale": [(2 * (L - 1), 2 * (L - 1) * 3, L - 1)],
    }.get(name)
    if launches is None:
        return float("nan"), float("nan")
    limbs = sum(x[0] for x in launches) / len(launches)
    by = sum(x[1] * limb + x[2] * tw for x in launches) / len(launches)
    return limbs, by


def other_shapes_section(reps: int):
    """The other single-ciphertext shapes: N = 2^16, 24 limbs with alpha = 4 (dnum = 6,
    the shape whose special modulus covers a digit, so results decrypt), and the small
    N = 2^12 chain (60 + 40-bit primes, one special prime, alpha = 1) whose
    HMult+Relin -> rescale is launch-bound.  Per-op times from back-to-back loops."""
    import torch

    import synthetic
    from paper_2503_22227_amd import Context
    from paper_2503_22227_amd.params import chain_for

    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    out = {}
    for name, label in (("ckks_n16_l24_a4", "n16_l24_alpha4"), ("ckks_n12", "n12_l2_alpha1")):
        w = synthetic.WORKLOADS[name]
        ch = chain_for(w)
        n = 1 << w["log_n"]
        ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(w["seed"])
        qp = ch["q"] + ch["p"]
        L = len(ch["q"])
        a = torch.stack([synthetic.device_uniform_residues(ch["q"], n, gen, "cuda") for _ in range(2)])
        b = torch.stack([synthetic.device_uniform_residues(ch["q"], n, gen, "cuda") for _ in range(2)])
        key = lambda: torch.stack([torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda")  # noqa: E731
                                                for _ in range(2)]) for _ in range(ctx.dnum)])
        rlk, gk = key(), key()
        g = ctx.galois_element(int(synthetic.rotation_index(synthetic.streams(w["seed"])["rot"], n)))
        mo, ro, rs = torch.empty_like(a), torch.empty_like(a), ctx.empty(2, L - 1, n)
        hm = timed(lambda: ctx.hmult_relin(a, b, rlk, out=mo))
        rt = timed(lambda: ctx.rotate(a, g, gk, out=ro))
        sc = timed(lambda: ctx.rescale(mo, out=rs))
        chain = timed(lambda: (ctx.hmult_relin(a, b, rlk, out=mo), ctx.rescale(mo, out=rs)))
        out[label] = {"log_n": w["log_n"], "limbs": L, "special_primes": len(ch["p"]), "alpha": w["alpha"],
                      "dnum": ctx.dnum, "hmult_relin_us": round(hm, 2), "hrotate_us": round(rt, 2),
                      "rescale_us": round(sc, 2), "hmult_relin_rescale_us": round(chain, 2),
                      "hmult_relin_per_s": round(1e6 / hm, 1), "hrotate_per_s": round(1e6 / rt, 1)}
        del a, b, rlk, gk, mo, ro, rs
        ctx.close()
    return out


def autotune_section(shapes=((16, 24), (16, 8), (15, 14), (15, 4), (14, 24), (14, 8)), rounds: int = 7,
                     reps: int = 10):
    """Kernel variants per (ring degree, limb count): the autotuner's search for the
    level's step (HMult+Relin, rescale, HRotate at that level), then the default and
    the tuned setting timed in alternation (``rounds`` times ``reps`` steps each;
    medians), on the chain of the batched workload (24 Q-primes, 4 special primes,
    alpha = 8) at N = 2^14..2^16."""
    import statistics

    import torch

    import synthetic
    from paper_2503_22227_amd import Context, autotune
    from paper_2503_22227_amd.params import chain_for

    w = synthetic.WORKLOADS["ckks_batch"]
    ch = chain_for(w)
    qp = ch["q"] + ch["p"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w["seed"] + 7)
    out = []
    ctxs = {}
    for ln, nl in shapes:
        if ln not in ctxs:
            ctxs[ln] = Context(ch["q"], ch["p"], ln, w["alpha"], log_nmax=w["log_nmax"])
        ctx = ctxs[ln]
        n = 1 << ln
        a = torch.stack([synthetic.device_uniform_residues(ch["q"][:nl], n, gen, "cuda") for _ in range(2)])
        b = torch.stack([synthetic.device_uniform_residues(ch["q"][:nl], n, gen, "cuda") for _ in range(2)])
        dn = (nl + w["alpha"] - 1) // w["alpha"]
        rlk = torch.stack([torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda") for _ in range(2)])
                           for _ in range(ctx.dnum)])
        g = ctx.galois_element(3)
        mo, ro = torch.empty_like(a), torch.empty_like(a)
        rs = ctx.empty(2, max(nl - 1, 1), n)

        def step():
            ctx.hmult_relin(a, b, rlk, out=mo)
            if nl > 1:
                ctx.rescale(mo, out=rs)
            ctx.rotate(a, g, rlk, out=ro)

        res = autotune.tune_level(ctx, nl, step, reps=reps, use_cache=False)
        t_def, t_tun = [], []
        for _ in range(rounds):
            ctx.set_tuning(nl, res["default"])
            t_def.append(autotune.time_fn(step, reps, repeats=1))
            ctx.set_tuning(nl, res["setting"])
            t_tun.append(autotune.time_fn(step, reps, repeats=1))
        d_us, t_us = statistics.median(t_def) * 1e3, statistics.median(t_tun) * 1e3
        out.append({"log_n": ln, "limbs": nl, "digits": dn, "step_default_us": round(d_us, 2),
                    "step_tuned_us": round(t_us, 2), "gain": round(d_us / t_us - 1.0, 4),
                    "setting": res["setting"], "search_trials": res["trials"],
                    "differs_from_default": res["setting"] != res["default"]})
        ctx.set_tuning(nl, res["default"])
        del a, b, rlk, mo, ro, rs
    for ctx in ctxs.values():
        ctx.close()
    return {"workload": "per (N, limbs): HMult+Relin, rescale and HRotate at that level on the 24 + 4 prime "
                        "chain (alpha=8); default vs autotuned kernel variants, medians of %d alternating runs of "
                        "%d steps" % (rounds, reps), "shapes": out}


def batch_stage_bytes(shapes, q_count: int, K: int, alpha: int) -> dict:
    """Algorithmic HBM bytes of each stage of one batched HMult+Relin run over
    ``shapes`` [(log_n, limbs)] (names as the library's profile scopes): every
    residue a stage and its fused prologue / epilogue must read or write once
    (8 B), plus each row pass's twiddle table (N 16-byte pairs) once per distinct
    prime and ring degree.  The two inverse column passes (of d2 and of the
    special-prime limbs) share one scope name."""
    from collections import defaultdict
    out = defaultdict(float)
    primes = defaultdict(lambda: defaultdict(set))
    for ln, nl in shapes:
        n = 1 << ln
        limb = 8.0 * n
        dn = (nl + alpha - 1) // alpha
        ext = sum(nl - min(alpha, nl - j * alpha) + K for j in range(dn))
        out["batch_ntt_inv_rows_tensor"] += 3 * nl * limb      # a1, b1 read, d2 row written
        out["batch_ntt_inv_cols"] += 2 * nl * limb + 2 * (2 * K) * limb
        out["batch_modup_bconv"] += algorithmic_bytes("modup_bconv", nl, K, alpha, n, "hmult")
        out["batch_ntt_fwd_cols"] += 2 * ext * limb
        out["batch_ntt_fwd_rows"] += 2 * ext * limb
        out["batch_inner_product"] += algorithmic_bytes("inner_product", nl, K, alpha, n, "hmult")
        out["batch_ntt_inv_rows"] += 2 * (2 * K) * limb
        out["batch_ntt_fwd_cols_moddown"] += (2 * K + 2 * nl) * limb
        out["batch_ntt_fwd_rows_moddown"] += 6 * nl * limb      # conv, ip' read, result written
        primes[ln]["q"].update(range(nl))
        primes[ln]["ext"].update(list(range(nl)) + [q_count + k for k in range(K)])
        primes[ln]["p"].update(q_count + k for k in range(K))
    for ln, ps in primes.items():
        tw = 16.0 * (1 << ln)
        out["batch_ntt_inv_rows_tensor"] += tw * len(ps["q"])
        out["batch_ntt_fwd_rows"] += tw * len(ps["ext"])
        out["batch_ntt_inv_rows"] += tw * len(ps["p"])
        out["batch_ntt_fwd_rows_moddown"] += tw * len(ps["q"])
    return dict(out)


def batch_section(reps: int, tune: bool = True):
    """256 HMult+Relin items of mixed N in {2^14, 2^15, 2^16} and 4..24 limbs: one graph
    replay of the batched launches vs one HMult+Relin call per item on the same stream,
    issued back to back (``plain``) and with a synchronisation after every call
    (``plain_synced``, one operation per launch chain)."""
    import torch

    import synthetic
    from paper_2503_22227_amd import BatchPlan, Context, autotune
    from paper_2503_22227_amd.params import chain_for

    w = synthetic.WORKLOADS["ckks_batch"]
    ch = chain_for(w)
    st = synthetic.streams(w["seed"])
    shapes = synthetic.batch_shapes(st["batch_shape"], w["items"], w["log_n_choices"], w["limbs_range"])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w["seed"])
    qp = ch["q"] + ch["p"]
    ctxs, keys = {}, {}
    for ln in sorted({x[0] for x in shapes}):
        ctxs[ln] = Context(ch["q"], ch["p"], ln, w["alpha"], log_nmax=w["log_nmax"])
        n = 1 << ln
        dnum = ctxs[ln].dnum
        keys[ln] = torch.stack([torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda")
                                             for _ in range(2)]) for _ in range(dnum)])
    items = []
    for ln, nl in shapes:
        n = 1 << ln
        a = torch.stack([synthetic.device_uniform_residues(ch["q"][:nl], n, gen, "cuda") for _ in range(2)])
        b = torch.stack([synthetic.device_uniform_residues(ch["q"][:nl], n, gen, "cuda") for _ in range(2)])
        items.append((ctxs[ln], a, b, keys[ln], torch.empty_like(a)))
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    def plain():
        for ctx, a, b, k, out in items:
            ctx.hmult_relin(a, b, k, out=out)

    def plain_synced():
        for ctx, a, b, k, out in items:
            ctx.hmult_relin(a, b, k, out=out)
            torch.cuda.synchronize()

    t_plain = timed(plain)
    t_plain_synced = timed(plain_synced)
    plan = BatchPlan(items)
    t_default = timed(lambda: plan.run(graph=True))
    setting = autotune.tune(plan, shapes, reps=2, use_cache=False) if tune else None
    t_batch = timed(lambda: plan.run(graph=True))
    # per-stage times of eager runs (HIP events around each stage's launches),
    # against the stage's algorithmic bytes
    from paper_2503_22227_amd import _lib
    plan.run(graph=False)
    torch.cuda.synchronize()
    _lib.profile_read()
    _lib.profile_enable(True)
    for _ in range(3):
        plan.run(graph=False)
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    sbytes = batch_stage_bytes(shapes, len(ch["q"]), len(ch["p"]), w["alpha"])
    stages = {}
    for name, (cnt, ms) in sorted(prof.items()):
        if name in sbytes and cnt:
            sec = ms / 3 * 1e-3  # the stage's total time per run
            stages[name] = {"ms_per_run": round(ms / 3, 3), "gb": round(sbytes[name] / 1e9, 3),
                            "hbm_frac": round(sbytes[name] / sec / (HBM_PEAK_GBS * 1e9), 3)}
    n_items = len(items)
    limb_bytes = sum(7 * nl * (8 << ln) for ln, nl in shapes)
    out = {"workload": "256 CKKS HMult+Relin items, N in {2^14,2^15,2^16}, 4..24 limbs, k=4, alpha=8",
           "items": n_items, "batched_items_per_s": round(n_items / t_batch, 1),
           "plain_items_per_s": round(n_items / t_plain, 1), "speedup": round(t_plain / t_batch, 3),
           "plain_synced_items_per_s": round(n_items / t_plain_synced, 1),
           "speedup_vs_synced": round(t_plain_synced / t_batch, 3),
           "batched_ms": round(t_batch * 1e3, 3), "plain_ms": round(t_plain * 1e3, 3),
           "batched_default_ms": round(t_default * 1e3, 3), "autotuned": setting,
           "ciphertext_bytes_in_out": limb_bytes, "stages": stages}
    plan.close()
    return out


def bfv_bgv_section(reps: int):
    """BFV (BEHZ) and BGV HMult+Relin at N=2^15 with 14 55-bit primes, t=65537, one 60-bit
    special prime (alpha=1), seeded uniform residues."""
    import torch

    import synthetic
    from paper_2503_22227_amd import Context
    from paper_2503_22227_amd.params import chain_for

    out = {}
    for name in ("bfv_n15", "bgv_n15"):
        w = synthetic.WORKLOADS[name]
        ch = chain_for(w)
        n = 1 << w["log_n"]
        ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"], scheme=w["scheme"],
                      t=w["t"], b=ch["b"], m_sk=ch["msk"])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(w["seed"])
        qp = ch["q"] + ch["p"]
        rlk = torch.stack([torch.stack([synthetic.device_uniform_residues(qp, n, gen, "cuda") for _ in range(2)])
                           for _ in range(ctx.dnum)])
        a = torch.stack([synthetic.device_uniform_residues(ch["q"], n, gen, "cuda") for _ in range(2)])
        b = torch.stack([synthetic.device_uniform_residues(ch["q"], n, gen, "cuda") for _ in range(2)])
        o = torch.empty_like(a)
        ctx.hmult_relin(a, b, rlk, out=o)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            ctx.hmult_relin(a, b, rlk, out=o)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        out[w["scheme"]] = {"hmult_relin_us": round(us, 2), "hmult_relin_per_s": round(1e6 / us, 1)}
        ctx.close()
    out["workload"] = "N=2^15, 14 x 55-bit Q, t=65537, 1 special 60-bit prime (alpha=1); BFV B = 14 x 60-bit + m_sk"
    return out


def pdq_section(n_queries: int, n_warmup: int):
    """Private-table range-sum and search-and-average queries at CKKS N=2^16, 24 limbs,
    alpha=4, scale 2^45 served by the continuous-batching server, with keys, tables
    and the multiply-inverse client step made by the client-side kernels:
    saturation rate from a burst, then Poisson
    arrivals at 0.25 / 0.5 / 0.75 / 0.9 of it (4 slots, 6 GiB budget); one point where
    the budget, not the slot count, bounds admission (8 slots); one uncapped run
    (8 slots, no budget).  Latency = arrival to result on the host; p50 / p99 over
    ``n_queries`` queries per point after ``n_warmup`` served first."""
    import numpy as np
    import torch

    import synthetic
    from paper_2503_22227_amd import Context, pdq
    from paper_2503_22227_amd import _lib
    from paper_2503_22227_amd.params import chain_for
    from paper_2503_22227_amd.serve import GpuQueryExecutor, Request, Server

    w = synthetic.WORKLOADS["pdq"]
    ch = chain_for(w)
    n = 1 << w["log_n"]
    L = len(ch["q"])
    D = 2.0 ** w["log_scale"]
    ctx = Context(ch["q"], ch["p"], w["log_n"], w["alpha"], log_nmax=w["log_nmax"])
    st = synthetic.streams(w["seed"])
    rng = st["arrivals"]
    # the client side on the GPU: secret key, relinearisation and power-of-two
    # rotation keys, encrypted tables and bounds
    s_ntt = ctx.key_ntt(torch.from_numpy(synthetic.ternary(st["sk"], n)).cuda())
    client = pdq.GpuClient(ctx, s_ntt, st["ct_a"], st["ct_e"])
    keys = client.switch_keys([1 << i for i in range(12)], st["rlk"])
    opx = pdq.GpuExecutor(ctx, keys, client)
    ct_bytes = 2 * L * n * 8
    # the key-switching workspace every slot holds (HMult+Relin needs the most)
    ws_bytes = max(ctx.workspace_bytes(_lib.RF_OP_HMULT_RELIN, L), ctx.workspace_bytes(_lib.RF_OP_ROTATE, L))
    # queries read their encrypted table and bounds and never write them: one
    # table per row padding (16 .. 1024 rows) and a pool of bounds are shared
    tables = {}
    for k in range(4, 11):
        rows_t = int(rng.integers((1 << (k - 1)) + 1, (1 << k) + 1))
        tables[1 << k] = client.encrypt_table(rng.integers(0, 1000, size=(rows_t, 4)), L, D)
    bounds = []
    for _ in range(8):
        lo, hi = sorted(int(x) for x in rng.integers(0, 1000, 2))
        bounds.append(client.encrypt_bounds(lo, hi, L, D))
    plans = {}

    def make(count, rate):
        reqs, t = [], 0.0
        for i in range(count):
            rows = int(round(np.exp(rng.uniform(np.log(10), np.log(1000)))))
            a, b = (int(x) for x in rng.choice(4, 2, replace=False))
            avg = rng.random() < 0.25  # a quarter are search-and-average queries
            key = (rows, a, b, avg)
            if key not in plans:
                if avg:
                    r = float(np.exp(rng.uniform(0.0, np.log(64.0))))
                    ops, outs, regs = pdq.plan_average_query(ch["q"], L, D, rows, a, b, r)
                else:
                    ops, outs, regs = pdq.plan_query(ch["q"], L, D, rows, a, b)
                plans[key] = (ops, outs, (pdq.peak_live(ops, outputs=outs) + 3 + int(avg)) * ct_bytes)
            ops, outs, fp = plans[key]
            if rate:
                t += rng.exponential(1.0 / rate)
            lo_ct, hi_ct = bounds[i % len(bounds)]
            reqs.append(Request(rid=i, arrival=t, ops=ops,
                                inputs={"T": tables[pdq.r_pad(rows)], "LO": lo_ct, "HI": hi_ct}, outputs=outs,
                                footprint=fp))
        torch.cuda.synchronize()  # keys, tables and bounds are written before any query starts
        return reqs

    def serve(reqs, slots, budget):
        # every slot keeps its own workspace: charged once per slot, not per query
        avail = (1 << 62) if budget is None else budget - slots * ws_bytes
        return Server(GpuQueryExecutor(opx, slots), avail, slots=slots).run(reqs)

    def point(s2, **kw):
        d = {"queries_per_s": round(s2.completed / s2.makespan, 2), "p50_ms": round(s2.percentile(50) * 1e3, 2),
             "p99_ms": round(s2.percentile(99) * 1e3, 2), "samples": len(s2.latencies), "completed": s2.completed,
             "failed": s2.failed, "peak_inflight": s2.peak_inflight, "peak_admitted_gib": round(s2.peak_bytes / 2 ** 30, 2)}
        d.update(kw)
        return d

    budget = 6 << 30
    serve(make(n_warmup, 0), 4, budget)
    burst = make(n_queries, 0)
    stb = serve(burst, 4, budget)
    sat = stb.completed / stb.makespan
    points = []
    for f in (0.25, 0.5, 0.75, 0.9):
        points.append(point(serve(make(n_queries, f * sat), 4, budget), load=f, arrival_rate_qps=round(f * sat, 2),
                            slots=4, budget_gib=6))
    mean_fp = float(np.mean([r.footprint for r in burst]))
    tight = 8 * ws_bytes + int(2.5 * mean_fp)
    points.append(point(serve(make(n_queries, 0.9 * sat), 8, tight), load=0.9, arrival_rate_qps=round(0.9 * sat, 2),
                        slots=8, budget_gib=round(tight / 2 ** 30, 2), note="budget-bound admission"))
    points.append(point(serve(make(n_queries, 0.9 * sat), 8, None), load=0.9, arrival_rate_qps=round(0.9 * sat, 2),
                        slots=8, budget_gib=None, note="uncapped admission"))
    return {"workload": "range-sum queries (a quarter search-and-average, with the client's multiply-inverse "
                        "step on the GPU), CKKS N=2^16 24 limbs alpha=4 scale 2^45, tables of 10..1000 rows x 4 "
                        "columns (log-uniform), keys and encrypted tables made by the GPU client, %d queries per "
                        "point after %d warm-up, Poisson arrivals" % (n_queries, n_warmup),
            "ops_per_query_mean": round(float(np.mean([len(r.ops) for r in burst])), 1),
            "query_footprint_mean_mib": round(mean_fp / 2 ** 20, 1),
            "slot_workspace_mib": round(ws_bytes / 2 ** 20, 1),
            "saturation_qps": round(sat, 2), "burst_p50_ms": round(stb.percentile(50) * 1e3, 2),
            "burst_p99_ms": round(stb.percentile(99) * 1e3, 2), "points": points}


def _oracle_pairs(args):
    """Worker: ``pairs`` HMult+Relin + HRotate pairs of the oracle at full size; returns
    (pairs, seconds of the timed loop)."""
    w, pairs, seed = args
    import numpy as np

    import synthetic
    from oracle import ckks as C
    from oracle import params as P

    p = P.make_params(w)
    rng = np.random.default_rng(seed)
    ct = lambda: np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])  # noqa: E731
    qp = p.q + p.p
    key = lambda: np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])  # noqa: E731
                            for _ in range(p.dnum())])
    a, b, rlk, gk = ct(), ct(), key(), key()
    g = C.galois_element(3, p.n)
    t0 = time.perf_counter()
    for _ in range(pairs):
        C.hmult_relin(C.Ciphertext(a, 1.0), C.Ciphertext(b, 1.0), rlk, p)
        C.rotate(C.Ciphertext(a, 1.0), g, gk, p)
    return pairs, time.perf_counter() - t0


def cpu_baseline(w, min_seconds: float = 10.0, max_pairs: int = 12):
    """The oracle, as it stands, on a bounded sample of the same workload.
    Single thread: HMult+Relin / HRotate pairs at full size until at least
    ``min_seconds`` (at most ``max_pairs``).  All host cores: one process per
    logical CPU (at most 16), each timing one pair on its own operands; the
    rate is the pairs over the slowest process's loop.  Also the BFV and BGV
    HMult+Relin of the N = 2^15, 14-limb chain, one each, single thread."""
    import multiprocessing as mp

    import numpy as np

    import synthetic
    from oracle import bfv as OF
    from oracle import bgv as OB
    from oracle import params as P

    pairs, dt = 0, 0.0
    while pairs < max_pairs and (pairs == 0 or dt < min_seconds):
        k, t = _oracle_pairs((w, 1, 1 + pairs))
        pairs, dt = pairs + k, dt + t
    procs = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_pairs, [(w, 1, 100 + i) for i in range(procs)])
    par_dt = max(t for _, t in res)
    exact = {}
    for name in ("bfv_n15", "bgv_n15"):
        wx = synthetic.WORKLOADS[name]
        p = P.make_params(wx)
        rng = np.random.default_rng(2)
        ct = np.stack([synthetic.uniform_residues(rng, p.q, p.n) for _ in range(2)])
        qp = p.q + p.p
        rlk = np.stack([np.stack([synthetic.uniform_residues(rng, qp, p.n) for _ in range(2)])
                        for _ in range(p.dnum())])
        t0 = time.perf_counter()
        if name == "bfv_n15":
            OF.hmult_relin(ct, ct, rlk, p)
        else:
            OB.hmult_relin(OB.Ciphertext(ct), OB.Ciphertext(ct), rlk, p)
        exact[wx["scheme"]] = {"hmult_relin_s": round(time.perf_counter() - t0, 3)}
    return {"value": round(2 * procs / par_dt, 4), "unit": "ops/s", "cores": procs, "kind": "oracle",
            "sample": "%d processes, each 1 HMult+Relin + 1 HRotate at N=2^16, 24 limbs, dnum=3 (slowest %.1f s)"
                      % (procs, par_dt),
            "single_thread": {"value": round(2 * pairs / dt, 4), "cores": 1,
                              "sample": "%d HMult+Relin + %d HRotate (%.1f s)" % (pairs, pairs, dt)},
            "bfv_bgv_single_thread": exact,
            "host_cpu": _cpu_model(), "host_logical_cpus": os.cpu_count()}


def _cpu_model() -> str:
    """The timing host's CPU model (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
