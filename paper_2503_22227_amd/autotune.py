"""Autotuner of the kernel variants (the segmentation and grouping choices of
the paper's kernel-fusion section, III-A.3, searched per shape instead of fixed;
the stream-pool size ablation of V-C is the paper's own analogue of such a
search).

Single operations, per (ring degree, limb count) of a context
(``tune_level``): the knobs of ``rf_tuning``

  * ntt_small_below: below how many 4096-residue tiles an (I)NTT launch runs
    small tiles (0: never);
  * ntt_small_tile: 1024- or 2048-residue small tiles (0: by launch size);
  * ntt_small_radix: residues per thread of the small tiles, i.e. radix-4 or
    radix-8 LDS rounds (the 4096-residue tiles always run radix-16 rounds);
  * modup_chunk: ModUp output limbs per thread (the conversion's limb grouping);
  * ntt_fused_small_below: the small-tile threshold of the launches that carry
    a fused step (tensor, automorphism, ModDown conversion and tail, rescale
    lift and tail).

Batches (``tune``): the workgroup count of each class of batched launch (one
per work unit, or a fixed persistent count walking contiguous ranges) and the
batched ModUp limb grouping.

Settings found on a device can be shipped with the package
(``tuned_variants.json``, written by ``python -m paper_2503_22227_amd.autotune
--write-table``): a context created on a device of the same architecture and CU count
applies the entry of its ring degree, alpha and special-prime count at every
level it lists (``apply_shipped``; RF_NO_SHIPPED_TUNING=1 keeps the defaults).

Both searches are coordinate descent from the defaults: each candidate value of
one knob is timed with HIP events, and a change is kept only if it is faster
than the best so far by more than ``min_gain`` (a relative margin, so timing
noise does not move the setting).  Results are cached per device (architecture and
CU count) and shape in a JSON file (RF_AUTOTUNE_CACHE, default
~/.cache/rnsfhe_autotune.json).  Every variant computes the same residues, so
tuning changes speed only.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

# ---------------------------------------------------------------- batches
CLASSES = {
    "ntt": (1, 2, 4, 5, 7, 8, 10, 11),
    "bconv": (3, 9),
    "elementwise": (0, 6, 12),
}
CANDIDATES = (0, 256, 512, 1024, 2048, 4096)
MODUP_CHUNKS = (4, 8, 16)

# ---------------------------------------------------------------- single operations
LEVEL_CANDIDATES = {
    "ntt_small_below": (0, 64, 128, 256, 512, 1024, 4096),
    "ntt_small_tile": (0, 1024, 2048),
    "ntt_small_radix": (4, 8),
    "modup_chunk": (4, 8, 16),
    "ntt_fused_small_below": (0, 128, 256, 512, 1024),
}
DEFAULT_LEVEL = {"ntt_small_below": 256, "ntt_small_tile": 0, "ntt_small_radix": 4, "modup_chunk": 8,
                 "ntt_fused_small_below": 0}


def cache_path() -> str:
    return os.environ.get("RF_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/rnsfhe_autotune.json"))


def device_key(device=None) -> str:
    """Architecture and CU count (the marketing name a process sees depends on
    how the runtime was loaded, e.g. under a profiler)."""
    p = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return "%s|%dcu" % (arch.split(":")[0], p.multi_processor_count)


def shape_key(shape) -> str:
    """Key of a batch: sorted (log_n, limbs) pairs."""
    s = ",".join("%d:%d" % x for x in sorted(shape))
    return hashlib.sha1(s.encode()).hexdigest()[:16]


def _load_cache(path: str) -> dict:
    if os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            pass
    return {}


def _store_cache(path: str, cache: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_fn(fn, reps: int, repeats: int = 3) -> float:
    """Best of ``repeats`` mean times (ms) of ``reps`` back-to-back calls of fn on
    the current stream, after one untimed call."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def _descend(knobs: dict, apply, measure, min_gain: float, log=None, rounds: int = 2, confirm: int = 2):
    """Coordinate descent over ``knobs`` ({name: candidates}) starting from the
    setting ``apply`` was last given; returns (setting, best_ms, trials,
    start_ms).  The first measurement is a discarded warm-up (clocks, caches,
    first launches), and a setting that differs from the start is kept only if
    ``confirm`` alternating re-measurements of both (best of each) still show
    the gain; best_ms and start_ms are then those re-measured times."""
    setting = dict(apply.current)
    start = dict(setting)
    apply(setting)
    measure()
    best = measure()
    start_ms = best
    trials = [(dict(setting), best)]
    for _ in range(rounds):
        moved = False
        for name, cands in knobs.items():
            for cand in cands:
                if cand == setting[name]:
                    continue
                trial = dict(setting)
                trial[name] = cand
                apply(trial)
                ms = measure()
                trials.append((trial, ms))
                if log:
                    log("autotune %s=%s: %.4f ms" % (name, cand, ms))
                if ms < best * (1.0 - min_gain):
                    best, setting, moved = ms, trial, True
        if not moved:
            break
    if setting != start and confirm > 0:
        t_start, t_best = [], []
        for _ in range(confirm):
            apply(start)
            t_start.append(measure())
            apply(setting)
            t_best.append(measure())
        start_ms, best = min(t_start), min(t_best)
        if log:
            log("autotune confirm: start %.4f ms, chosen %.4f ms" % (start_ms, best))
        if not best < start_ms * (1.0 - min_gain):
            setting, best = start, start_ms
    apply(setting)
    return setting, best, trials, start_ms


class _LevelApply:
    def __init__(self, ctx, nlimbs):
        self.ctx, self.nlimbs = ctx, nlimbs
        self.current = ctx.get_tuning(nlimbs)

    def __call__(self, setting):
        self.ctx.set_tuning(self.nlimbs, setting)
        self.current = dict(setting)


def level_key(ctx, nlimbs: int, tag: str) -> str:
    h = hashlib.sha1(",".join(str(x) for x in ctx.q + ctx.p).encode()).hexdigest()[:12]
    return "level:%s:%d:%d:%d:%s:%s" % (ctx.scheme, ctx.log_n, nlimbs, ctx.alpha, h, tag)


def tune_level(ctx, nlimbs: int, workload, reps: int = 10, min_gain: float = 0.01, use_cache: bool = True,
               tag: str = "step", log=None) -> dict:
    """Best rf_tuning of level ``nlimbs`` of ``ctx`` for ``workload`` (a callable
    running the operations to optimise once, e.g. HMult+Relin, HRotate and rescale
    at that level); applied to the context before returning.  Returns
    {"setting", "default", "default_ms", "tuned_ms", "trials", "cached"}."""
    path = cache_path()
    key = level_key(ctx, nlimbs, tag)
    dkey = device_key(ctx.device)
    cache = _load_cache(path) if use_cache else {}
    hit = cache.get(dkey, {}).get(key)
    if hit:
        ctx.set_tuning(nlimbs, hit["setting"])
        return dict(hit, cached=True)
    ap = _LevelApply(ctx, nlimbs)
    ap(DEFAULT_LEVEL)
    setting, best, trials, default_ms = _descend(LEVEL_CANDIDATES, ap, lambda: time_fn(workload, reps), min_gain,
                                                 log)
    res = {"setting": setting, "default": dict(DEFAULT_LEVEL), "default_ms": default_ms, "tuned_ms": best,
           "trials": len(trials)}
    if use_cache:
        cache = _load_cache(path)
        cache.setdefault(dkey, {})[key] = res
        _store_cache(path, cache)
    return dict(res, cached=False)


class _BatchApply:
    def __init__(self, plan):
        self.plan = plan
        self.current = {cls: 0 for cls in CLASSES}
        self.current["modup_chunk"] = 8

    def __call__(self, setting):
        for cls, stages in CLASSES.items():
            for st in stages:
                self.plan.set_grid(st, int(setting.get(cls, 0)))
        self.plan.set_modup_chunk(int(setting.get("modup_chunk", 8)))
        self.current = dict(setting)


def apply(plan, setting: dict) -> None:
    _BatchApply(plan)(setting)


def tune(plan, shape, reps: int = 3, use_cache: bool = True, min_gain: float = 0.01, log=None) -> dict:
    """Best {class: workgroups, "modup_chunk": limbs} for a batch plan; applied to
    the plan before returning."""
    key = "batch:" + shape_key(shape)
    path = cache_path()
    dkey = device_key()
    cache = _load_cache(path) if use_cache else {}
    hit = cache.get(dkey, {}).get(key)
    if hit:
        apply(plan, hit["setting"])
        return hit["setting"]
    knobs = {cls: CANDIDATES for cls in CLASSES}
    knobs["modup_chunk"] = MODUP_CHUNKS
    ap = _BatchApply(plan)
    setting, best, trials, _ = _descend(knobs, ap, lambda: time_fn(lambda: plan.run(graph=True), reps, repeats=2),
                                        min_gain, log, rounds=1)
    if use_cache:
        cache = _load_cache(path)
        cache.setdefault(dkey, {})[key] = {"setting": setting, "ms": best, "trials": len(trials)}
        _store_cache(path, cache)
    return setting


# ---------------------------------------------------------------- shipped table
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_variants.json")


def shipped_key(scheme: str, log_n: int, alpha: int, k: int, nlimbs: int) -> str:
    return "%s:%d:%d:%d:%d" % (scheme, log_n, alpha, k, nlimbs)


def apply_shipped(ctx, path: str = SHIPPED) -> int:
    """Apply the shipped settings of ``ctx``'s device and shape to its levels;
    returns the number of levels set (0 when the table has no entry)."""
    if os.environ.get("RF_NO_SHIPPED_TUNING") == "1" or not os.path.exists(path):
        return 0
    try:
        with open(path) as f:
            table = json.load(f).get(device_key(ctx.device), {})
    except (OSError, ValueError):
        return 0
    n = 0
    for nl in range(1, ctx.L + 1):
        setting = table.get(shipped_key(ctx.scheme, ctx.log_n, ctx.alpha, ctx.k, nl))
        if setting:
            ctx.set_tuning(nl, setting)
            n += 1
    return n


# (workload, ring degrees) searched by write_table
TABLE_WORKLOADS = (("ckks_batch", (14, 15, 16)), ("pdq", (16,)), ("bgv_n15", (15,)), ("bfv_n15", (15,)))


def write_table(out: str, workloads=TABLE_WORKLOADS, levels=None, reps: int = 10) -> dict:
    """Tune each level of each workload's chain for one operation at a time: CKKS
    HMult+Relin, rescale and HRotate; BGV HMult+Relin, modulus switch and HRotate;
    BFV HMult+Relin and HRotate (at all L limbs, the only level BFV runs at).
    Settings that differ from the defaults are merged into this device's entry of
    ``out``; with ``levels`` given, a level in between takes the setting of the
    tuned level below it."""
    import synthetic
    from .fhe import Context
    from .params import chain_for

    dkey = device_key()
    table = {}
    saved = os.environ.get("RF_NO_SHIPPED_TUNING")
    os.environ["RF_NO_SHIPPED_TUNING"] = "1"  # search from the defaults
    for wname, lns in workloads:
        w = synthetic.WORKLOADS[wname]
        ch = chain_for(w)
        qp = ch["q"] + ch["p"]
        scheme = w["scheme"]
        kw = {}
        if scheme != "ckks":
            kw = dict(scheme=scheme, t=w["t"])
        if scheme == "bfv":
            kw.update(b=ch["b"], m_sk=ch["msk"])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(w["seed"] + 11)
        for ln in lns:
            ctx = Context(ch["q"], ch["p"], ln, w["alpha"], log_nmax=w["log_nmax"], **kw)
            n = 1 << ln
            key = torch.stack([torch.stack([_residues(qp, n, gen) for _ in range(2)]) for _ in range(ctx.dnum)])
            tuned_levels = [ctx.L] if scheme == "bfv" else (levels or range(1, ctx.L + 1))
            prev = None
            for nl in range(1, ctx.L + 1):
                if nl in tuned_levels:
                    a = torch.stack([_residues(ch["q"][:nl], n, gen) for _ in range(2)])
                    b = torch.stack([_residues(ch["q"][:nl], n, gen) for _ in range(2)])
                    g = ctx.galois_element(3)

                    def step():
                        m = ctx.hmult_relin(a, b, key)
                        if nl > 1 and scheme == "ckks":
                            ctx.rescale(m)
                        elif nl > 1 and scheme == "bgv":
                            ctx.modswitch(m)
                        ctx.rotate(a, g, key)

                    res = tune_level(ctx, nl, step, reps=reps, use_cache=False)
                    prev = res["setting"] if res["setting"] != res["default"] else None
                    print("tuned %s N=2^%d limbs=%d: %s (%.4f -> %.4f ms)" % (
                        wname, ln, nl, res["setting"], res["default_ms"], res["tuned_ms"]), flush=True)
                if prev is not None and (levels is not None or nl in tuned_levels):
                    table[shipped_key(scheme, ln, w["alpha"], len(ch["p"]), nl)] = prev
            ctx.close()
    if saved is None:
        del os.environ["RF_NO_SHIPPED_TUNING"]
    else:
        os.environ["RF_NO_SHIPPED_TUNING"] = saved
    doc = {}
    if os.path.exists(out):
        try:
            with open(out) as f:
                doc = json.load(f)
        except (OSError, ValueError):
            doc = {}
    doc.setdefault(dkey, {}).update(table)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    return table


def _residues(moduli, n, gen):
    import synthetic
    return synthetic.device_uniform_residues(moduli, n, gen, "cuda")


if __name__ == "__main__":
    import sys
    if len(sys.argv) >= 2 and sys.argv[1] == "--write-table":
        names = sys.argv[3:]
        wl = tuple(w for w in TABLE_WORKLOADS if not names or w[0] in names)
        print(json.dumps(write_table(sys.argv[2] if len(sys.argv) > 2 else SHIPPED, wl), indent=1))
    else:
        raise SystemExit("usage: python -m paper_2503_22227_amd.autotune --write-table [path [workload ...]]")
