"""Autotuner of the batched key-switching launches.

Knob: the number of persistent workgroups of each launch of a batch plan
(one per work unit, or a fixed count that walks the units in contiguous
ranges), chosen per class of launch: NTT passes, base conversions, and the
element-wise steps (tensor, inner product, tail).  The search is coordinate
descent over the classes, each candidate timed with HIP events on whole-batch
graph replays; the best setting is cached per batch shape (the multiset of
ring degree and limb count) in a JSON file (RF_AUTOTUNE_CACHE, default
~/.cache/rnsfhe_autotune.json).
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

CLASSES = {
    "ntt": (1, 2, 4, 5, 7, 8, 10, 11),
    "bconv": (3, 9),
    "elementwise": (0, 6, 12),
}
CANDIDATES = (0, 256, 512, 1024, 2048, 4096)


def cache_path() -> str:
    return os.environ.get("RF_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/rnsfhe_autotune.json"))


def shape_key(shape) -> str:
    """Key of a batch: sorted (log_n, limbs) pairs."""
    s = ",".join("%d:%d" % x for x in sorted(shape))
    return hashlib.sha1(s.encode()).hexdigest()[:16]


def _time(plan, reps: int) -> float:
    stream = torch.cuda.current_stream()
    plan.run(graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.run(graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def apply(plan, setting: dict) -> None:
    for cls, stages in CLASSES.items():
        for st in stages:
            plan.set_grid(st, int(setting.get(cls, 0)))


def tune(plan, shape, reps: int = 3, use_cache: bool = True, log=None) -> dict:
    """Best {class: workgroups} for the plan; applied to the plan before returning."""
    key = shape_key(shape)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        apply(plan, cache[key]["setting"])
        return cache[key]["setting"]
    setting = {cls: 0 for cls in CLASSES}
    apply(plan, setting)
    best = _time(plan, reps)
    trials = [(dict(setting), best)]
    for cls in CLASSES:
        for cand in CANDIDATES:
            if cand == setting[cls]:
                continue
            trial = dict(setting)
            trial[cls] = cand
            apply(plan, trial)
            ms = _time(plan, reps)
            trials.append((trial, ms))
            if log:
                log("autotune %s=%d: %.3f ms" % (cls, cand, ms))
            if ms < best:
                best, setting = ms, trial
    apply(plan, setting)
    if use_cache:
        cache[key] = {"setting": setting, "ms": best, "trials": len(trials)}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return setting
