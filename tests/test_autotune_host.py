"""Host logic of the autotuner (no GPU): the coordinate descent keeps a change
only past its noise margin, visits every candidate of every knob, and the
per-device cache round-trips; timings come from a fake cost model."""
import json

from paper_2503_22227_amd import autotune as A


class FakeApply:
    def __init__(self, start):
        self.current = dict(start)
        self.calls = 0

    def __call__(self, setting):
        self.current = dict(setting)
        self.calls += 1


def test_descent_finds_the_best_of_a_separable_cost():
    knobs = {"x": (0, 1, 2, 3), "y": (4, 8, 16)}
    ap = FakeApply({"x": 0, "y": 8})
    cost = {"x": {0: 1.0, 1: 0.7, 2: 0.9, 3: 1.2}, "y": {4: 0.95, 8: 1.0, 16: 1.1}}

    def measure():
        return cost["x"][ap.current["x"]] * cost["y"][ap.current["y"]]

    setting, best, trials, start_ms = A._descend(knobs, ap, measure, min_gain=0.01)
    assert setting == {"x": 1, "y": 4}
    assert abs(best - 0.7 * 0.95) < 1e-12 and start_ms == 1.0
    assert ap.current == setting
    tried = {(t["x"], t["y"]) for t, _ in trials}
    assert {(x, 8) for x in knobs["x"]} <= tried      # every x tried from the start
    assert {(1, y) for y in knobs["y"]} <= tried      # every y tried at the new x


def test_descent_ignores_gains_inside_the_margin():
    knobs = {"x": (0, 1)}
    ap = FakeApply({"x": 0})
    setting, best, _, _ = A._descend(knobs, ap, lambda: 1.0 if ap.current["x"] == 0 else 0.995, min_gain=0.01)
    assert setting == {"x": 0} and best == 1.0


class FakeCtx:
    scheme, log_n, alpha, device = "ckks", 15, 8, 0
    q, p = [97, 193], [257]

    def __init__(self):
        self.levels = {}

    def get_tuning(self, nl):
        return dict(self.levels.get(nl, A.DEFAULT_LEVEL))

    def set_tuning(self, nl, setting):
        self.levels[nl] = dict(setting)


def test_tune_level_caches_per_device(tmp_path, monkeypatch):
    monkeypatch.setenv("RF_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setattr(A, "device_key", lambda device=None: "fake-gpu|256cu")
    ctx = FakeCtx()

    def fake_time(fn, reps, repeats=3):
        t = ctx.levels[14]
        return 1.0 - 0.1 * (t["modup_chunk"] == 4) - 0.05 * (t["ntt_small_below"] == 128)

    monkeypatch.setattr(A, "time_fn", fake_time)
    res = A.tune_level(ctx, 14, lambda: None)
    assert not res["cached"]
    assert res["setting"]["modup_chunk"] == 4 and res["setting"]["ntt_small_below"] == 128
    assert ctx.levels[14] == res["setting"]
    assert res["default"] == A.DEFAULT_LEVEL and res["tuned_ms"] < res["default_ms"]
    cache = json.load(open(tmp_path / "cache.json"))
    assert A.level_key(ctx, 14, "step") in cache["fake-gpu|256cu"]
    # a second call applies the cached setting without timing anything
    ctx2 = FakeCtx()
    monkeypatch.setattr(A, "time_fn", lambda *a, **k: (_ for _ in ()).throw(AssertionError("timed")))
    res2 = A.tune_level(ctx2, 14, lambda: None)
    assert res2["cached"] and ctx2.levels[14] == res["setting"]


def test_level_candidates_are_the_library_values():
    # the values rf_ctx_set_tuning accepts (include/rnsfhe.h)
    assert set(A.LEVEL_CANDIDATES["ntt_small_tile"]) == {0, 1024, 2048}
    assert set(A.LEVEL_CANDIDATES["ntt_small_radix"]) == {4, 8}
    assert set(A.LEVEL_CANDIDATES["modup_chunk"]) == {4, 8, 16}
    assert set(A.MODUP_CHUNKS) == {4, 8, 16}
    for k, v in A.DEFAULT_LEVEL.items():
        assert v in A.LEVEL_CANDIDATES[k]


def test_shipped_table_applies_matching_entries(tmp_path, monkeypatch):
    monkeypatch.setattr(A, "device_key", lambda device=None: "fake-gpu|256cu")
    monkeypatch.delenv("RF_NO_SHIPPED_TUNING", raising=False)
    table = {"fake-gpu|256cu": {A.shipped_key("ckks", 15, 8, 1, 2): dict(A.DEFAULT_LEVEL, modup_chunk=4)},
             "other|304cu": {A.shipped_key("ckks", 15, 8, 1, 1): dict(A.DEFAULT_LEVEL, modup_chunk=16)}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(table))
    ctx = FakeCtx()
    ctx.L, ctx.k = 2, 1
    assert A.apply_shipped(ctx, str(path)) == 1
    assert ctx.levels == {2: dict(A.DEFAULT_LEVEL, modup_chunk=4)}
    monkeypatch.setenv("RF_NO_SHIPPED_TUNING", "1")
    ctx2 = FakeCtx()
    ctx2.L, ctx2.k = 2, 1
    assert A.apply_shipped(ctx2, str(path)) == 0 and ctx2.levels == {}


def test_descent_discards_the_warm_up_and_confirms_a_change():
    """A first measurement inflated by warm-up cannot make the start look slow,
    and a change that a single noisy measurement favoured is dropped when the
    alternating re-measurements do not confirm it."""
    knobs = {"x": (0, 1)}
    ap = FakeApply({"x": 0})
    calls = {"n": 0}

    def measure():
        calls["n"] += 1
        if calls["n"] == 1:
            return 5.0                     # warm-up
        if calls["n"] == 3:
            return 0.9                     # one lucky measurement of x = 1
        return 1.0                         # both settings really cost the same

    setting, best, trials, start_ms = A._descend(knobs, ap, measure, min_gain=0.01)
    assert trials[0][1] == 1.0             # the warm-up was not recorded
    assert setting == {"x": 0} and best == start_ms == 1.0
    assert ap.current == {"x": 0}
