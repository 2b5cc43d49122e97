"""Host logic of the autotuner (no GPU): the coordinate descent finds the
best thresholds of a synthetic cost model, keeps the defaults when nothing
beats them by the minimum gain, and the cache is used only while its key
(source hash and device) matches."""
import json
import os

import pytest

from paper_2311_03010_amd import autotune


@pytest.fixture(autouse=True)
def _restore_thresholds(monkeypatch):
    # apply() writes the environment; monkeypatch restores it afterwards
    for k in autotune.KNOBS:
        monkeypatch.delenv(k, raising=False)


class _FakeWorkloads:
    # time of each workload as a function of the thresholds set in the
    # environment: separable, minimal at the chosen optimum
    optimum = {"EECMG_TALL_MIN_TILES": 4096, "EECMG_SHORT_MAX_TILES": 512, "EECMG_FOLD_MAX_TILES": 4096,
               "EECMG_FOLD_MAX_TILES_STREAM": 512, "EECMG_LAZY_MIN_PIXELS": 1 << 20,
               "EECMG_COARSE_MAX_PIXELS": 1024, "EECMG_MAX_AHEAD": 2,
               "EECMG_PACE_STEPS": 3, "EECMG_BATCH_LANES": 2}

    def __init__(self, *a, **k):
        pass

    def time(self, reps=5):
        cost = 1.0
        for knob, opt in self.optimum.items():
            cands = autotune.KNOBS[knob][1]
            cost *= 1.0 + 0.05 * abs(cands.index(int(os.environ[knob])) - cands.index(opt))
        return {"a": cost, "b": 2 * cost}


def test_coordinate_descent_finds_the_optimum(monkeypatch):
    monkeypatch.setattr(autotune, "_Workloads", _FakeWorkloads)
    res = autotune.tune(None, None, None)
    assert res["settings"] == _FakeWorkloads.optimum
    assert res["time_vs_defaults"] < 1.0
    assert all(os.environ[k] == str(v) for k, v in res["settings"].items())


def test_defaults_kept_below_the_minimum_gain(monkeypatch):
    class Flat(_FakeWorkloads):
        def time(self, reps=5):
            return {"a": 1.0}

    monkeypatch.setattr(autotune, "_Workloads", Flat)
    res = autotune.tune(None, None, None)
    assert res["settings"] == autotune.defaults()


def test_cache_used_only_for_the_same_sources_and_device(monkeypatch, tmp_path):
    class FakeCuda:
        @staticmethod
        def get_device_name(i):
            return "dev-A"

    class FakeTorch:
        cuda = FakeCuda

    calls = []
    monkeypatch.setattr(autotune, "tune", lambda *a, **k: calls.append(1) or {"settings": autotune.defaults()})
    cache = tmp_path / "t.json"
    r1 = autotune.load_or_tune(FakeTorch, None, None, cache=str(cache))
    r2 = autotune.load_or_tune(FakeTorch, None, None, cache=str(cache))
    assert (r1["source"], r2["source"]) == ("tuned", "cache") and len(calls) == 1
    c = json.loads(cache.read_text())
    c["key"]["source_hash"] = "0" * 16
    cache.write_text(json.dumps(c))
    assert autotune.load_or_tune(FakeTorch, None, None, cache=str(cache))["source"] == "tuned"
    assert len(calls) == 2


def test_defaults_kept_when_the_final_check_shows_no_gain(monkeypatch):
    """A change accepted during the descent (its trial looked faster) is
    dropped when the final comparison against the defaults is not faster."""
    # one pass of the descent times every candidate but the current one
    n_descent = sum(len([c for c in cands if c != dflt]) for dflt, cands in autotune.KNOBS.values())
    calls = {"n": 0, "accepted": False}

    def fake_ab(wl, a, b, reps):
        calls["n"] += 1
        gain = a == dict(autotune.defaults(), EECMG_PACE_STEPS=3) and b == autotune.defaults()
        if gain and calls["n"] <= n_descent:
            calls["accepted"] = True
            return {"a": 0.95, "b": 0.96}  # looks faster in the descent
        if gain:
            return {"a": 1.01, "b": 1.0}   # ... but not in the final check
        return {"a": 1.0, "b": 1.0}

    class Flat(_FakeWorkloads):
        def time(self, reps=5):
            return {"a": 1.0, "b": 1.0}

    monkeypatch.setattr(autotune, "_Workloads", Flat)
    monkeypatch.setattr(autotune, "_ab", fake_ab)
    res = autotune.tune(None, None, None, passes=1)
    assert calls["accepted"] and calls["n"] == n_descent + 1
    assert res["settings"] == autotune.defaults()
    assert res["time_vs_defaults"] == 1.0
