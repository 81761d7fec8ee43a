"""Host logic of the launch-shape autotuner (no GPU): the search finds the
fastest configuration by coordinate descent, never picks one whose result
differs from the default's, and the cache round-trips per device."""
from paper_1810_11765_amd import tune


def test_coordinate_descent_finds_separable_minimum():
    calls = []

    def measure(cfg):
        calls.append(dict(cfg))
        t = (cfg["a"] - 3) ** 2 + (cfg["b"] - 1) ** 2 + 1.0
        return t, "same"
    rec = tune.search(measure, {"a": [0, 1, 2, 3, 4], "b": [5, 1, 2]}, reps=1, equal=lambda x, y: x == y)
    assert rec["best"] == {"a": 3, "b": 1}
    assert rec["default"] == {"a": 0, "b": 5} and rec["speedup"] == rec["default_s"] / rec["best_s"]
    assert all(t["same_result"] for t in rec["trials"])
    assert len({tuple(sorted(c.items())) for c in calls}) == len(calls)   # no configuration timed twice


def test_candidates_with_a_different_result_are_rejected():
    def measure(cfg):
        # the fastest value computes something else: it must not be chosen
        return {0: 5.0, 1: 1.0, 2: 3.0}[cfg["k"]], ("wrong" if cfg["k"] == 1 else "right")
    rec = tune.search(measure, {"k": [0, 1, 2]}, reps=3, equal=lambda a, b: a == b)
    assert rec["best"] == {"k": 2}
    bad = [t for t in rec["trials"] if not t["same_result"]]
    assert len(bad) == 1 and bad[0]["cfg"] == {"k": 1}


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "device_arch", lambda: "gfxTEST")
    path = str(tmp_path / "tuned.json")
    assert tune.load(path, "w") is None
    tune.save(path, "w", {"best": {"x": 1}, "trials": []})
    tune.save(path, "v", {"best": {"y": 2}, "trials": []})
    assert tune.load(path, "w") == {"x": 1} and tune.load(path, "v") == {"y": 2}
    monkeypatch.setattr(tune, "device_arch", lambda: "gfxOTHER")
    assert tune.load(path, "w") is None
