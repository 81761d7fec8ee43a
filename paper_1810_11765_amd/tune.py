"""Autotuner for launch shapes: the per-heap smmo_launch fields, the batch
grid (workgroups per CU) and the steps per batched launch.

The paper leaves the do-all's thread count to hand tuning (Sec. 3.7).  Here a
search measures candidate shapes on the caller's own workload, rejects every
candidate whose result differs from the default shape's (a launch shape must
never change results), and keeps the fastest; records are cached in a JSON
file per (device architecture, workload key).

The search is coordinate descent: start from the defaults (the first value of
every knob), try each value of one knob with the others fixed at the best so
far, move to the next knob, and repeat the pass while it still improves
(at most `passes` passes).  Each candidate is timed `reps` times and the
median is kept.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Any, Callable


def device_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", None) or p.name


def search(measure: Callable[[dict], tuple[float, Any]], space: dict[str, list], reps: int = 3,
           equal: Callable[[Any, Any], bool] | None = None, passes: int = 2) -> dict:
    """measure(cfg) -> (seconds, result) runs the workload once with the knob
    values of `cfg`; space maps each knob to its candidate values, the first
    being the default.  equal(default_result, result) decides whether a
    candidate computed the same thing (None: accept all).  Returns the best
    and default configurations with their median times and every trial."""
    default = {k: v[0] for k, v in space.items()}
    trials: list[dict] = []
    seen: dict[tuple, float | None] = {}

    def timed(cfg: dict, ref=None):
        key = tuple(sorted(cfg.items()))
        if key in seen:
            return seen[key], None
        times, result = [], None
        for _ in range(reps):
            t, result = measure(dict(cfg))
            times.append(t)
        med = statistics.median(times)
        ok = True if (equal is None or ref is None) else bool(equal(ref, result))
        trials.append({"cfg": dict(cfg), "median_s": med, "times_s": times, "same_result": ok})
        seen[key] = med if ok else None
        return seen[key], result

    t0, ref = timed(default)
    best, best_t = dict(default), t0
    for _ in range(passes):
        improved = False
        for knob, values in space.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = dict(best)
                cand[knob] = v
                t, _ = timed(cand, ref)
                if t is not None and t < best_t:
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    return {"default": default, "default_s": t0, "best": best, "best_s": best_t,
            "speedup": (t0 / best_t) if best_t else None, "trials": trials}


def save(path: str, key: str, record: dict) -> None:
    """Store `record` under (device architecture, key) in the JSON cache."""
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(device_arch(), {})[key] = record
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, path)


def load(path: str, key: str) -> dict | None:
    """The best configuration cached for this device and key, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(device_arch(), {}).get(key)
    return None if rec is None else rec.get("best")
