"""Autotuner of the launch shapes (spalu_tuning) for one workload.

A coordinate search: starting from the library's defaults, each field in
turn takes each of its candidate values with the others at the best set so
far, and a value is kept when the median time of a factorization plus the
refined solve drops by more than 1 %.  A candidate whose solve does not
converge counts as infinitely slow.  Results go to a JSON cache keyed by the
device and the workload (grid, storage precision, predictor, right-hand
sides, tolerance), which `apply_cached` reads back.
"""
from __future__ import annotations

import json
import os
import statistics
import time

from . import spalu as S

# candidate values per field, the default first
SPACE = [
    ("id_lds_c", [155648, 114688, 81920, 65536]),
    ("id_c_ydiv", [2, 1, 4]),
    ("id_lds_b2", [155648, 114688, 81920]),
    ("id_lds_b", [73728, 49152, 98304]),
    ("id_lds_a", [24576, 16384, 32768]),
    ("melim_lds", [65536, 32768, 98304]),
    ("melim_wave_cap", [32, 16]),
    ("solve_lanes_min", [8, 16]),
    ("solve_lanes_max", [64, 32]),
]

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def device_name():
    """The GPU architecture (the marketing name is not reported on every
    machine, the architecture is)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "") or p.name


def workload_key(dims, precision, learned, nrhs, eps, device=None, symmetric=False):
    return "%s | grid %s | %s | %s | nrhs %d | eps %g%s" % (
        device or device_name(), "x".join(str(int(d)) for d in dims), "fp32" if precision == S.FP32 else "fp64",
        "learned" if learned else "adaptive", int(nrhs), float(eps), " | symmetric" if symmetric else "")


def load_cache(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply_cached(key, path=CACHE):
    """Sets the cached launch shapes of this workload; returns them, or None
    (defaults kept) when the cache has no entry."""
    ent = load_cache(path).get(key)
    if ent is None:
        return None
    return S.set_tuning(**ent["tuning"])


def tune(run, key, reps=3, path=CACHE, log=print):
    """run() performs one factorization + refined solve and returns
    (seconds, converged).  Leaves the best shapes set, stores them under key
    and returns them."""
    def timed(t):
        S.set_tuning(**t)
        run()                       # a first run re-plans the tiers
        ts = []
        for _ in range(reps):
            sec, ok = run()
            ts.append(sec if ok else float("inf"))
        return statistics.median(ts)

    best = S.tuning_default()
    best_s = timed(best)
    default_s = best_s
    trials = [dict(tuning=dict(best), ms=best_s * 1e3)]
    log("autotune %s: defaults %.2f ms" % (key, best_s * 1e3))
    for field, values in SPACE:
        for v in values:
            if v == best[field]:
                continue
            cand = dict(best)
            cand[field] = v
            try:
                s = timed(cand)
            except S.SpaluError as e:        # refused combination
                log("  %s=%d refused: %s" % (field, v, e))
                continue
            trials.append(dict(tuning=dict(cand), ms=s * 1e3))
            log("  %s=%d: %.2f ms" % (field, v, s * 1e3))
            if s < best_s * 0.99:
                best, best_s = cand, s
    S.set_tuning(**best)
    cache = load_cache(path)
    cache[key] = dict(tuning=best, ms=round(best_s * 1e3, 3), default_ms=round(default_s * 1e3, 3),
                      reps=reps, trials=trials, when=time.strftime("%Y-%m-%d %H:%M:%S"))
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    log("autotune %s: best %.2f ms (defaults %.2f ms): %s" % (key, best_s * 1e3, default_s * 1e3,
                                                             {k: v for k, v in best.items()
                                                              if v != S.tuning_default()[k]}))
    return best
