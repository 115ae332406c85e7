"""Autotuner of the tangent-contraction launch variants.

For a plan it times every launch variant of ``hrom_eval`` (kinematics plus
tangent contraction) on the plan's own inputs and keeps the fastest.  Mixed
plans with several clusters launch the tangent once per cluster, so there the
variant is tuned cluster by cluster (the others held at their current
choice) and ``variant`` is the list of per-cluster choices.  The
choice is cached on disk, keyed by GPU architecture, precision, split flag and
the (m, Q, count) of every cluster, so later plans of the same shape skip the
timing.  The cache file is ``$HROM_TUNE_CACHE`` or
``~/.cache/hrom/tune.json``.  Variants never change results (same arithmetic,
same order), only speed.
"""
from __future__ import annotations

import json
import os

import torch

from . import binding as B


def cache_path() -> str:
    return os.environ.get("HROM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hrom", "tune.json"))


def plan_key(plan: B.Plan) -> str:
    arch = torch.cuda.get_device_properties(plan._dev()).gcnArchName.split(":")[0]
    shapes = ",".join(f"{c.m}x{c.Q}x{c.count}" for c in plan.clusters)
    return f"{arch}|prec{plan.precision}|split{int(plan.split)}|{shapes}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(plan: B.Plan, theta, Fbar, a, reps: int = 3, use_cache: bool = True,
             path: str | None = None) -> dict:
    """Pick the fastest launch variant for ``plan``; returns
    ``{"variant": v, "ms": {v: ms, ...}, "cached": bool}`` (mixed plans with
    several clusters: ``v`` is the list of per-cluster variants and ``ms``
    maps each cluster to its sweep)."""
    path = path or cache_path()
    key = plan_key(plan)
    cache = _load_cache(path) if use_cache else {}
    per_cluster = plan.precision != B.FP64 and len(plan.clusters) > 1
    if key in cache:
        v = cache[key]["variant"]
        if isinstance(v, list):
            for c, vc in enumerate(v):
                plan.set_variant(int(vc), c)
        else:
            v = int(v)
            plan.set_variant(v)
        return {"variant": v, "ms": cache[key].get("ms", {}), "cached": True}
    status = plan.status()

    def sweep(cluster):
        times = {}
        for v in range(B.Plan.num_variants()):
            plan.set_variant(v, cluster)
            plan.eval(theta, Fbar, a, status)       # warm-up (first launch of the variant)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(reps):
                plan.eval(theta, Fbar, a, status)
            ev[1].record()
            torch.cuda.synchronize()
            times[v] = ev[0].elapsed_time(ev[1]) / reps
        best = min(times, key=times.get)
        plan.set_variant(best, cluster)
        return best, times

    if per_cluster:
        best, times = [], {}
        for c in range(len(plan.clusters)):
            b, t = sweep(c)
            best.append(b)
            times[c] = t
    else:
        best, times = sweep(-1)
    if use_cache:
        ms = ({str(c): {str(k): x for k, x in t.items()} for c, t in times.items()} if per_cluster
              else {str(k): x for k, x in times.items()})
        cache[key] = {"variant": best, "ms": ms}
        _store_cache(path, cache)
    return {"variant": best, "ms": times, "cached": False}
