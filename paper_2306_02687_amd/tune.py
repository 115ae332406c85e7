"""Autotuner of the launch variants.

For a plan it times, on the plan's own inputs, every launch variant of
* the tangent contraction (``hrom_eval``: one or two macro points per
  wavefront, occupancy, operand prefetch),
* the kinematics (``hrom_eval``: four or eight wavefronts per 32-point
  workgroup) and
* the register condensation (``hrom_condense``: the register budget of three
  or two wavefronts per SIMD),
and keeps the fastest.  Mixed plans with several clusters launch the tangent
once per cluster, so there its variant is tuned cluster by cluster (the others
held at their current choice) and ``variant`` is the list of per-cluster
choices; the kinematics and condensation variants are always per cluster.
The choice is cached on disk, keyed by GPU architecture, precision, split
flag and the (m, Q, count) of every cluster, so later plans of the same shape
skip the timing.  The cache file is ``$HROM_TUNE_CACHE`` or
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
    return f"v2|{arch}|prec{plan.precision}|split{int(plan.split)}|{shapes}"


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


def _time(fn, reps):
    fn()                                   # warm-up (first launch of the variant)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        fn()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps


def autotune(plan: B.Plan, theta, Fbar, a, reps: int = 3, use_cache: bool = True,
             path: str | None = None) -> dict:
    """Pick the fastest launch variants for ``plan``; returns
    ``{"variant": v, "kin": [..], "cond": [..], "ms": {...}, "cached": bool}``
    (``v``: the tangent variant, a per-cluster list for mixed plans with
    several clusters; ``kin`` and ``cond``: per-cluster kinematics and
    condensation variants)."""
    path = path or cache_path()
    key = plan_key(plan)
    cache = _load_cache(path) if use_cache else {}
    ncl = len(plan.clusters)
    per_cluster = plan.precision != B.FP64 and ncl > 1
    if key in cache:
        e = cache[key]
        v = e["variant"]
        if isinstance(v, list):
            for c, vc in enumerate(v):
                plan.set_variant(int(vc), c)
        else:
            v = int(v)
            plan.set_variant(v)
        for c in range(ncl):
            plan.set_kernel_variant(B.VK_KIN, int(e["kin"][c]), c)
            plan.set_kernel_variant(B.VK_CONDENSE, int(e["cond"][c]), c)
        return {"variant": v, "kin": e["kin"], "cond": e["cond"], "ms": e.get("ms", {}),
                "cached": True}
    status = plan.status()

    def evaluate():
        plan.eval(theta, Fbar, a, status)

    def sweep(set_fn, n, fn):
        times = {}
        for v in range(n):
            set_fn(v)
            times[v] = _time(fn, reps)
        best = min(times, key=times.get)
        set_fn(best)
        return best, times

    ms = {}
    if per_cluster:
        best = []
        for c in range(ncl):
            b, t = sweep(lambda v, c=c: plan.set_variant(v, c), B.Plan.num_variants(), evaluate)
            best.append(b)
            ms[f"tangent{c}"] = t
    else:
        best, ms["tangent"] = sweep(lambda v: plan.set_variant(v, -1), B.Plan.num_variants(), evaluate)
    kin, cond = [], []
    for c in range(ncl):
        b, ms[f"kin{c}"] = sweep(lambda v, c=c: plan.set_kernel_variant(B.VK_KIN, v, c),
                                 B.Plan.num_kernel_variants(B.VK_KIN), evaluate)
        kin.append(b)
    evaluate()
    Pb, Cb = plan.zeros_points(9), plan.zeros_points(81)
    rn = torch.zeros(Fbar.shape[1], dtype=torch.float64, device=Fbar.device)
    for c in range(ncl):
        b, ms[f"cond{c}"] = sweep(lambda v, c=c: plan.set_kernel_variant(B.VK_CONDENSE, v, c),
                                  B.Plan.num_kernel_variants(B.VK_CONDENSE),
                                  lambda: plan.condense(Pb, Cb, rn, status))
        cond.append(b)
    if use_cache:
        cache[key] = {"variant": best, "kin": kin, "cond": cond,
                      "ms": {k: {str(i): x for i, x in t.items()} for k, t in ms.items()}}
        _store_cache(path, cache)
    return {"variant": best, "kin": kin, "cond": cond, "ms": ms, "cached": False}
