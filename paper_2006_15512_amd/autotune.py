"""Plan shape chosen by measurement, and Algorithm 1's anytime planning loop.

The block size of the elimination steps sets the matrix nodes' shapes (a
step over k variables sums K = 2^k entries), and the tree seed changes the
whole contraction order; which one runs fastest depends on the formula, the
precision and the device.  ``autotune_plan`` builds every candidate plan,
times ``wmc_contract`` on the device and keeps the fastest; a JSON cache
keyed by the formula, the options and the device name makes later calls
build only the winner.  It launches nothing of its own: every candidate runs
through the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import Network, Plan, WmcError, wmc_contract, workspace


def _key(f, precision: str, kinds: Sequence[Tuple], rank_cap: int, mem_cap_bytes: int, device: str) -> str:
    h = hashlib.sha256()
    h.update(f"{f.n}|{precision}|{rank_cap}|{mem_cap_bytes}|{device}|{kinds}".encode())
    for c in f.clauses:
        h.update(np.asarray(c, dtype=np.int32).tobytes() + b";")
    return h.hexdigest()[:24]


def autotune_plan(f, precision: str = "fp64", blocks: Sequence[int] = (1, 2, 3, 4, 5, 6),
                  seeds: Sequence[int] = (0,), order: Optional[Sequence[int]] = None, rank_cap: int = 0,
                  mem_cap_bytes: int = 0, reps: int = 3, cache: Optional[str] = None) -> Tuple[Plan, Dict]:
    """Fastest plan of formula ``f`` (a ``wmc_workloads.Formula``-like object
    with n, clauses, weights) among the block sizes ``blocks`` on ``order``
    (or min-fill trees with ``seeds``).  Returns (plan, report);
    report["cached"] is True when the cache decided."""
    import torch
    net = Network.from_formula(f)
    kinds: List[Dict] = []
    for b in blocks:
        if order is not None:
            kinds.append(dict(kind="order", order=list(order), block=int(b)))
        else:
            for s in seeds:
                kinds.append(dict(kind="minfill", seed=int(s), block=int(b)))
    common = dict(precision=precision, rank_cap=rank_cap, mem_cap_bytes=mem_cap_bytes)
    device = torch.cuda.get_device_name(0)
    tag = [[k["kind"], k.get("seed", -1), k["block"]] for k in kinds]
    key = _key(f, precision, tag, rank_cap, mem_cap_bytes, device)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table:
        best = kinds[table[key]["best"]]
        rep = dict(table[key])
        rep["cached"] = True
        return Plan(net, **best, **common), rep
    results = []
    best_i, best_t, best_plan = -1, float("inf"), None
    for i, kw in enumerate(kinds):
        try:
            p = Plan(net, **kw, **common)
        except WmcError as e:
            results.append({"candidate": tag[i], "error": str(e)})
            continue
        ws = workspace(p)
        wmc_contract(p, None, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            wmc_contract(p, None, ws)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        del ws
        results.append({"candidate": tag[i], "ms": round(t * 1e3, 4), "max_rank": p.stats()["max_rank"]})
        if t < best_t:
            best_i, best_t, best_plan = i, t, p
    if best_plan is None:
        raise WmcError(3, "autotune_plan: no candidate plan could be built")
    rep = {"best": best_i, "best_candidate": tag[best_i], "ms": round(best_t * 1e3, 4), "results": results,
           "device": device, "cached": False}
    if cache:
        table[key] = {k: v for k, v in rep.items() if k != "cached"}
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1)
        os.replace(tmp, cache)
    return best_plan, rep


# ---------------------------------------------------------------------------
# Anytime planning (Algorithm 1): generate contraction trees until the chosen
# one's predicted execution time, scaled by the performance factor alpha,
# falls below the time already spent planning.
# ---------------------------------------------------------------------------

# Execution-time model per launch: max(bytes / bandwidth, flops / rate) for
# the launch's node class, plus a fixed launch cost; class rates are the
# achieved figures measured on MI355X (FP64; FP32 moves half the bytes).
DEFAULT_RATES = {
    "launch_s": 5e-6,
    0: (0.05e12, 1e12),    # small nodes: launch/latency-bound
    1: (2.5e12, 30e12),    # streaming nodes
    2: (4.4e12, 30e12),    # matrix nodes
}


def time_cost(plan, rates: Optional[Dict] = None) -> float:
    """Predicted seconds for one wmc_contract of ``plan`` (all slices)."""
    from . import plan_launches
    r = dict(DEFAULT_RATES)
    if rates:
        r.update(rates)
    b, fl, cls = plan_launches(plan)
    t = 0.0
    for k in range(len(b)):
        c = int(cls[k])
        bw, fr = r.get(c, r[0]) if c >= 0 else (r[0][0], r[0][1])
        t += max(float(b[k]) / bw, float(fl[k]) / fr) + r["launch_s"]
    return t * plan.stats()["n_slices"]


def anytime_plan(f, alpha: float, precision: str = "fp64", blocks: Sequence[int] = (1, 2, 3, 4, 5, 6),
                 rank_cap: int = 0, mem_cap_bytes: int = 0, max_candidates: int = 64,
                 rates: Optional[Dict] = None) -> Tuple[Plan, Dict]:
    """Algorithm 1's planning loop: candidate trees (seeded min-fill orders
    with seeds 0, 1, 2, ... at each block size) are generated one after
    another; the best by ``time_cost`` is kept, and planning stops once
    alpha * time_cost(best) < planning time so far (or after
    ``max_candidates``).  Returns (best plan, report)."""
    net = Network.from_formula(f)
    t0 = time.perf_counter()
    best, best_cost, tried, history = None, float("inf"), 0, []
    seed = 0
    while tried < max_candidates:
        for b in blocks:
            if tried >= max_candidates:
                break
            try:
                p = Plan(net, kind="minfill", seed=seed, block=int(b), precision=precision, rank_cap=rank_cap,
                         mem_cap_bytes=mem_cap_bytes)
            except WmcError:
                tried += 1
                continue
            tried += 1
            c = time_cost(p, rates)
            history.append({"seed": seed, "block": int(b), "cost_s": c})
            if c < best_cost:
                best, best_cost = p, c
            if best is not None and alpha * best_cost < time.perf_counter() - t0:
                return best, {"candidates": tried, "plan_seconds": time.perf_counter() - t0,
                              "predicted_seconds": best_cost, "history": history, "stopped": "alpha"}
        seed += 1
    if best is None:
        raise WmcError(3, "anytime_plan: no candidate plan could be built")
    return best, {"candidates": tried, "plan_seconds": time.perf_counter() - t0, "predicted_seconds": best_cost,
                  "history": history, "stopped": "max_candidates"}
