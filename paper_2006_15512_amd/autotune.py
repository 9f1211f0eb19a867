"""Plan shape chosen by measurement.

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
