"""Plan shape and executor tuning chosen by measurement, and Algorithm 1's
anytime planning loop.

The block size of the elimination steps sets the matrix nodes' shapes (a
step over k variables sums K = 2^k entries), and the tree seed changes the
whole contraction order; which one runs fastest depends on the formula, the
precision and the device.  ``autotune_plan`` builds every candidate plan,
times ``wmc_contract`` on the device and keeps the fastest; a JSON cache
keyed by the formula, the options and the device name makes later calls
build only the winner.  It launches nothing of its own: every candidate runs
through the library's kernels.

``tune_executor`` measures the executor's tuning table (grid caps,
register-tile bits, lane orders, which streaming nodes go to the matrix
cores, summed-index splits) by coordinate descent over representative
plans, and fits per-class execution rates from per-launch timings; the
result is a JSON table keyed by device name (``tuning.json`` beside this
file holds the MI355X one) that ``load_tuning`` installs for plans made
afterwards and that ``time_cost`` reads its rates from.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import Network, Plan, WmcError, tuning_get, tuning_set, wmc_contract, workspace

TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


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
# the launch's node class, plus a fixed cost per launch.  The rates come from
# the tuning table measured on the device (``tune_executor`` fits them to
# per-launch timings); these fallbacks are used only where no table exists.
DEFAULT_RATES = {
    "launch_s": 5e-6,
    0: (0.05e12, 1e12),    # small nodes: launch/latency-bound
    1: (4.0e12, 30e12),    # streaming nodes
    2: (4.4e12, 30e12),    # matrix nodes
}


def _device_name() -> Optional[str]:
    """cuda:0's architecture (e.g. 'gfx950'), the key of the tuning tables."""
    try:
        import torch
        if torch.cuda.is_available():
            prop = torch.cuda.get_device_properties(0)
            arch = getattr(prop, "gcnArchName", "").split(":")[0]
            return arch or prop.name
    except Exception:  # noqa: BLE001 - no device, no table
        return None
    return None


def load_table(path: str = TUNING_PATH, device: Optional[str] = None) -> Optional[Dict]:
    """The tuning table stored for ``device`` (default: cuda:0's
    architecture)."""
    device = device or _device_name()
    if not device or not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get(device)


def load_tuning(path: str = TUNING_PATH, device: Optional[str] = None) -> bool:
    """Install the measured executor tables for ``device`` (default: cuda:0)
    for plans made afterwards.  Returns False when none is stored."""
    t = load_table(path, device)
    if not t:
        return False
    for prec in ("fp64", "fp32"):
        if prec in t:
            tuning_set(prec, t[prec]["table"])
    return True


def measured_rates(precision: str = "fp64", path: str = TUNING_PATH, device: Optional[str] = None) -> Optional[Dict]:
    """Per-class (bandwidth B/s, flop rate) and per-launch cost fitted on the
    device by ``tune_executor``, or None."""
    t = load_table(path, device)
    if not t or precision not in t or "rates" not in t[precision]:
        return None
    r = t[precision]["rates"]
    out = {"launch_s": float(r["launch_s"])}
    for c, v in r["classes"].items():
        out[int(c)] = (float(v[0]), float(v[1]))
    return out


def time_cost(plan, rates: Optional[Dict] = None) -> float:
    """Predicted seconds for one wmc_contract of ``plan`` (all slices).
    ``rates`` defaults to the rates measured on this device for the plan's
    precision (``measured_rates``), else ``DEFAULT_RATES``."""
    from . import plan_launches
    r = dict(DEFAULT_RATES)
    if rates is None:
        rates = measured_rates(plan.precision if plan.precision != "fp32_scaled" else "fp32")
    if rates:
        r.update(rates)
    st = plan.stats()
    b, fl, cls = plan_launches(plan)
    t = 0.0
    for k in range(len(b)):
        c = int(cls[k])
        bw, fr = r.get(c, r[0]) if c >= 0 else (r[0][0], r[0][1])
        t += max(float(b[k]) / bw, float(fl[k]) / fr)
    # a launch covers slice_group slices at once: its fixed cost is paid once
    n_slices, group = st["n_slices"], max(1, st.get("slice_group", 1))
    launches = len(b) * ((n_slices + group - 1) // group)
    return t * n_slices + r["launch_s"] * launches


# ---------------------------------------------------------------------------
# Executor tuning by measurement
# ---------------------------------------------------------------------------
SEARCH_SPACE = {
    "fp64": {"stream2_grid_cap": [2048, 4096, 8192, 16384], "stream_mfma_grid_cap": [1024, 2048, 4096, 8192],
             "stream_mfma_min_bits": [0, 3, 4], "stream2_low_bits": [4, 6, 8], "split_lanes": [0, 4],
             "stream2_tile_bits": [1, 2], "stream2_min_thread_bits": [12, 14, 16],
             "gemm_tpw_max_nt": [0, 1, 2, 4], "gemm_orient": [0, 1, 2], "stream2_vec": [0, 1]},
    "fp32": {"stream2_grid_cap": [768, 1536, 3072, 6144, 12288], "stream_mfma_grid_cap": [1024, 2048, 4096, 8192],
             "stream_mfma_min_bits": [0, 3, 4], "stream2_low_bits": [4, 6, 8], "stream2_tile_bits": [1, 2],
             "stream2_min_thread_bits": [12, 14, 16], "gemm_tpw_max_nt": [0, 1, 2, 4], "gemm_orient": [0, 1, 2],
             "stream2_vec": [0, 1]},
}


def _time_plans(cases, precision: str, reps: int) -> List[float]:
    """Best-of-``reps`` seconds per solve of each case."""
    import torch
    total = []
    for net, kw in cases:
        p = Plan(net, precision=precision, **kw)
        ws = workspace(p)
        wmc_contract(p, None, ws)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            wmc_contract(p, None, ws)
            best = min(best, time.perf_counter() - t0)
        del ws
        total.append(best)
    return total


def _fit_rates(cases, precision: str) -> Dict:
    """Per node class: time = launch cost + bytes / bandwidth (least squares
    over every launch of the cases' profiled solves, HIP-event durations)."""
    from . import plan_launches, wmc_contract_profile
    rows = []
    for net, kw in cases:
        p = Plan(net, precision=precision, **kw)
        ws = workspace(p)
        st = p.stats()
        _, ms = wmc_contract_profile(p, None, ws)
        b, fl, cls = plan_launches(p)
        launches = (st["n_slices"] + max(1, st["slice_group"]) - 1) // max(1, st["slice_group"])
        for k in range(len(b)):
            if cls[k] >= 0 and ms[k] > 0:
                rows.append((int(cls[k]), float(b[k]) * st["n_slices"], float(fl[k]) * st["n_slices"],
                             float(ms[k]) * 1e-3, launches))
        del ws
    out = {"classes": {}}
    launch_s = []
    for c in sorted({r[0] for r in rows}):
        rs = [r for r in rows if r[0] == c]
        A = np.array([[r[4], r[1]] for r in rs])
        y = np.array([r[3] for r in rs])
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        a, inv_bw = float(coef[0]), float(coef[1])
        tot_b, tot_f, tot_t = sum(r[1] for r in rs), sum(r[2] for r in rs), sum(r[3] for r in rs)
        bw = 1.0 / inv_bw if inv_bw > 0 else tot_b / tot_t
        fr = max(tot_f / tot_t, 1e9)
        out["classes"][str(c)] = [bw, fr]
        if a > 0:
            launch_s.append(a)
    out["launch_s"] = float(np.median(launch_s)) if launch_s else DEFAULT_RATES["launch_s"]
    return out


def tune_executor(cases: Sequence[Tuple], precisions: Sequence[str] = ("fp64", "fp32"), reps: int = 3,
                  passes: int = 2, path: Optional[str] = TUNING_PATH, space: Optional[Dict] = None,
                  log=None) -> Dict:
    """Coordinate descent over the executor tuning table: for each field in
    turn every candidate value is installed, the ``cases`` (pairs of a
    ``Network`` and ``Plan`` keyword arguments) are planned and timed, and
    the fastest value is kept; passes repeat until one changes nothing.
    The winning table and rates fitted from per-launch timings are stored
    under the device's name in ``path`` (when given) and left installed."""
    device = _device_name()
    if device is None:
        raise RuntimeError("tune_executor needs a GPU")
    space = space or SEARCH_SPACE
    result = {}
    for prec in precisions:
        tuning_set(prec, None)
        cur = tuning_get(prec)
        # objective: mean over the cases of a candidate's time relative to
        # the current table's, both timed back to back (the device's clocks
        # drift over a tuning run, so a baseline timed once at the start
        # would favour whatever ran first); best_t is the product of the
        # accepted ratios, i.e. the time relative to the built-in table
        base = _time_plans(cases, prec, reps)
        best_t = 1.0
        trace = [{"table": dict(cur), "s": base}]
        for _ in range(passes):
            changed = False
            for field, values in space[prec].items():
                for v in values:
                    if v == cur[field]:
                        continue
                    trial = dict(cur, **{field: v})
                    tuning_set(prec, trial)
                    ts = _time_plans(cases, prec, reps)
                    tuning_set(prec, cur)
                    tb = _time_plans(cases, prec, reps)
                    r = sum(t / b for t, b in zip(ts, tb)) / len(tb)
                    trace.append({field: v, "s": ts, "current": tb})
                    if log:
                        log(f"{prec} {field}={v}: {r:.4f} of the current table "
                            f"[{', '.join(f'{x * 1e3:.2f}' for x in ts)} vs "
                            f"{', '.join(f'{x * 1e3:.2f}' for x in tb)} ms]")
                    if r < 0.995:
                        best_t, cur, changed = best_t * r, trial, True
                tuning_set(prec, cur)
            if not changed:
                break
        tuning_set(prec, cur)
        result[prec] = {"table": cur, "relative_time": best_t, "default_seconds": base,
                        "rates": _fit_rates(cases, prec), "trials": len(trace)}
    entry = {"device": device, **result}
    if path:
        table = {}
        if os.path.exists(path):
            with open(path) as fh:
                table = json.load(fh)
        table[device] = entry
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1)
        os.replace(tmp, path)
    return entry


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
