"""Write tests/golden/oracle_values.json: oracle results for the full-size
workloads that the oracle cannot recompute within a test's time budget.

Calls only the CPU oracle (O2, FP64 bucket elimination with a carried
power-of-two exponent) on inputs from the seeded generators; nothing here
touches the GPU library.  Usage:

    python tests/golden/make_golden.py [name ...]
    python tests/golden/make_golden.py batch512
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import wmc_workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")


def cases():
    """name -> (formula factory, elimination order factory or None, description)."""
    return {
        "grid24x24_t0.10_s0": (lambda: wl.grid_cnf(24, 24, 0.10, seed=0),
                               lambda f: wl.row_major_order(24, 24),
                               "grid_cnf(24, 24, 0.10, seed=0), planted signs; row-major order"),
        "grid12x24_t0.10_s1": (lambda: wl.grid_cnf(12, 24, 0.10, seed=1),
                               lambda f: wl.row_major_order(12, 24),
                               "grid_cnf(12, 24, 0.10, seed=1), planted signs; row-major order"),
        "banded300_m1050_W37_s0": (lambda: wl.banded_3cnf(300, 1050, 37, seed=0), None,
                                   "banded_3cnf(300, 1050, window 37, seed=0); oracle min-fill order"),
    }


BATCH_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512_oracle.json")


def make_batch512():
    """Oracle values of all 512 instances of the batch recipe
    (`wmc_workloads.batch_instance(i)`, oracle min-fill order)."""
    t0 = time.time()
    rows = []
    for i in range(512):
        f = wl.batch_instance(i)
        m, e = oracle.bucket(f)
        rows.append({"i": i, "digest": f.digest(), "n": f.n, "m": f.m, "mantissa_hex": float(m).hex(),
                     "exp2": int(e)})
    with open(BATCH_OUT, "w") as fh:
        json.dump({"description": "batch_instance(i), i < 512; oracle bucket elimination (FP64, carried exponent)",
                   "instances": rows}, fh, indent=0)
    print("batch512", f"{time.time() - t0:.1f}s", sum(1 for r in rows if float.fromhex(r["mantissa_hex"]) == 0.0),
          "zero", flush=True)


def main(names):
    if names == ["batch512"]:
        make_batch512()
        return
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    all_cases = cases()
    for name in names or list(all_cases):
        make, order_of, desc = all_cases[name]
        f = make()
        order = order_of(f) if order_of else None
        t0 = time.time()
        m, e, width = oracle.bucket(f, order=order, max_log2=31, return_width=True)
        dt = time.time() - t0
        data[name] = {"description": desc, "digest": f.digest(), "n": f.n, "m": f.m,
                      "mantissa_hex": float(m).hex(), "mantissa": m, "exp2": int(e), "width": int(width),
                      "oracle": "bucket elimination (FP64, carried exponent)", "seconds": round(dt, 1),
                      "threads": os.environ.get("OMP_NUM_THREADS", str(os.cpu_count()))}
        print(name, m, e, width, f"{dt:.1f}s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
