"""The committed counter summaries: every traffic entry names an existing
profile summary, kernels the library has, and positive byte counts; the
bench reads an entry only while the kernel sources match its digest, and
only for the contraction tree (min-fill seed) it was taken on."""
import json
import os

import bench
import paper_2006_15512_amd as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_entries_are_well_formed():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    assert data
    for key, ent in data.items():
        wname, prec, blk = key.split("/")
        assert prec in ("fp64", "fp32") and blk.startswith("block")
        bench.workload(wname)
        assert os.path.exists(os.path.join(ROOT, ent["profile"]))
        assert 1.5 < ent["fetch_scale"] < 2.5 and 0.5 < ent["write_scale"] < 1.5
        for kn, b in ent["hbm_bytes_per_launch"].items():
            assert kn in W.KERNEL_NAMES and b > 0
        seed = ent.get("tree_seed")
        got = bench.traffic_for(wname, prec, int(blk[5:]), "k_begin", seed)
        if ent["kernel_sources"] == bench.source_digest():
            assert got == ent["hbm_bytes_per_launch"]["k_begin"]
            # another tree of the same workload reads no entry
            other = (seed or 0) + 1
            assert bench.traffic_for(wname, prec, int(blk[5:]), "k_begin", other) is None
        else:
            assert got is None


def test_headline_tree_is_the_least_time_cost_seed():
    """The banded formula's benchmark plan is the min-fill tree whose seed,
    among the candidates, has the least TimeCost; the seed-0 comparison
    plans exactly seed 0; both meet the rank cap (host only: no device
    timing enters the choice)."""
    from paper_2006_15512_amd.autotune import time_cost
    f, pkw, _, _ = bench.workload("banded300")
    pkw = dict(pkw)
    blk = pkw.pop("block")
    plan, tree = bench.make_plan(W, f, "fp64", blk, pkw)
    assert tree["candidates"] == pkw["tree_seeds"]
    net = W.Network.from_formula(f)
    opts = {k: v for k, v in pkw.items() if k != "tree_seeds"}
    costs = [time_cost(W.Plan(net, precision="fp64", block=blk, seed=s, **opts)) for s in range(tree["candidates"])]
    assert tree["seed"] == min(range(len(costs)), key=costs.__getitem__)
    assert plan.stats()["max_rank"] <= pkw["rank_cap"] and plan.n_slices == tree["n_slices"]
    fixed = dict(opts, seed=0)
    p0, t0 = bench.make_plan(W, f, "fp64", blk, fixed)
    assert t0 is None and p0.stats()["max_rank"] <= pkw["rank_cap"]
    assert p0.n_slices >= plan.n_slices
