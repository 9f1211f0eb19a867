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
