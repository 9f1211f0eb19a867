"""GPU tests of batched execution (many plans in shared launches)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def frac(v):
    return Fraction(0) if v.mantissa == 0.0 else Fraction(v.mantissa) * Fraction(2) ** v.exp2


def rel(a, b):
    return 0.0 if a == b else float(abs(a - b) / max(abs(a), abs(b)))


@pytest.fixture(scope="module")
def instances():
    fs = [wl.batch_instance(i) for i in range(64)]
    refs = []
    for f in fs:
        m, e = oracle.bucket(f)
        refs.append(Fraction(m) * Fraction(2) ** e)
    return fs, refs


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch_instances_vs_oracle(instances, precision, tol):
    """64 instances of the 512-instance batch recipe (n 30-150, ratio
    3.0-4.2, banded window 20) in one batch, against the oracle."""
    fs, refs = instances
    say(f"batch64 {precision}")
    plans = [W.Plan(W.Network.from_formula(f), seed=i, precision=precision) for i, f in enumerate(fs)]
    b = W.Batch(plans)
    vals = b.contract()
    for i, (v, r) in enumerate(zip(vals, refs)):
        got = frac(v)
        assert (got == 0) if r == 0 else rel(got, r) <= tol, i


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch_equals_solo_bit_exact(instances, precision, tol):
    """Every instance's value in the batch is bit-identical to the same
    instance in a batch of its own (the per-node reduction order does not
    depend on the batch composition), in both precisions, and equals its
    solo wmc_contract: bit for bit in FP64, within the FP32 tolerance in
    scaled FP32 (the solo executor may pick another kernel family)."""
    fs, _ = instances
    plans = [W.Plan(W.Network.from_formula(f), seed=i, block=1 + i % 3, precision=precision)
             for i, f in enumerate(fs[:24])]
    vals = W.Batch(plans).contract()
    for i, p in enumerate(plans):
        say(f"solo {precision} {i}")
        (own,) = W.Batch([p]).contract()
        assert (own.mantissa, own.exp2) == (vals[i].mantissa, vals[i].exp2), i
        solo = W.wmc_contract(p)
        if precision == "fp64":
            assert (solo.mantissa, solo.exp2) == (vals[i].mantissa, vals[i].exp2), i
        else:
            assert rel(frac(solo), frac(vals[i])) <= tol, i


def test_batch_graph_replays_match_eager(instances):
    """Graph capture: replay several times, with eager work in between; every
    replay equals the eager result; resident descriptors are reused."""
    import torch
    fs, _ = instances
    plans = [W.Plan(W.Network.from_formula(f), seed=i) for i, f in enumerate(fs[:32])]
    b = W.Batch(plans)
    ws = b.workspace()
    eager = b.contract(ws=ws)
    rng = np.random.default_rng(0)
    for rep in range(4):
        say(f"graph replay {rep}")
        flags = W.BATCH_GRAPH | (W.BATCH_RESIDENT if rep else 0)
        got = b.contract(ws=ws, flags=flags)
        assert [(v.mantissa, v.exp2) for v in got] == [(v.mantissa, v.exp2) for v in eager]
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert float(x.sum()) == float(x.sum())
        _ = W.wmc_contract(plans[rep])
    # new weights through the same graph (weights are uploaded before each replay)
    w = []
    refs = []
    for f in fs[:32]:
        ww = rng.uniform(0.1, 0.9, size=f.n)
        Wt = np.stack([1 - ww, ww], axis=1)
        w.append(Wt.reshape(-1))
        m, e = oracle.bucket(f.with_weights(Wt))
        refs.append(Fraction(m) * Fraction(2) ** e)
    got = b.contract(np.concatenate(w), ws=ws, flags=W.BATCH_GRAPH | W.BATCH_RESIDENT)
    for v, r in zip(got, refs):
        assert (frac(v) == 0) if r == 0 else rel(frac(v), r) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch_mixes_sliced_and_unsliced_plans(instances, precision, tol):
    """Sliced plans (slices of uneven size: different slice counts and
    sliced variables) batched with unsliced ones: every result against the
    oracle, and each sliced plan's result equal to its solo wmc_contract (bit
    for bit in FP64; the slices are summed in the same order with the same
    compensated arithmetic)."""
    fs, refs = instances
    plans, want = [], []
    for i, f in enumerate(fs[:12]):
        r0 = W.Plan(W.Network.from_formula(f), seed=i).stats()["max_rank"]
        cap = r0 - 1 - i % 3 if i % 3 else 0
        plans.append(W.Plan(W.Network.from_formula(f), seed=i, rank_cap=cap, precision=precision))
        want.append(refs[i])
    ns = [p.n_slices for p in plans]
    assert max(ns) >= 8 and min(ns) == 1 and len(set(ns)) >= 3
    say(f"sliced batch {precision}: slices {ns}")
    b = W.Batch(plans)
    for flags in (0, W.BATCH_GRAPH, W.BATCH_GRAPH | W.BATCH_RESIDENT):
        vals = b.contract(flags=flags)
        for i, (v, r) in enumerate(zip(vals, want)):
            got = frac(v)
            assert (got == 0) if r == 0 else rel(got, r) <= tol, (i, ns[i])
    for i, p in enumerate(plans):
        solo = W.wmc_contract(p)
        if precision == "fp64":
            assert (solo.mantissa, solo.exp2) == (vals[i].mantissa, vals[i].exp2), i
        else:
            assert rel(frac(solo), frac(vals[i])) <= tol, i


def test_batch_workspace_too_small(instances):
    import torch
    fs, _ = instances
    b = W.Batch([W.Plan(W.Network.from_formula(fs[0]))])
    ws = torch.empty(b.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(W.WmcError) as e:
        b.contract(ws=ws)
    assert e.value.status == 2


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch512_all_instances_vs_stored_oracle(precision, tol):
    """Every instance of the 512-instance batch in one batch against the
    oracle values stored by tests/golden/make_golden.py (half the recipe's
    instances are unsatisfiable: those must come back exactly 0)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch512_oracle.json")
    with open(path) as fh:
        rows = json.load(fh)["instances"]
    fs = [wl.batch_instance(i) for i in range(512)]
    for f, r in zip(fs, rows):
        assert f.digest() == r["digest"]
    plans = [W.Plan(W.Network.from_formula(f), seed=i, precision=precision) for i, f in enumerate(fs)]
    b = W.Batch(plans)
    say(f"batch512 {precision}: {b.n_launches} launches")
    vals = b.contract(flags=W.BATCH_GRAPH)
    zeros = 0
    for q, (v, r) in enumerate(zip(vals, rows)):
        ref = Fraction(float.fromhex(r["mantissa_hex"])) * Fraction(2) ** r["exp2"]
        if ref == 0:
            zeros += 1
            assert v.mantissa == 0.0, q
        else:
            assert rel(frac(v), ref) <= tol, q
    assert zeros == sum(1 for r in rows if float.fromhex(r["mantissa_hex"]) == 0.0)


def test_batch_long_clauses_with_new_weights():
    """Instances with factored long clauses in one batch; caller weights
    (2n per instance) are expanded with the auxiliary variables' (1, 1)."""
    fs = [wl.random_long(s) for s in range(10)] + [wl.batch_instance(i) for i in range(6)]
    plans = [W.Plan(W.Network.from_formula(f), seed=i) for i, f in enumerate(fs)]
    b = W.Batch(plans)
    rng = np.random.default_rng(11)
    news = []
    for f in fs:
        w = rng.uniform(0.1, 0.9, size=f.n)
        news.append(np.stack([1 - w, w], axis=1))
    for flags in (0, W.BATCH_GRAPH):
        vals = b.contract(np.concatenate([x.reshape(-1) for x in news]), flags=flags)
        for q, (f, Wt, v) in enumerate(zip(fs, news, vals)):
            m, e = oracle.bucket(f.with_weights(Wt))
            assert rel(frac(v), Fraction(m) * Fraction(2) ** e) <= 1e-12, q


def test_batch_with_big_nodes_vs_oracle():
    """Instances whose merged steps hold nodes of 2^20+ outputs next to small
    ones, against the oracle; batch equals solo bit for bit."""
    fs = [wl.banded_3cnf(120, 400, 24, seed=s) for s in range(3)] + [wl.batch_instance(i) for i in range(5)]
    plans = [W.Plan(W.Network.from_formula(f), seed=s) for s, f in enumerate(fs)]
    b = W.Batch(plans)
    for flags in (0, W.BATCH_GRAPH):
        vals = b.contract(flags=flags)
        for q, (f, p, v) in enumerate(zip(fs, plans, vals)):
            m, e = oracle.bucket(f)
            assert rel(frac(v), Fraction(m) * Fraction(2) ** e) <= 1e-12, q
            solo = W.wmc_contract(p)
            assert (solo.mantissa, solo.exp2) == (v.mantissa, v.exp2), q


def test_batch_resident_flag_on_a_new_workspace():
    """The first call of a batch on a workspace uploads the descriptors even
    when the caller passes RESIDENT (they cannot be there yet), with or
    without graph replay, and so does the first call on a second workspace:
    every result equals the solo one bit for bit (FP64)."""
    import torch
    fs = [wl.batch_instance(i) for i in range(4)]
    plans = [W.Plan(W.Network.from_formula(f), seed=i) for i, f in enumerate(fs)]
    solo = [W.wmc_contract(p) for p in plans]
    b = W.Batch(plans)
    for flags in (W.BATCH_RESIDENT, W.BATCH_GRAPH | W.BATCH_RESIDENT):
        for _ in range(2):  # a fresh workspace each time
            ws = b.workspace()
            ws.zero_()
            torch.cuda.synchronize()
            for rep in range(2):
                got = b.contract(ws=ws, flags=flags)
                for g, s in zip(got, solo):
                    assert (g.mantissa, g.exp2) == (s.mantissa, s.exp2), (flags, rep)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_persistent_equals_launch_per_step(instances, precision):
    """The persistent form (every merged step in one cooperative launch)
    gives the launch-per-step results bit for bit, for unsliced and sliced
    instances, on a first and a second workspace, with RESIDENT, and after
    the workspace was overwritten (a call without RESIDENT); a batch with
    matrix nodes, which runs the launch-per-step form under the flag, too."""
    fs, _ = instances
    plans = [W.Plan(W.Network.from_formula(f), seed=i, precision=precision) for i, f in enumerate(fs)]
    for i, f in enumerate(fs[:6]):
        r0 = W.Plan(W.Network.from_formula(f), seed=i).stats()["max_rank"]
        plans.append(W.Plan(W.Network.from_formula(f), seed=i, rank_cap=r0 - 2, precision=precision))
    b = W.Batch(plans)
    want = [(v.mantissa, v.exp2) for v in b.contract()]
    for k in range(2):
        ws = b.workspace()
        for flags in (W.BATCH_PERSISTENT, W.BATCH_PERSISTENT | W.BATCH_RESIDENT,
                      W.BATCH_PERSISTENT | W.BATCH_GRAPH | W.BATCH_RESIDENT):
            say(f"persistent {precision} workspace {k} flags {flags}")
            got = b.contract(ws=ws, flags=flags)
            assert [(v.mantissa, v.exp2) for v in got] == want, (k, flags)
    # without RESIDENT the step arguments go up again with the descriptors
    ws.zero_()
    got = b.contract(ws=ws, flags=W.BATCH_PERSISTENT)
    assert [(v.mantissa, v.exp2) for v in got] == want
    big = [wl.banded_3cnf(120, 400, 24, seed=0)] + [wl.batch_instance(i) for i in range(3)]
    bb = W.Batch([W.Plan(W.Network.from_formula(f), seed=s, precision=precision) for s, f in enumerate(big)])
    say(f"persistent {precision} with matrix nodes")
    want = [(v.mantissa, v.exp2) for v in bb.contract()]
    assert [(v.mantissa, v.exp2) for v in bb.contract(flags=W.BATCH_PERSISTENT)] == want


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_persistent_degenerate_instances(precision):
    """The persistent form on batches whose plans have few or no node
    launches (a single clause, a formula with an empty clause, a variable
    in no clause, one tiny random formula): every value equals the
    launch-per-step result bit for bit and the oracle's."""
    from wmc_workloads import Formula
    fs = [Formula(1, [[1]], np.array([[0.3, 0.7]])),
          Formula(2, [[1, -2], []], np.array([[0.4, 0.6], [0.2, 0.8]])),
          Formula(3, [[1, 2]], np.array([[0.5, 0.5], [0.1, 0.9], [0.25, 0.75]])),
          wl.random_kcnf(6, 10, 3)]
    for group in ([fs[0]], [fs[1]], fs[:3], fs):
        plans = [W.Plan(W.Network.from_formula(f), precision=precision) for f in group]
        b = W.Batch(plans)
        want = b.contract()
        got = b.contract(flags=W.BATCH_PERSISTENT)
        assert [(v.mantissa, v.exp2) for v in got] == [(v.mantissa, v.exp2) for v in want]
        for f, v in zip(group, got):
            ref = Fraction(oracle.brute(f))
            assert (frac(v) == 0) if ref == 0 else rel(frac(v), ref) <= (1e-12 if precision == "fp64" else 1e-5)
