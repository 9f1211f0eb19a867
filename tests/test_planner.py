"""Host-side tests of the reduction and the planner (no GPU needed).

The plans' device descriptors are replayed on the CPU by the kernel emulator
(tests/plan_emulator.py) and the result is compared with the oracle.  This
covers the tree construction, variable closure, tied storage modes, index
slicing, layouts, bit-extraction run lists and arena placement before any
kernel runs.  The GPU parity tests then check the kernels themselves.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl
from wmc_workloads import Formula
from plan_emulator import emulate, rel_err, parse

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(W.LIB_PATH), reason="libwmc.so not built")


def ref_fraction(f):
    if f.n <= 20:
        return Fraction(oracle.brute(f))
    m, e = oracle.bucket(f)
    return Fraction(m) * Fraction(2) ** e


def random_parent(f, seed):
    """A uniformly random merge order over the n+m leaves, as a parent array
    in the ABI's numbering (A_x first, then B_C, then internal vertices)."""
    rng = np.random.default_rng(seed)
    L = f.n + f.m
    parent = np.full(2 * L - 1, -1, dtype=np.int64)
    roots = list(range(L))
    nxt = L
    while len(roots) > 1:
        i, j = sorted(rng.choice(len(roots), size=2, replace=False))
        a, b = roots[i], roots[j]
        parent[a] = parent[b] = nxt
        roots.pop(j)
        roots[i] = nxt
        nxt += 1
    return parent


# --------------------------------------------------------------- reduction
def test_fig1_network_info():
    """Figure 1: 8 tensors and 10 indices."""
    net = W.Network.from_formula(wl.fig1_formula())
    assert net.info() == {"n_tensors": 8, "n_indices": 10}


def test_network_info_counts_distinct_incidences():
    f = Formula(3, [[1, 1, 2], [2, -2, 3], [-3]], np.ones((3, 2)))
    assert W.Network.from_formula(f).info() == {"n_tensors": 6, "n_indices": 5}


@pytest.mark.parametrize("clauses,n,weights,status", [
    ([[4]], 3, None, 1),                  # literal out of range
    ([[0, 1]], 3, None, 1),               # zero literal
    ([[1]], 1, [[np.nan, 1.0]], 1),       # NaN weight
    ([[1]], 1, [[np.inf, 1.0]], 1),       # Inf weight
])
def test_build_network_errors(clauses, n, weights, status):
    w = np.ones((n, 2)) if weights is None else np.array(weights)
    with pytest.raises(W.WmcError) as e:
        W.Network(n, clauses, w)
    assert e.value.status == status


def test_plan_errors():
    f = wl.random_kcnf(10, 20, 1)
    net = W.Network.from_formula(f)
    with pytest.raises(W.WmcError) as e:
        W.Plan(net, kind="order", order=[1, 2, 3])
    assert e.value.status == 1
    with pytest.raises(W.WmcError) as e:
        W.Plan(net, kind="order", order=[1] * 10)
    assert e.value.status == 1
    bad = random_parent(f, 0)
    bad[0] = bad[1]
    bad[2] = -1
    with pytest.raises(W.WmcError) as e:
        W.Plan(net, kind="explicit", parent=bad)
    assert e.value.status == 1
    with pytest.raises(W.WmcError) as e:
        W.Plan(net, kind="explicit", parent=random_parent(f, 0)[:-1])
    assert e.value.status == 1


# --------------------------------------------------------------- plans replayed on the CPU
@pytest.mark.parametrize("kind", ["minfill", "order", "explicit"])
def test_emulated_plans_match_oracle(kind):
    """Every tree kind, replayed from its descriptors, equals the oracle."""
    rng = np.random.default_rng(1)
    for s in range(60):
        f = wl.random_mixed(s, n_max=12, m_max=24)
        net = W.Network.from_formula(f)
        if kind == "minfill":
            p = W.Plan(net, seed=s)
        elif kind == "order":
            p = W.Plan(net, kind="order", order=rng.permutation(f.n) + 1, block=int(rng.integers(1, 4)))
        else:
            p = W.Plan(net, kind="explicit", parent=random_parent(f, s))
        got, _ = emulate(p, f.weights)
        ref = ref_fraction(f)
        if ref == 0:
            assert got == 0, s
        else:
            assert rel_err(got, ref) < 1e-12, (s, float(got), float(ref))


def test_emulated_negative_weights():
    for s in range(30):
        f = wl.random_mixed(s, n_max=10, m_max=16, negative=True)
        p = W.Plan(W.Network.from_formula(f), seed=s)
        got, _ = emulate(p, f.weights)
        ref = Fraction(oracle.brute(f))
        scale = float(np.prod(np.abs(f.weights).sum(axis=1)))
        assert abs(float(got - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("block", [1, 2, 5])
def test_emulated_grid_sweep(block):
    """A small lattice swept row by row, in blocks of variables."""
    f = wl.grid_cnf(5, 6, 0.2, seed=3)
    p = W.Plan(W.Network.from_formula(f), kind="order", order=wl.row_major_order(5, 6), block=block)
    got, _ = emulate(p, f.weights)
    m, e = oracle.bucket(f)
    assert rel_err(got, Fraction(m) * Fraction(2) ** e) < 1e-12


def test_emulated_weights_override():
    """The same plan with another weight vector (the serving pattern)."""
    f = wl.random_kcnf(16, 50, 12)
    p = W.Plan(W.Network.from_formula(f), seed=2)
    rng = np.random.default_rng(0)
    for _ in range(5):
        w = rng.uniform(0.1, 0.9, size=f.n)
        Wt = np.stack([1 - w, w], axis=1)
        got, _ = emulate(p, Wt)
        ref = Fraction(oracle.brute(f.with_weights(Wt)))
        assert rel_err(got, ref) < 1e-12


def test_emulated_fp32_storage():
    """FP32 storage with per-tensor power-of-two exponents stays within 1e-5."""
    for s in range(20):
        f = wl.random_kcnf(18, 70, 200 + s)
        p = W.Plan(W.Network.from_formula(f), seed=s, precision="fp32")
        got, _ = emulate(p, f.weights, store=np.float32)
        ref = Fraction(oracle.brute(f))
        if ref == 0:
            assert got == 0
        else:
            assert rel_err(got, ref) < 1e-5


# --------------------------------------------------------------- slicing (Algorithm 3)
@pytest.mark.parametrize("cap", [2, 4, 6])
def test_rank_cap_slicing(cap):
    """Slicing meets the rank cap; the slices sum to W (slicing theorem) and
    each slice equals the oracle with the sliced variables fixed."""
    f = wl.random_kcnf(16, 56, 31)
    net = W.Network.from_formula(f)
    p = W.Plan(net, seed=1, rank_cap=cap)
    s = p.stats()
    assert s["max_rank"] <= cap
    assert s["n_slices"] == 2 ** s["n_sliced"]
    assert s["max_rank_unsliced"] > cap
    got, per = emulate(p, f.weights)
    assert rel_err(got, Fraction(oracle.brute(f))) < 1e-12
    sv = s["sliced_vars"]
    for eta in range(min(len(per), 16)):
        units = [[v if (eta >> i) & 1 else -v] for i, v in enumerate(sv)]
        ref = Fraction(oracle.brute(f.with_clauses(units)))
        if ref == 0:
            assert per[eta] == 0
        else:
            assert rel_err(per[eta], ref) < 1e-12


@pytest.mark.parametrize("fseed,block,seed,drop,want", [(1, 2, 0, 1, 3), (2, 1, 0, 3, 4)])
def test_rank_cap_takes_the_fewest_sliced_variables(fseed, block, seed, drop, want):
    """Banded formulas where the memory greedy of Algorithm 3 alone slices 5
    variables (32 slices): the plan slices the fewest variables that meet
    the rank cap.  Checked by brute force over the unsliced plan's tensors:
    the chosen set brings every storage rank to the cap and no smaller set
    of variables does; the replayed slices sum to the oracle's value."""
    f = wl.banded_3cnf(120, 420, 24, seed=fseed)
    net = W.Network.from_formula(f)
    p0 = W.Plan(net, seed=seed, block=block)
    cap = p0.stats()["max_rank"] - drop
    tensors, _, _ = p0.export()
    sets = [set(t[2]) for t in tensors]
    hot = [t for t in sets if len(t) > cap]
    p = W.Plan(net, seed=seed, block=block, rank_cap=cap)
    s = p.stats()
    assert s["n_sliced"] == want and s["max_rank"] <= cap
    chosen = set(s["sliced_vars"])
    assert all(len(t - chosen) <= cap for t in sets)
    cand = sorted(set().union(*hot))
    for k in range(1, want):
        for sub in itertools.combinations(cand, k):
            assert any(len(t - set(sub)) > cap for t in hot), sub
    if fseed == 1:
        got, _ = emulate(p, f.weights)
        assert rel_err(got, Fraction(oracle.bucket_value(f))) < 1e-12


def test_mem_cap_slicing():
    f = wl.random_kcnf(18, 64, 5)
    net = W.Network.from_formula(f)
    p0 = W.Plan(net, seed=0)
    peak = p0.stats()["peak_live_bytes"]
    p = W.Plan(net, seed=0, mem_cap_bytes=int(peak // 5))
    s = p.stats()
    assert s["peak_live_bytes"] <= s["arena_bytes"] <= peak // 5
    assert s["n_sliced"] >= 1
    got, _ = emulate(p, f.weights)
    assert rel_err(got, Fraction(oracle.brute(f))) < 1e-12


def _cap_sweep_formulas():
    """Random, banded and grid formulas whose arenas are dominated by their
    intermediates (not by the 256-byte floor of the leaves)."""
    fs = []
    for seed in range(6):
        fs.append(("random", wl.random_kcnf(26 + seed, 100 + 6 * seed, 100 + seed)))
    for seed in range(3):
        fs.append(("banded", wl.banded_3cnf(80 + 10 * seed, 280 + 35 * seed, 16 + seed, seed)))
    fs.append(("grid", wl.grid_cnf(14, 16, 0.10, seed=14)))
    return fs


@pytest.mark.parametrize("objective,blocks", [("memory", (1, 2, 3, 4, 5)), ("flops", (1, 5))])
def test_mem_cap_is_met_by_the_placed_arena(objective, blocks):
    """Algorithm 3's bound m holds for the memory the plan allocates: over
    random, banded and grid formulas, blocks 1-5 and caps of arena/3 to
    arena/9, every plan keeps its arena (the bytes its tensors occupy as
    placed, alignment included), and so its live peak, within the cap, or
    reports CAP_UNREACHABLE; the replayed descriptors of capped plans of the
    smaller formulas equal the oracle."""
    n_plans = n_capped = n_checked = 0
    for fi, (kind, f) in enumerate(_cap_sweep_formulas()):
        net = W.Network.from_formula(f)
        for block in blocks:
            base = W.Plan(net, seed=fi, block=block).stats()
            for div in range(3, 10):
                cap = int(base["arena_bytes"] // div)
                try:
                    p = W.Plan(net, seed=fi, block=block, mem_cap_bytes=cap, slice_objective=objective)
                except W.WmcError as e:
                    assert e.status == 3, (kind, fi, block, div)
                    continue
                s = p.stats()
                n_plans += 1
                assert s["arena_bytes"] <= cap, (kind, fi, block, div, s["arena_bytes"], cap)
                assert s["peak_live_bytes"] <= s["arena_bytes"], (kind, fi, block, div)
                assert s["workspace_bytes"] >= s["arena_bytes"]
                n_capped += s["n_sliced"] > 0
                if kind == "random" and fi < 3 and div in (3, 9) and block == blocks[-1]:
                    got, _ = emulate(p, f.weights)
                    assert rel_err(got, Fraction(oracle.bucket_value(f))) < 1e-12
                    n_checked += 1
    need = 250 if len(blocks) == 5 else 100
    assert n_plans >= need and n_capped == n_plans and n_checked >= 6, (n_plans, n_capped, n_checked)


def test_flops_objective_never_slices_more_work():
    """The flops objective (least summed flops, then unneeded slices dropped)
    never does more total work than the memory greedy on the same cap, and
    both meet it."""
    for seed in range(8):
        f = wl.banded_3cnf(120, 420, 14, seed)
        net = W.Network.from_formula(f)
        r0 = W.Plan(net, seed=seed).stats()["max_rank"]
        cap = r0 - 3
        a = W.Plan(net, seed=seed, rank_cap=cap).stats()
        b = W.Plan(net, seed=seed, rank_cap=cap, slice_objective="flops").stats()
        assert a["max_rank"] <= cap and b["max_rank"] <= cap
        work_a = a["flops_per_slice"] * a["n_slices"]
        work_b = b["flops_per_slice"] * b["n_slices"]
        assert work_b <= work_a * 1.0000001, (seed, work_a, work_b)


def test_cap_unreachable():
    f = wl.random_kcnf(12, 40, 5)
    with pytest.raises(W.WmcError) as e:
        W.Plan(W.Network.from_formula(f), seed=0, mem_cap_bytes=8)
    assert e.value.status == 3


# --------------------------------------------------------------- statistics and edge cases
def test_stats_recount():
    """flops and bytes per slice recounted from the exported tensors."""
    f = wl.grid_cnf(4, 5, 0.3, seed=1)
    p = W.Plan(W.Network.from_formula(f), kind="order", order=wl.row_major_order(4, 5))
    tensors, nodes, sliced = p.export()
    s = p.stats()
    fl = by = 0.0
    for a, b, c, _ in nodes:
        ra, rb, rc = (len(tensors[t][2]) for t in (a, b, c))
        shared = set(tensors[a][2]) & set(tensors[b][2])
        nk = len(shared - set(tensors[c][2]))
        fl += 2.0 * 2 ** (rc + nk)
        by += 8.0 * (2 ** ra + 2 ** rb + 2 ** rc)
    assert fl == s["flops_per_slice"]
    assert by == s["bytes_per_slice"]
    assert s["max_rank"] == max(len(t[2]) for t in tensors)


def test_tree_independence_emulated():
    """Different trees (seeds, orders, blocks, explicit) give the same W."""
    f = wl.random_kcnf(14, 45, 77)
    net = W.Network.from_formula(f)
    ref = Fraction(oracle.brute(f))
    for seed in range(6):
        got, _ = emulate(W.Plan(net, seed=seed), f.weights)
        assert rel_err(got, ref) < 1e-12
    for seed in range(4):
        got, _ = emulate(W.Plan(net, kind="explicit", parent=random_parent(f, seed)), f.weights)
        assert rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("f", [
    Formula(0, [], np.zeros((0, 2))),
    Formula(1, [], np.array([[0.3, 0.4]])),
    Formula(2, [[]], np.array([[0.3, 0.4], [0.5, 0.5]])),
    Formula(2, [[1, -1]], np.array([[0.3, 0.4], [0.5, 0.25]])),
    Formula(3, [[1], [-1]], np.full((3, 2), 0.5)),
    Formula(3, [[2, 2, 2]], np.array([[1, 2], [3, 4], [5, 6]], dtype=float)),
])
def test_degenerate_formulas(f):
    p = W.Plan(W.Network.from_formula(f))
    got, _ = emulate(p, f.weights)
    ref = Fraction(oracle.brute(f)) if f.n else Fraction(1)
    assert rel_err(got, ref) < 1e-14


def test_fig1_index_rank_and_storage_rank():
    """Storage rank counts tied variables; the index rank counts Theorem-2
    indices and is never smaller."""
    f = wl.fig1_formula()
    s = W.Plan(W.Network.from_formula(f)).stats()
    assert s["max_rank"] <= s["max_index_rank"]


def test_grid24_sweep_plan_shape():
    """The 24x24 lattice swept row-major has max storage rank 25 (width 24-25)."""
    f = wl.grid_cnf(24, 24, 0.10, seed=0)
    assert f.m == 2 * 1104 + 110
    p = W.Plan(W.Network.from_formula(f), kind="order", order=wl.row_major_order(24, 24))
    s = p.stats()
    assert 24 <= s["max_rank"] <= 26
    assert s["class_hist"]["stream"] > 500


@pytest.mark.parametrize("rows,cols,block", [(8, 16, 4), (8, 16, 6), (6, 18, 5), (5, 20, 7)])
def test_emulated_matrix_nodes(rows, cols, block):
    """Blocked sweeps create matrix-shaped nodes (the MFMA class); their
    descriptors replayed on the CPU equal the oracle, in FP64 and FP32."""
    f = wl.grid_cnf(rows, cols, 0.1, seed=2)
    net = W.Network.from_formula(f)
    order = wl.row_major_order(rows, cols)
    m, e = oracle.bucket(f, order=order)
    ref = Fraction(m) * Fraction(2) ** e
    p = W.Plan(net, kind="order", order=order, block=block)
    assert p.stats()["class_hist"]["gemm"] > 0
    got, _ = emulate(p, f.weights)
    assert rel_err(got, ref) < 1e-12
    p32 = W.Plan(net, kind="order", order=order, block=block, precision="fp32")
    got32, _ = emulate(p32, f.weights, store=np.float32)
    assert rel_err(got32, ref) < 1e-5


def test_emulated_batch_merging():
    """A batch merges many plans' launch lists by index with patched offsets;
    the merged descriptors replayed on the CPU give each instance's oracle value."""
    from plan_emulator import emulate_batch
    fs = [wl.random_mixed(s, n_max=12, m_max=24) for s in range(30)]
    fs += [wl.grid_cnf(6, 8, 0.2, seed=1), wl.banded_3cnf(60, 200, 14, seed=3), Formula(0, [], np.zeros((0, 2)))]
    plans = [W.Plan(W.Network.from_formula(f), seed=i, block=1 + i % 3) for i, f in enumerate(fs)]
    b = W.Batch(plans)
    w = np.concatenate([f.weights.reshape(-1) for f in fs])
    vals = emulate_batch(b, w)
    for f, v in zip(fs, vals):
        ref = ref_fraction(f) if f.n else Fraction(1)
        assert (v == 0) if ref == 0 else rel_err(v, ref) < 1e-12


def test_batch_takes_sliced_plans_as_slice_instances():
    """A sliced plan enters a batch as one instance per slice: the image holds
    one root per slice, each with its own arena region; mixed precisions are
    refused."""
    f = wl.random_kcnf(14, 50, 3)
    net = W.Network.from_formula(f)
    sliced = W.Plan(net, seed=0, rank_cap=4)
    ns = sliced.stats()["n_slices"]
    assert ns > 1
    b = W.Batch([W.Plan(net, seed=0), sliced])
    assert b.n == 2
    _, info = b.image()
    assert info["n_instances"] == 1 + ns
    assert info["arena_elems"] >= ns * (sliced.stats()["arena_bytes"] // 8)
    with pytest.raises(W.WmcError) as e:
        W.Batch([W.Plan(net, seed=0), W.Plan(net, seed=0, precision="fp32")])
    assert e.value.status == 1


# ------------------------------------------------------------------ long clauses
def _long_clause_formula(k, extra, seed):
    rng = np.random.default_rng(seed)
    n = k + extra
    sign = rng.choice([-1, 1], size=k)
    clause = [int(sign[i] * (i + 1)) for i in range(k)]
    w = rng.uniform(0.1, 0.9, size=n)
    weights = np.stack([1 - w, w], axis=1) * rng.uniform(0.5, 2.0, size=(n, 1))
    return Formula(n, [clause], weights), clause


@pytest.mark.parametrize("k", [9, 12, 26, 40, 64])
def test_long_clause_closed_form(k):
    """One clause l_1 v ... v l_k: W = prod_x (W0+W1) - prod_{x in C} W(x, falsifying)
    * prod_{x not in C} (W0+W1).  Clauses longer than WMC_FACTOR_ABOVE are
    factored into k-2 auxiliary variables; the replayed descriptors must give
    the closed form."""
    f, clause = _long_clause_formula(k, 3, seed=k)
    tot = Fraction(1)
    for x in range(f.n):
        tot *= Fraction(f.weights[x, 0]) + Fraction(f.weights[x, 1])
    fals = Fraction(1)
    for l in clause:
        x = abs(l) - 1
        fals *= Fraction(f.weights[x, 0] if l > 0 else f.weights[x, 1])
    for x in range(k, f.n):
        fals *= Fraction(f.weights[x, 0]) + Fraction(f.weights[x, 1])
    ref = tot - fals
    p = W.Plan(W.Network.from_formula(f), seed=0)
    assert p.stats()["n_aux_vars"] == k - 2
    assert p.stats()["n_vars"] == f.n
    got, _ = emulate(p, f.weights)
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_long_clauses_vs_brute(seed):
    """Random formulas over 13 variables with two long clauses (9-11 literals,
    one with a repeated literal) among 3-clauses, on min-fill trees and the
    oracle's elimination order (auxiliary variables placed by the planner),
    against brute force."""
    rng = np.random.default_rng(100 + seed)
    n = 13
    clauses = []
    for _ in range(2):
        k = int(rng.integers(9, 12))
        vs = rng.choice(n, size=k, replace=False) + 1
        clauses.append([int(v) * int(s) for v, s in zip(vs, rng.choice([-1, 1], size=k))])
    clauses[0].append(clauses[0][0])
    for _ in range(16):
        vs = rng.choice(n, size=3, replace=False) + 1
        clauses.append([int(v) * int(s) for v, s in zip(vs, rng.choice([-1, 1], size=3))])
    w = rng.uniform(0.1, 0.9, size=n)
    f = Formula(n, clauses, np.stack([1 - w, w], axis=1))
    ref = oracle.brute(f)
    order = [int(x) for x in oracle.minfill_order(f)]
    for kw in (dict(seed=seed), dict(kind="order", order=order), dict(kind="order", order=order, block=3)):
        p = W.Plan(W.Network.from_formula(f), **kw)
        assert p.stats()["n_aux_vars"] > 0
        got, _ = emulate(p, f.weights)
        assert rel_err(got, Fraction(ref)) <= 1e-11, kw


def test_long_tautology_is_dropped():
    """x v ... v not-x with more than WMC_FACTOR_ABOVE literals weighs 1."""
    f = Formula(10, [list(range(1, 11)) + [-3]], np.full((10, 2), 0.5))
    p = W.Plan(W.Network.from_formula(f), seed=0)
    assert p.stats()["n_aux_vars"] == 0
    got, _ = emulate(p, f.weights)
    assert got == 1


def test_long_clause_rejects_supplied_tree():
    f, _ = _long_clause_formula(10, 0, seed=1)
    net = W.Network.from_formula(f)
    parent = [-1] * (2 * (f.n + 1) - 1)
    with pytest.raises(W.WmcError) as e:
        W.Plan(net, kind="explicit", parent=parent)
    assert e.value.status == 6


def test_batch_with_big_nodes_replays():
    """Batches whose merged steps hold nodes of 2^20+ outputs (streaming
    tasks) next to small ones: the replayed batch image equals the oracle."""
    from plan_emulator import emulate_batch
    fs = [wl.banded_3cnf(120, 400, 24, seed=s) for s in range(2)] + [wl.random_long(0)]
    b = W.Batch([W.Plan(W.Network.from_formula(f), seed=s) for s, f in enumerate(fs)])
    vals = emulate_batch(b, np.concatenate([f.weights.reshape(-1) for f in fs]))
    for f, v in zip(fs, vals):
        m, e = oracle.bucket(f)
        assert rel_err(v, Fraction(m) * Fraction(2) ** e) <= 1e-12


# ------------------------------------------------------------------ anytime planning (Algorithm 1)
def test_anytime_plan_stops_by_alpha_and_keeps_the_best():
    """alpha = 0 stops after the first candidate; a large alpha keeps
    planning up to the candidate limit and returns the cheapest predicted
    plan; the plan still computes W (replayed on the CPU)."""
    from paper_2006_15512_amd.autotune import anytime_plan, time_cost
    from plan_emulator import emulate
    f = wl.banded_3cnf(60, 200, 14, seed=3)
    p0, r0 = anytime_plan(f, alpha=0.0)
    assert r0["candidates"] == 1 and r0["stopped"] == "alpha"
    p1, r1 = anytime_plan(f, alpha=1e9, blocks=(1, 2, 3), max_candidates=9)
    assert r1["candidates"] == 9 and r1["stopped"] == "max_candidates"
    assert r1["predicted_seconds"] == min(h["cost_s"] for h in r1["history"])
    assert abs(time_cost(p1) - r1["predicted_seconds"]) <= 1e-12 * r1["predicted_seconds"]
    got, _ = emulate(p1, f.weights)
    m, e = oracle.bucket(f)
    assert rel_err(got, Fraction(m) * Fraction(2) ** e) <= 1e-12


def test_time_cost_grows_with_slices():
    """Slicing to a lower rank multiplies the predicted time by the slices."""
    from paper_2006_15512_amd.autotune import time_cost
    f = wl.banded_3cnf(120, 400, 24, seed=1)
    net = W.Network.from_formula(f)
    a = W.Plan(net, seed=1)
    b = W.Plan(net, seed=1, rank_cap=a.stats()["max_rank"] - 3)
    assert b.stats()["n_slices"] >= 8
    assert time_cost(b) > time_cost(a)


def test_checkpoint_refuses_other_weights_precision_or_formula(tmp_path):
    """A saved slice-loop checkpoint resumes only the same plan, formula,
    precision and weights: any other is refused before anything runs."""
    import json
    f = wl.banded_3cnf(60, 200, 14, seed=3)
    p = W.Plan(W.Network.from_formula(f), seed=0, rank_cap=8)
    path = str(tmp_path / "ck.json")
    with open(path, "w") as fh:
        json.dump({"plan": W.checkpoint_identity(p), "s": (0.5).hex(), "c": (0.0).hex(), "e": 0,
                   "next_slice": 1, "n_slices": p.n_slices}, fh)
    w2 = np.array(f.weights, dtype=np.float64).copy()
    w2[0, 1] = 0.25
    w2[0, 0] = 0.75
    with pytest.raises(ValueError):
        W.contract_checkpointed(p, path, weights=w2)
    p32 = W.Plan(W.Network.from_formula(f), seed=0, rank_cap=8, precision="fp32")
    with pytest.raises(ValueError):
        W.contract_checkpointed(p32, path)
    g = wl.banded_3cnf(60, 200, 14, seed=4)  # same shape, other clauses
    pg = W.Plan(W.Network.from_formula(g.with_weights(f.weights)), seed=0, rank_cap=8)
    if pg.n_slices == p.n_slices and pg.stats()["sliced_vars"] == p.stats()["sliced_vars"]:
        with pytest.raises(ValueError):
            W.contract_checkpointed(pg, path)
    assert W.checkpoint_identity(pg)["clauses_sha256"] != W.checkpoint_identity(p)["clauses_sha256"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_launch_is_bounds_checked(precision):
    """wmc_plan proves on the host, for every launch, that the largest
    address each kernel's index maps can form lies inside the tensors it
    reads and writes (and every tensor inside the arena).  Driven through
    every kernel family by varying the tuning fields that choose kernels and
    tiles; a plan that failed the check would raise."""
    import bench
    f = wl.banded_3cnf(200, 700, 26, seed=6)
    g = wl.grid_cnf(8, 16, 0.1, seed=2)
    saved = W.tuning_get(precision)
    variants = [{}, {"stream2_vec": 1 - saved["stream2_vec"]}, {"stream_mfma_min_bits": 0},
                {"stream2_tile_bits": 1}, {"stream2_min_thread_bits": 0, "stream2_low_bits": 0},
                {"split_lanes": 4 if precision == "fp64" else 0}, {"gemm_orient": 2}]
    kinds = set()
    try:
        for v in variants:
            W.tuning_set(precision, dict(saved, **v))
            for net, kw in ((W.Network.from_formula(f), dict(block=4)), (W.Network.from_formula(f), dict(block=1)),
                            (W.Network.from_formula(f), dict(block=3, rank_cap=17, slice_group=3)),
                            (W.Network.from_formula(g), dict(kind="order", order=wl.row_major_order(8, 16), block=5))):
                p = W.Plan(net, seed=0, precision=precision, **kw)
                kinds |= {W.KERNEL_NAMES[k] for k in W.plan_kernels(p)}
    finally:
        W.tuning_set(precision, saved)
    expect = {"k_nodes", "k_stream2", "k_stream_mfma", "k_gemm_p", "k_stream2_vec"}
    if precision == "fp64":
        expect.add("k_stream2_split")
    assert expect <= kinds, kinds
