"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64: relative error <= 1e-12 (non-negative weights; an exact zero must come
back as exactly zero).  Scaled FP32: <= 1e-5.  Bit-exact where the
arithmetic is exact: all weights 1/2 (W = #models / 2^n) and all weights 1
(W = #models) while the counts stay below 2^53 (FP64) or 2^24 (FP32).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl
from wmc_workloads import Formula

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    W.lib()  # fails loudly if libwmc.so is missing
    return torch


def value_fraction(v):
    if v.mantissa == 0.0:
        return Fraction(0)
    return Fraction(v.mantissa) * Fraction(2) ** v.exp2


def ref_of(f):
    if f.n <= 22:
        return Fraction(oracle.brute(f))
    m, e = oracle.bucket(f)
    return Fraction(m) * Fraction(2) ** e


def rel(a: Fraction, b: Fraction) -> float:
    if a == b:
        return 0.0
    return float(abs(a - b) / max(abs(a), abs(b)))


def run(f, weights=None, **kw):
    net = W.Network.from_formula(f)
    p = W.Plan(net, **kw)
    v = W.wmc_contract(p, weights)
    return v, p


# ------------------------------------------------------------------ small random formulas
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_mixed_small(precision, tol):
    for s in range(120):
        f = wl.random_mixed(s, n_max=14, m_max=28)
        say(f"mixed seed={s} n={f.n} m={f.m} {precision}")
        v, _ = run(f, seed=s, precision=precision)
        ref = Fraction(oracle.brute(f))
        got = value_fraction(v)
        if ref == 0:
            assert got == 0, s
        else:
            assert rel(got, ref) <= tol, (s, float(got), float(ref))


@pytest.mark.parametrize("scale", [1e50, 1e-50, 1e300])
def test_fp32_weights_beyond_the_fp32_range(scale):
    """Weights far outside FP32's range (above its largest or below its
    smallest normal number): each weight leaf carries a power-of-two
    exponent, so scaled FP32 still matches the oracle."""
    f = wl.random_kcnf(16, 50, seed=5)
    rng = np.random.default_rng(11)
    Wt = np.stack([rng.uniform(0.1, 0.9, f.n), rng.uniform(0.1, 0.9, f.n)], axis=1) * scale
    g = f.with_weights(Wt)
    m, e = oracle.bucket(g)
    ref = Fraction(m) * Fraction(2) ** e
    for prec, tol in (("fp32", 1e-5), ("fp64", 1e-12)):
        v = W.wmc_contract(W.Plan(W.Network.from_formula(g), seed=0, precision=prec))
        assert v.mantissa != 0.0 and math.isfinite(v.mantissa)
        assert rel(value_fraction(v), ref) <= tol, (prec, scale)


def test_negative_weights():
    for s in range(40):
        f = wl.random_mixed(s, n_max=12, m_max=20, negative=True)
        say(f"negative seed={s}")
        v, _ = run(f, seed=s)
        ref = oracle.brute(f)
        scale = float(np.prod(np.abs(f.weights).sum(axis=1)))
        assert abs(v.value - ref) <= 1e-12 * scale


def test_config1_random3cnf_seed_sweep():
    """Random 3-CNF, 20 variables, 85 clauses: seeds 0..39 against brute force."""
    n_sat = 0
    for s in range(40):
        f = wl.random_kcnf(20, 85, s)
        say(f"config1 seed={s}")
        v, p = run(f, seed=0)
        ref = Fraction(oracle.brute(f))
        got = value_fraction(v)
        if ref == 0:
            assert got == 0
        else:
            n_sat += 1
            assert rel(got, ref) <= 1e-12
    assert n_sat > 10


# ------------------------------------------------------------------ exact modes
def test_all_half_bit_exact():
    """All weights 1/2: W = #models / 2^n exactly (FP64 and FP32 while the
    counts stay below 2^24)."""
    for s in range(30):
        f = wl.random_kcnf(22, 60 + s, 300 + s)
        half = f.with_weights(np.full((f.n, 2), 0.5))
        cnt = oracle.exact_count(f)
        say(f"half seed={s} count={cnt}")
        for prec in ("fp64", "fp32"):
            v, _ = run(half, seed=s, precision=prec)
            assert value_fraction(v) == Fraction(cnt, 2 ** f.n), (s, prec)


def test_all_ones_bit_exact():
    """All weights 1: W = #models exactly."""
    for s in range(20):
        f = wl.banded_3cnf(40, 100, 12, seed=s)
        ones = f.with_weights(np.ones((f.n, 2)))
        cnt = oracle.exact_count(f)
        assert cnt < 2 ** 53
        say(f"ones seed={s} count={cnt}")
        v, _ = run(ones, seed=s)
        assert value_fraction(v) == cnt


# ------------------------------------------------------------------ trees and slicing
def test_tree_independence():
    f = wl.random_kcnf(20, 70, 9)
    ref = Fraction(oracle.brute(f))
    vals = []
    for seed in range(8):
        say(f"tree seed={seed}")
        v, _ = run(f, seed=seed)
        vals.append(value_fraction(v))
        assert rel(vals[-1], ref) <= 1e-12
    for block in (2, 3, 5):
        v, _ = run(f, kind="order", order=oracle.minfill_order(f), block=block)
        assert rel(value_fraction(v), ref) <= 1e-12


@pytest.mark.parametrize("cap", [3, 6, 9])
def test_slicing(cap):
    f = wl.random_kcnf(20, 75, 41)
    say(f"slicing cap={cap}")
    net = W.Network.from_formula(f)
    p = W.Plan(net, seed=3, rank_cap=cap)
    st = p.stats()
    assert st["max_rank"] <= cap and st["n_sliced"] > 0
    tot, per = W.wmc_contract_slices(p, 0, p.n_slices, per_slice=True)
    ref = Fraction(oracle.brute(f))
    assert rel(value_fraction(tot), ref) <= 1e-12
    sv = st["sliced_vars"]
    for eta in range(min(p.n_slices, 8)):
        units = [[v if (eta >> i) & 1 else -v] for i, v in enumerate(sv)]
        r = Fraction(oracle.brute(f.with_clauses(units)))
        got = value_fraction(per[eta])
        assert (got == 0) if r == 0 else rel(got, r) <= 1e-12
    # a partition of the slices sums to the whole (the multi-GPU split)
    half = p.n_slices // 2
    a = value_fraction(W.wmc_contract_slices(p, 0, half))
    b = value_fraction(W.wmc_contract_slices(p, half, p.n_slices))
    assert rel(a + b, ref) <= 1e-12


@pytest.mark.parametrize("objective", ["memory", "flops"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_mem_capped_sliced_plan_vs_oracle(objective, precision, tol):
    """A plan sliced to meet a memory cap (Algorithm 3's bound m on the
    arena) runs within the cap it was given and matches the oracle."""
    f = wl.banded_3cnf(120, 420, 22, seed=3)
    net = W.Network.from_formula(f)
    base = W.Plan(net, seed=0, block=2, precision=precision).stats()
    cap = base["arena_bytes"] // 4
    say(f"mem cap {cap} {objective} {precision}")
    p = W.Plan(net, seed=0, block=2, precision=precision, mem_cap_bytes=cap, slice_objective=objective)
    st = p.stats()
    assert st["arena_bytes"] <= cap and st["n_sliced"] >= 3
    v = W.wmc_contract(p)
    m, e = oracle.bucket(f)
    assert rel(value_fraction(v), Fraction(m) * Fraction(2) ** e) <= tol


def test_weights_override_and_reuse():
    f = wl.grid_cnf(6, 7, 0.2, seed=4)
    net = W.Network.from_formula(f)
    p = W.Plan(net, kind="order", order=wl.row_major_order(6, 7))
    ws = W.workspace(p)
    rng = np.random.default_rng(0)
    for q in range(10):
        w = rng.uniform(0.1, 0.9, size=f.n)
        Wt = np.stack([1 - w, w], axis=1)
        v = W.wmc_contract(p, Wt, ws)
        m, e = oracle.bucket(f.with_weights(Wt))
        assert rel(value_fraction(v), Fraction(m) * Fraction(2) ** e) <= 1e-12


@pytest.mark.parametrize("f", [
    Formula(0, [], np.zeros((0, 2))),
    Formula(1, [], np.array([[0.3, 0.4]])),
    Formula(2, [[]], np.array([[0.3, 0.4], [0.5, 0.5]])),
    Formula(2, [[1, -1]], np.array([[0.3, 0.4], [0.5, 0.25]])),
    Formula(3, [[1], [-1]], np.full((3, 2), 0.5)),
    Formula(3, [[2, 2, 2]], np.array([[1, 2], [3, 4], [5, 6]], dtype=float)),
    wl.psi_formula(20),
])
def test_degenerate(f):
    say(f"degenerate {f.clauses[:3]}")
    v, _ = run(f)
    ref = Fraction(oracle.brute(f)) if f.n else Fraction(1)
    assert rel(value_fraction(v), ref) <= 1e-14


def test_workspace_too_small():
    f = wl.random_kcnf(12, 30, 1)
    p = W.Plan(W.Network.from_formula(f))
    import torch
    ws = torch.empty(p.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(W.WmcError) as e:
        W.wmc_contract(p, None, ws)
    assert e.value.status == 2


# ------------------------------------------------------------------ full-size lattice
def _golden(name):
    with open(GOLDEN) as fh:
        return json.load(fh)[name]


@pytest.mark.parametrize("name,rows", [("grid12x24_t0.10_s1", 12), ("grid24x24_t0.10_s0", 24)])
@pytest.mark.parametrize("block", [1, 6])
def test_grid_lattice_vs_golden(name, rows, block):
    """The 24-column lattice swept row by row (max storage rank 25) against
    the oracle's stored value for the same seeded instance."""
    g = _golden(name)
    seed = 0 if name.endswith("s0") else 1
    f = wl.grid_cnf(rows, 24, 0.10, seed=seed)
    assert f.digest() == g["digest"]
    say(f"{name} block={block}")
    v, p = run(f, kind="order", order=wl.row_major_order(rows, 24), block=block)
    ref = Fraction(float.fromhex(g["mantissa_hex"])) * Fraction(2) ** g["exp2"]
    assert rel(value_fraction(v), ref) <= 1e-12


@pytest.mark.parametrize("rows,cols", [(8, 16), (6, 18), (5, 20)])
@pytest.mark.parametrize("block", [1, 3, 4, 6, 7])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_grid_blocks_vs_oracle(rows, cols, block, precision, tol):
    """Blocked sweeps put matrix-shaped nodes on MFMA (FP64 or FP32)."""
    f = wl.grid_cnf(rows, cols, 0.1, seed=2)
    order = wl.row_major_order(rows, cols)
    say(f"grid {rows}x{cols} block={block} {precision}")
    v, p = run(f, kind="order", order=order, block=block, precision=precision)
    m, e = oracle.bucket(f, order=order)
    assert rel(value_fraction(v), Fraction(m) * Fraction(2) ** e) <= tol


@pytest.mark.parametrize("block", [1, 3, 4])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_banded300_sliced_vs_golden(precision, tol, block):
    """Banded random 3-CNF, 300 variables, ratio 3.5: seeded min-fill tree of
    max storage rank 30 sliced to rank 27 (index slicing), against the
    oracle's stored value."""
    g = _golden("banded300_m1050_W37_s0")
    f = wl.banded_3cnf(300, 1050, 37, seed=0)
    assert f.digest() == g["digest"]
    say(f"banded300 {precision}")
    v, p = run(f, kind="minfill", seed=0, rank_cap=27, precision=precision, block=block)
    st = p.stats()
    assert st["max_rank"] <= 27 and st["max_rank_unsliced"] >= 29 and st["n_slices"] >= 8
    ref = Fraction(float.fromhex(g["mantissa_hex"])) * Fraction(2) ** g["exp2"]
    assert rel(value_fraction(v), ref) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_grid24_minfill_sliced_vs_golden(precision, tol):
    """The same 24x24 lattice on its seeded min-fill tree (max storage rank
    34) sliced to rank 26: 128 slices, against the oracle's stored value."""
    g = _golden("grid24x24_t0.10_s0")
    f = wl.grid_cnf(24, 24, 0.10, seed=0)
    assert f.digest() == g["digest"]
    say(f"grid24 minfill sliced {precision}")
    v, p = run(f, kind="minfill", seed=0, rank_cap=26, block=3, precision=precision)
    st = p.stats()
    assert st["max_rank"] <= 26 and st["max_rank_unsliced"] >= 32 and st["n_slices"] >= 64
    ref = Fraction(float.fromhex(g["mantissa_hex"])) * Fraction(2) ** g["exp2"]
    assert rel(value_fraction(v), ref) <= tol


@pytest.mark.parametrize("seed", range(4))
def test_banded_medium_stream_shapes_fp32(seed):
    """Scaled FP32 through the streaming and matrix kernels on irregular
    layouts (banded 3-CNF, 140 variables, ratio 2.8, satisfiable, min-fill
    trees, blocks 1-4)."""
    f = wl.banded_3cnf(140, 390, 26, seed=seed)
    m, e = oracle.bucket(f)
    ref = Fraction(m) * Fraction(2) ** e
    assert ref > 0
    for kw in (dict(seed=seed), dict(seed=seed, block=2), dict(seed=seed, block=4),
               dict(seed=seed, block=3, rank_cap=17)):
        say(f"banded140 fp32 seed={seed} {kw}")
        v, _ = run(f, precision="fp32", **kw)
        assert rel(value_fraction(v), ref) <= 1e-5


@pytest.mark.parametrize("seed", range(6))
def test_banded_medium_stream_shapes(seed):
    """Banded 3-CNF of 120 variables (max rank ~20): min-fill trees with
    several seeds and blocks exercise the streaming and matrix kernels on
    irregular layouts; FP64 against the oracle."""
    f = wl.banded_3cnf(120, 400, 24, seed=seed)
    m, e = oracle.bucket(f)
    ref = Fraction(m) * Fraction(2) ** e
    for kw in (dict(seed=seed), dict(kind="order", order=oracle.minfill_order(f), block=3),
               dict(kind="order", order=oracle.minfill_order(f), block=5), dict(seed=seed, block=4, rank_cap=18)):
        say(f"banded120 seed={seed} {kw}")
        v, _ = run(f, **kw)
        assert rel(value_fraction(v), ref) <= 1e-12


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
def test_banded_medium_k32_blocks_fp32(seed):
    """Scaled FP32 on min-fill orders in blocks of 5: streaming nodes with 32
    summed entries and short matrices per batch value (the matrix-core
    streaming kernel at K = 32, rows or columns repeated where a side has
    only 3 bits) against the oracle."""
    f = wl.banded_3cnf(120, 400, 24, seed=seed)
    m, e = oracle.bucket(f)
    ref = Fraction(m) * Fraction(2) ** e
    assert ref > 0
    say(f"banded120 fp32 k32 seed={seed}")
    v, _ = run(f, kind="order", order=oracle.minfill_order(f), block=5, precision="fp32")
    assert rel(value_fraction(v), ref) <= 1e-5


# ------------------------------------------------------------------ long clauses
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_long_clauses_vs_brute(precision, tol):
    """Clauses of 9-11 literals factored into chains over auxiliary
    variables: results (network weights and new weights) against brute force."""
    rng = np.random.default_rng(7)
    for s in range(12):
        f = wl.random_long(s)
        say(f"long seed={s} {precision}")
        net = W.Network.from_formula(f)
        for kw in (dict(seed=s), dict(kind="order", order=oracle.minfill_order(f), block=3)):
            p = W.Plan(net, precision=precision, **kw)
            assert p.stats()["n_aux_vars"] > 0
            v = W.wmc_contract(p)
            assert rel(value_fraction(v), Fraction(oracle.brute(f))) <= tol
            w = rng.uniform(0.1, 0.9, size=f.n)
            Wt = np.stack([1 - w, w], axis=1)
            v = W.wmc_contract(p, Wt)
            assert rel(value_fraction(v), Fraction(oracle.brute(f.with_weights(Wt)))) <= tol


def test_one_clause_of_200_literals_closed_form():
    """W of a single 200-literal clause: prod (W0+W1) - prod W(x, falsifying)."""
    rng = np.random.default_rng(3)
    k = 200
    w = rng.uniform(0.1, 0.9, size=k)
    Wt = np.stack([1 - w, w], axis=1)
    signs = rng.choice([-1, 1], size=k)
    f = Formula(k, [[int(signs[i] * (i + 1)) for i in range(k)]], Wt)
    tot, fals = Fraction(1), Fraction(1)
    for i in range(k):
        tot *= Fraction(Wt[i, 0]) + Fraction(Wt[i, 1])
        fals *= Fraction(Wt[i, 0] if signs[i] > 0 else Wt[i, 1])
    ref = tot - fals
    for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        v, p = run(f, seed=0, precision=precision)
        assert p.stats()["n_aux_vars"] == k - 2
        assert rel(value_fraction(v), ref) <= tol


# ------------------------------------------------------------------ checkpoint / resume
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_loop_checkpoint_resume_is_bit_exact(tmp_path, precision):
    """The slice loop stopped after some chunks, its state saved to a file,
    and resumed with a fresh plan object gives the bits of one wmc_contract."""
    f = wl.banded_3cnf(120, 400, 24, seed=1)
    kw = dict(seed=1, rank_cap=16, precision=precision)
    p = W.Plan(W.Network.from_formula(f), **kw)
    ns = p.stats()["n_slices"]
    assert ns >= 16
    full = W.wmc_contract(p)
    path = str(tmp_path / "slices.json")
    assert W.contract_checkpointed(p, path, chunk=3, stop_after=2) is None
    p2 = W.Plan(W.Network.from_formula(f), **kw)   # as after a restart
    v = W.contract_checkpointed(p2, path, chunk=5)
    assert (v.mantissa, v.exp2) == (full.mantissa, full.exp2)
    m, e = oracle.bucket(f)
    assert rel(value_fraction(v), Fraction(m) * Fraction(2) ** e) <= (1e-12 if precision == "fp64" else 1e-5)
    other = W.Plan(W.Network.from_formula(f), seed=1, rank_cap=15, precision=precision)
    with pytest.raises(ValueError):
        W.contract_checkpointed(other, path)


# ------------------------------------------------------------------ slices side by side
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_groups_are_bit_identical(precision):
    """Slices run G at a time in every launch (grid dimension z, one arena and
    meta table per slice) give the bits of one slice at a time, for groups
    that divide the slice count and groups that leave a partial last group;
    slice ranges and the checkpointed loop split groups anywhere."""
    f = wl.banded_3cnf(120, 400, 24, seed=1)
    kw = dict(seed=1, rank_cap=16, precision=precision, block=2)
    net = W.Network.from_formula(f)
    p1 = W.Plan(net, **kw)
    ns = p1.n_slices
    assert ns >= 16
    ref = W.wmc_contract(p1)
    m, e = oracle.bucket(f)
    assert rel(value_fraction(ref), Fraction(m) * Fraction(2) ** e) <= (1e-12 if precision == "fp64" else 1e-5)
    for g in (2, 5, ns):
        say(f"slice group {g} of {ns} ({precision})")
        pg = W.Plan(net, slice_group=g, **kw)
        st = pg.stats()
        assert st["slice_group"] == g
        assert st["workspace_bytes"] >= g * st["arena_bytes"]
        v = W.wmc_contract(pg)
        assert (v.mantissa, v.exp2) == (ref.mantissa, ref.exp2), g
        a = W.wmc_contract_slices(pg, 0, 7)
        a1 = W.wmc_contract_slices(p1, 0, 7)
        assert (a.mantissa, a.exp2) == (a1.mantissa, a1.exp2), g
        st_ = W.wmc_slice_state()
        for chunk in (3, ns):
            W.wmc_contract_resume(pg, st_, chunk)
        r = W.wmc_contract_resume(pg, st_, 0)
        assert (r.mantissa, r.exp2) == (ref.mantissa, ref.exp2), g
    # the profile accounts the grouped launches in the same order
    pg = W.Plan(net, slice_group=4, **kw)
    v, ms = W.wmc_contract_profile(pg)
    assert (v.mantissa, v.exp2) == (ref.mantissa, ref.exp2)
    assert len(ms) == len(W.plan_launches(pg)[0]) and float(ms.sum()) > 0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_banded300_all_slices_in_one_group_vs_golden(precision, tol):
    """The sliced 300-variable formula (8 slices) with every slice in each
    launch, as the benchmark runs it, against the stored oracle value."""
    with open(GOLDEN) as fh:
        g = json.load(fh)["banded300_m1050_W37_s0"]
    ref = Fraction(float.fromhex(g["mantissa_hex"])) * Fraction(2) ** g["exp2"]
    f = wl.banded_3cnf(300, 1050, 37, seed=0)
    say(f"banded300 group 8 {precision}")
    p = W.Plan(W.Network.from_formula(f), seed=0, rank_cap=27, block=4, precision=precision, slice_group=8)
    assert p.stats()["slice_group"] == 8
    v = W.wmc_contract(p)
    assert rel(value_fraction(v), ref) <= tol


# ------------------------------------------------------------------ executor tuning
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paired_k1_kernel_is_bit_identical(precision):
    """K = 1 streaming nodes with output bit 0 inside the thread (entry pairs)
    round exactly as the one-output-per-thread kernel: the same plan with the
    tuning switched either way gives the same bits, and the oracle's value."""
    f = wl.banded_3cnf(200, 700, 26, seed=6)
    net = W.Network.from_formula(f)
    saved = W.tuning_get(precision)
    try:
        vals = []
        for vec in (0, 1):
            W.tuning_set(precision, {"stream2_vec": vec, "stream_mfma_min_bits": 0})
            p = W.Plan(net, seed=0, block=3, precision=precision)
            kinds = set(W.KERNEL_NAMES[k] for k in W.plan_kernels(p))
            assert ("k_stream2_vec" in kinds) == bool(vec), kinds
            vals.append(W.wmc_contract(p))
    finally:
        W.tuning_set(precision, saved)
    assert (vals[0].mantissa, vals[0].exp2) == (vals[1].mantissa, vals[1].exp2)
    m, e = oracle.bucket(f)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert rel(value_fraction(vals[1]), Fraction(m) * Fraction(2) ** e) <= tol


# ------------------------------------------------------------------ Algorithm 1's anytime loop
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_anytime_plan_on_device_vs_oracle(precision, tol):
    """The anytime planning loop (Algorithm 1) with the execution-time model
    read from the rates measured on this device: the plan it returns runs
    on the GPU and matches the oracle, and its measured time is within an
    order of magnitude of the prediction."""
    import time
    from paper_2006_15512_amd.autotune import anytime_plan, measured_rates, time_cost
    rates = measured_rates(precision)
    assert rates is not None, "no measured rates stored for this device"
    f = wl.banded_3cnf(160, 560, 24, seed=2)
    p, rep = anytime_plan(f, alpha=1e-3, precision=precision, blocks=(1, 2, 3, 4), rank_cap=18, max_candidates=8)
    say(f"anytime {precision}: {rep['candidates']} candidates, predicted {rep['predicted_seconds'] * 1e3:.3f} ms")
    assert abs(time_cost(p) - rep["predicted_seconds"]) <= 1e-9 * rep["predicted_seconds"]
    ws = W.workspace(p)
    v = W.wmc_contract(p, None, ws)
    t0 = time.perf_counter()
    for _ in range(3):
        v = W.wmc_contract(p, None, ws)
    dt = (time.perf_counter() - t0) / 3
    m, e = oracle.bucket(f)
    assert rel(value_fraction(v), Fraction(m) * Fraction(2) ** e) <= tol
    assert rep["predicted_seconds"] / 10 <= dt <= rep["predicted_seconds"] * 10, (dt, rep["predicted_seconds"])


# ------------------------------------------------------------------ autotuned plan shape
def test_autotune_plan_picks_fastest_and_caches(tmp_path):
    """The autotuner times every candidate block size, returns the fastest
    (whose result matches the oracle) and answers from its cache next time."""
    from paper_2006_15512_amd.autotune import autotune_plan
    f = wl.grid_cnf(10, 20, 0.1, seed=3)
    order = wl.row_major_order(10, 20)
    cache = str(tmp_path / "tune.json")
    p, rep = autotune_plan(f, blocks=(1, 3, 5), order=order, reps=2, cache=cache)
    assert not rep["cached"] and len(rep["results"]) == 3
    assert rep["ms"] == min(r["ms"] for r in rep["results"] if "ms" in r)
    m, e = oracle.bucket(f, order=order)
    assert rel(value_fraction(W.wmc_contract(p)), Fraction(m) * Fraction(2) ** e) <= 1e-12
    p2, rep2 = autotune_plan(f, blocks=(1, 3, 5), order=order, reps=2, cache=cache)
    assert rep2["cached"] and rep2["best_candidate"] == rep["best_candidate"]
    assert p2.stats()["n_launches"] == p.stats()["n_launches"]
