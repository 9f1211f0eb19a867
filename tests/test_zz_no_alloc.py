"""GPU test of wmc_contract_noalloc, the contraction that allocates no
device memory (its workspace is the library's static device scratch)."""
import numpy as np
import pytest

import paper_2006_15512_amd as W
import wmc_workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def bits(v):
    return (v.mantissa, v.exp2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_wmc_contract_twice_then_smaller(precision):
    """Two calls in a row, the second on a smaller plan (the scratch keeps
    the first call's contents), each bit-identical to wmc_contract on a
    workspace of its own; then the first plan again with other weights, and
    a sliced plan."""
    big = wl.banded_3cnf(160, 560, 20, seed=4)
    small = wl.random_kcnf(16, 60, seed=3)
    p_big = W.Plan(W.Network.from_formula(big), seed=0, block=2, precision=precision)
    p_small = W.Plan(W.Network.from_formula(small), seed=0, precision=precision)
    assert p_small.workspace_bytes < p_big.workspace_bytes <= W.NOALLOC_SCRATCH_BYTES
    say(f"noalloc {precision}: big plan {p_big.workspace_bytes} B")
    a = W.wmc_contract_noalloc(p_big)
    assert bits(a) == bits(W.wmc_contract(p_big))
    say(f"noalloc {precision}: small plan {p_small.workspace_bytes} B")
    b = W.wmc_contract_noalloc(p_small)
    assert bits(b) == bits(W.wmc_contract(p_small))
    rng = np.random.default_rng(7)
    w = rng.uniform(0.1, 0.9, size=big.n)
    Wt = np.stack([1 - w, w], axis=1)
    assert bits(W.wmc_contract_noalloc(p_big, Wt)) == bits(W.wmc_contract(p_big, Wt))
    p_sl = W.Plan(W.Network.from_formula(big), seed=0, block=2, precision=precision, rank_cap=14)
    assert p_sl.n_slices > 1
    say(f"noalloc {precision}: sliced plan, {p_sl.n_slices} slices")
    assert bits(W.wmc_contract_noalloc(p_sl)) == bits(W.wmc_contract(p_sl))


def test_noalloc_rejects_plans_beyond_the_scratch():
    f = wl.grid_cnf(6, 24, 0.10, seed=0)
    p = W.Plan(W.Network.from_formula(f), kind="order", order=wl.row_major_order(6, 24))
    assert p.workspace_bytes > W.NOALLOC_SCRATCH_BYTES
    with pytest.raises(W.WmcError) as e:
        W.wmc_contract_noalloc(p)
    assert e.value.status == 2
