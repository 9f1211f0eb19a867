"""Planning from a supplied tree decomposition (PACE .td text) of the
primal graph: the derived elimination order, its width bound, and the
error paths.  Host only, except the last test (GPU parity of a plan built
from a decomposition)."""
import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl


def primal_adjacency(f):
    adj = {v: set() for v in range(1, f.n + 1)}
    for c in f.clauses:
        vs = {abs(l) for l in c}
        for a in vs:
            adj[a] |= vs - {a}
    return adj


def td_from_order(f, order):
    """Textbook decomposition of an elimination order: bag(x) = x and its
    later neighbours in the filled graph, joined to the bag of the earliest
    eliminated of those (or to the next bag when there are none)."""
    adj = {v: set(s) for v, s in primal_adjacency(f).items()}
    pos = {v: i for i, v in enumerate(order)}
    bags, edges = [], []
    for v in order:
        later = {u for u in adj[v] if pos[u] > pos[v]}
        bags.append(sorted({v} | later))
        for a in later:
            adj[a] |= later - {a}
    for i, v in enumerate(order[:-1]):
        later = [u for u in bags[i] if u != v]
        j = min(pos[u] for u in later) if later else i + 1
        edges.append((i + 1, j + 1))
    width = max(len(b) for b in bags) - 1
    lines = [f"c decomposition of an elimination order", f"s td {len(bags)} {width + 1} {f.n}"]
    lines += ["b %d %s" % (i + 1, " ".join(map(str, b))) for i, b in enumerate(bags)]
    lines += ["%d %d" % e for e in edges]
    return "\n".join(lines) + "\n", width


def induced_width(f, order):
    adj = {v: set(s) for v, s in primal_adjacency(f).items()}
    w = 0
    for v in order:
        nb = adj.pop(v)
        w = max(w, len(nb))
        for a in nb:
            adj[a] |= nb - {a}
            adj[a].discard(v)
    return w


def test_path_decomposition_exact_order():
    """Path x1-x2-x3-x4 with bags {1,2},{2,3},{3,4} rooted at the first bag:
    x4 leaves at the deepest bag, x3 next, x1 and x2 at the root."""
    f = wl.Formula(4, [[1, 2], [-2, 3], [3, -4]], np.full((4, 2), 0.5))
    net = W.Network.from_formula(f)
    td = "s td 3 2 4\nb 1 1 2\nb 2 2 3\nb 3 3 4\n1 2\n2 3\n"
    order, width = W.order_from_td(net, td)
    assert list(order) == [4, 3, 1, 2] and width == 1
    order, _ = W.order_from_td(net, td, root_bag=3)
    assert list(order) == [1, 2, 3, 4]


@pytest.mark.parametrize("make", [lambda: wl.grid_cnf(6, 9, 0.1, seed=1),
                                  lambda: wl.banded_3cnf(60, 210, 12, seed=3),
                                  lambda: wl.random_kcnf(24, 90, seed=5)])
def test_order_respects_width(make):
    """The derived order never exceeds the decomposition's width, whatever
    bag is the root, and a plan from it stays within width + 1."""
    f = make()
    td, width = td_from_order(f, oracle.minfill_order(f))
    net = W.Network.from_formula(f)
    for root in (0, 2, 7):
        order, w = W.order_from_td(net, td, root_bag=root)
        assert w == width
        assert sorted(order) == list(range(1, f.n + 1))
        assert induced_width(f, list(order)) <= width
    plan = W.Plan(net, kind="order", order=order)
    assert plan.stats()["max_rank"] <= width + 1


def test_isolated_variables_come_first():
    f = wl.Formula(5, [[1, 2], [2, 3]], np.full((5, 2), 0.5))
    net = W.Network.from_formula(f)
    order, width = W.order_from_td(net, "s td 2 2 5\nb 1 1 2\nb 2 2 3\n1 2\n")
    assert list(order[:2]) == [4, 5] and sorted(order) == [1, 2, 3, 4, 5] and width == 1


@pytest.mark.parametrize("td,what", [
    ("b 1 1 2\n", "before"),
    ("s td 1 2 9\nb 1 1 2\n", "vertices"),
    ("s td 2 2 3\nb 1 1 2\nb 2 2 3\n", "not a tree"),
    ("s td 3 2 3\nb 1 1 2\nb 2 3\nb 3 2 3\n1 2\n2 3\n", "not connected"),
    ("s td 2 2 3\nb 1 1 2\nb 2 3\n1 2\n", "clause"),
    ("s td 2 2 3\nb 1 1 2 7\nb 2 2 3\n1 2\n", "out of range"),
    ("s td 2 2 3\nb 1 1 2\nb 2 2 3\n1 1\n", "bad edge"),
    ("s td 1000000000000 2 3\nb 1 1 2\n", "bags in a text"),
])
def test_malformed_decompositions_rejected(td, what):
    f = wl.Formula(3, [[1, 2], [2, 3]], np.full((3, 2), 0.5))
    net = W.Network.from_formula(f)
    with pytest.raises(W.WmcError) as e:
        W.order_from_td(net, td)
    assert e.value.status == 1 and what in str(e.value)


@pytest.mark.parametrize("seed", range(8))
def test_decomposition_plans_replayed_match_oracle(seed):
    """Plans from supplied decompositions, replayed from their device
    descriptors on the CPU, equal the oracle; long clauses (factored into
    chains over auxiliary variables the decomposition never names) too."""
    from fractions import Fraction
    from plan_emulator import emulate, rel_err
    for f in (wl.random_mixed(seed, n_max=12, m_max=24), wl.random_long(seed)):
        td, width = td_from_order(f, oracle.minfill_order(f))
        net = W.Network.from_formula(f)
        order, w = W.order_from_td(net, td, root_bag=1 + seed % 3)
        assert w == width
        plan = W.Plan(net, kind="order", order=order, block=1 + seed % 2)
        got, _ = emulate(plan, f.weights)
        ref = Fraction(oracle.brute(f))
        if ref == 0:
            assert got == 0
        else:
            assert rel_err(got, ref) < 1e-12, (seed, float(got), float(ref))


@pytest.mark.gpu
def test_plan_from_decomposition_matches_oracle():
    from fractions import Fraction
    import torch  # noqa: F401
    f = wl.grid_cnf(8, 16, 0.1, seed=4)
    td, width = td_from_order(f, oracle.minfill_order(f))
    net = W.Network.from_formula(f)
    order, _ = W.order_from_td(net, td, root_bag=5)
    plan = W.Plan(net, kind="order", order=order, block=2)
    v = W.wmc_contract(plan)
    m, e = oracle.bucket(f)
    ref = Fraction(m) * Fraction(2) ** e
    got = Fraction(v.mantissa) * Fraction(2) ** v.exp2
    assert abs(got - ref) <= Fraction(1, 10 ** 12) * abs(ref)
