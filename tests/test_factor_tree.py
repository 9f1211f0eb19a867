"""FactorTree (Theorem 3): networks factored along a tree decomposition of
the incidence graph and planned with the elimination order that follows
it.  Host only (plans replayed on the CPU by the descriptor emulator),
except the GPU cases at the end."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl
from plan_emulator import emulate


def incidence_adjacency(f):
    """Variables 1..n, clause c as vertex n + 1 + c."""
    adj = {v: set() for v in range(1, f.n + len(f.clauses) + 1)}
    for c, cl in enumerate(f.clauses):
        cv = f.n + 1 + c
        for l in cl:
            adj[abs(l)].add(cv)
            adj[cv].add(abs(l))
    return adj


def min_degree_order(adj):
    adj = {v: set(s) for v, s in adj.items()}
    order = []
    while adj:
        v = min(adj, key=lambda u: (len(adj[u]), u))
        nb = adj.pop(v)
        for a in nb:
            adj[a] |= nb - {a}
            adj[a].discard(v)
        order.append(v)
    return order


def td_text(adj, order):
    """Decomposition of an elimination order: bag(v) = v and its later
    neighbours in the filled graph, joined to the bag of the earliest
    eliminated of those (or the next bag when there are none)."""
    adj = {v: set(s) for v, s in adj.items()}
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
    lines = [f"s td {len(bags)} {width + 1} {len(order)}"]
    lines += ["b %d %s" % (i + 1, " ".join(map(str, b))) for i, b in enumerate(bags)]
    lines += ["%d %d" % e for e in edges]
    return "\n".join(lines) + "\n", width


def incidence_td(f):
    adj = incidence_adjacency(f)
    return td_text(adj, min_degree_order(adj))


def psi_td(n):
    """Width-2 decomposition of psi's incidence graph: a path of bags
    {x_i, C1, C2}."""
    c1, c2 = n + 1, n + 2
    lines = [f"s td {n} 3 {n + 2}"] + [f"b {i} {i} {c1} {c2}" for i in range(1, n + 1)]
    lines += [f"{i} {i + 1}" for i in range(1, n)]
    return "\n".join(lines) + "\n"


def psi_value(w):
    """Closed form of psi = (x_1 v ... v x_n) & (-x_1 v ... v -x_n): every
    assignment but all-false and all-true."""
    tot, f0, f1 = Fraction(1), Fraction(1), Fraction(1)
    for w0, w1 in w:
        tot *= Fraction(w0) + Fraction(w1)
        f0 *= Fraction(w0)
        f1 *= Fraction(w1)
    return tot - f0 - f1


def rel(a, b):
    return 0.0 if a == b else float(abs(a - b) / max(abs(a), abs(b)))


def test_psi_from_a_width_2_incidence_decomposition():
    """psi with n = 200: its primal graph has treewidth n - 1, its incidence
    graph 2.  FactorTree on the width-2 decomposition plans at storage rank
    3 (index rank 6), within ceil(4(w + 1)/3) = 4, and the plan computes the
    closed form."""
    n = 200
    f = wl.psi_formula(n)
    net = W.Network.from_td(f, psi_td(n))
    assert net.td_width == 2
    p = W.Plan(net, kind="network")
    st = p.stats()
    assert st["max_rank"] <= math.ceil(4 * (2 + 1) / 3) == 4
    got, _ = emulate(p, f.weights)
    assert rel(got, psi_value(np.asarray(f.weights))) <= 1e-12


@pytest.mark.parametrize("seed", range(12))
def test_rank_bound_on_random_decompositions(seed):
    """Random, banded and mixed formulas with decompositions of their
    incidence graphs (min-degree elimination): the plan's storage rank stays
    within ceil(4(w + 1)/3) for width w, and the plan computes W."""
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        f = wl.random_kcnf(int(rng.integers(12, 20)), int(rng.integers(30, 60)), seed=seed)
    elif kind == 1:
        f = wl.banded_3cnf(int(rng.integers(40, 80)), int(rng.integers(120, 240)), 8, seed=seed)
    else:
        f = wl.random_mixed(seed, n_max=16, m_max=30, k_max=9)
    td, w = incidence_td(f)
    net = W.Network.from_td(f, td)
    assert net.td_width == w
    p = W.Plan(net, kind="network")
    bound = math.ceil(4 * (w + 1) / 3)
    assert p.stats()["max_rank"] <= bound, (p.stats()["max_rank"], w, bound)
    got, _ = emulate(p, f.weights)
    ref = Fraction(oracle.brute(f)) if f.n <= 20 else Fraction(oracle.bucket_value(f))
    assert (got == 0) if ref == 0 else rel(got, ref) <= 1e-12


def test_long_clauses_and_the_root_bag():
    """Clauses of 10 to 14 literals spread over many bags; every root bag
    choice gives W."""
    f = wl.random_long(3)
    td, w = incidence_td(f)
    ref = Fraction(oracle.brute(f))
    nb = int(td.split("\n")[0].split()[2])
    for root in (0, nb // 2, nb):
        p = W.Plan(W.Network.from_td(f, td, root_bag=root), kind="network")
        got, _ = emulate(p, f.weights)
        assert rel(got, ref) <= 1e-12, root


@pytest.mark.parametrize("bad,msg", [
    (lambda td: td.replace("s td", "s tdx"), "bad solution line"),
    (lambda td: td + "1 2\n", "not a tree"),
    (lambda td: "\n".join(l for l in td.split("\n") if not l.startswith("b 1 ")) + "\n", "no bag holds"),
])
def test_malformed_decompositions_are_refused(bad, msg):
    f = wl.psi_formula(6)
    with pytest.raises(W.WmcError) as e:
        W.Network.from_td(f, bad(psi_td(6)))
    assert e.value.status == 1
    assert msg in str(e.value)


def test_vertex_count_must_cover_clauses():
    f = wl.psi_formula(6)
    with pytest.raises(W.WmcError) as e:
        W.Network.from_td(f, psi_td(6).replace("s td 6 3 8", "s td 6 3 6"))
    assert e.value.status == 1


def test_network_order_needs_a_decomposition():
    f = wl.psi_formula(6)
    with pytest.raises(W.WmcError) as e:
        W.Plan(W.Network.from_formula(f), kind="network")
    assert e.value.status == 1


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_psi_factor_tree_on_gpu(precision, tol):
    """psi with n = 200 planned by FactorTree from its width-2 incidence
    decomposition, contracted on the GPU, against the closed form."""
    n = 200
    f = wl.psi_formula(n)
    p = W.Plan(W.Network.from_td(f, psi_td(n)), kind="network", precision=precision)
    assert p.stats()["max_rank"] <= 4
    v = W.wmc_contract(p)
    got = Fraction(v.mantissa) * Fraction(2) ** v.exp2
    assert rel(got, psi_value(np.asarray(f.weights))) <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(4))
def test_factor_tree_random_on_gpu(seed):
    f = wl.banded_3cnf(90, 330, 10, seed=seed)
    td, w = incidence_td(f)
    p = W.Plan(W.Network.from_td(f, td), kind="network")
    v = W.wmc_contract(p)
    m, e = oracle.bucket(f)
    ref = Fraction(m) * Fraction(2) ** e
    got = Fraction(v.mantissa) * Fraction(2) ** v.exp2 if v.mantissa else Fraction(0)
    assert (got == 0) if ref == 0 else rel(got, ref) <= 1e-12
