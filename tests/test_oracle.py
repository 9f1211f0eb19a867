"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library.  Each pin is chosen so that a plausible
slip in the oracle (a dropped weight, a swapped sign, a wrong exponent, a
transposed index) fails at least one of them:

* brute force (O1) is the definition of the weighted model count
  (Definition 1) written out; bucket elimination (O2), the exact integer
  elimination (O3) and the literal Theorem-2 network (O4) must reproduce it;
* closed forms: the empty formula, a single clause, the psi family of the
  planning section, the Figure 1 formula (count derived by hand), the
  implication chain (transfer-matrix form) far below the double range;
* invariants: variable-disjoint product, literal flip, monotonicity,
  elimination-order independence, conditioning (slicing) identity.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import wmc_workloads as wl
from wmc_workloads import Formula


def rel(a, b):
    if a == b:
        return 0.0
    return abs(a - b) / max(abs(a), abs(b))


def bucket_val(f, order=None):
    m, e = oracle.bucket(f, order)
    return math.ldexp(m, e)


# --------------------------------------------------------------- Figure 1
def test_fig1_network_structure():
    """Figure 1: the reduction of the four-clause formula has 8 tensors and
    10 indices; variable degrees w 2, x 2, y 4, z 2; clause ranks 3, 3, 2, 2."""
    f = wl.fig1_formula()
    tensors, n_idx = oracle.theorem2_network(f)
    assert len(tensors) == 8
    assert n_idx == 10
    ranks = [t.ndim for t, _ in tensors]
    assert ranks[:4] == [3, 3, 2, 2]            # B_C
    assert ranks[4:] == [2, 2, 4, 2]            # A_w, A_x, A_y, A_z


def test_fig1_value_all_half():
    """7 of the 16 assignments satisfy the Figure 1 formula: W = 7/16 at w = 1/2."""
    f = wl.fig1_formula()
    assert oracle.brute(f) == 7 / 16
    assert bucket_val(f) == 7 / 16
    assert oracle.exact_count(f) == 7
    assert oracle.einsum_network(f) == 7 / 16


def test_fig1_closed_form_random_weights():
    """Hand enumeration of the Figure 1 formula: the models are w=1,x=0,y=1,z=0
    and, with y=0, any x and (w,z) != (0,0)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        W = rng.uniform(0.05, 1.0, size=(4, 2))
        f = wl.fig1_formula(W)
        w0, w1 = W[0]
        x0, x1 = W[1]
        y0, y1 = W[2]
        z0, z1 = W[3]
        ref = w1 * x0 * y1 * z0 + y0 * (x0 + x1) * (w1 * z0 + w0 * z1 + w1 * z1)
        assert rel(oracle.brute(f), ref) < 1e-14
        assert rel(bucket_val(f), ref) < 1e-14
        assert rel(oracle.einsum_network(f), ref) < 1e-14


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [0, 1, 5, 17])
def test_empty_formula(n):
    """No clauses: W = prod_x (W(x,0) + W(x,1)); 1 when the weights sum to 1."""
    rng = np.random.default_rng(n)
    W = rng.uniform(0.1, 2.0, size=(n, 2))
    f = Formula(n, [], W)
    ref = float(np.prod(W.sum(axis=1))) if n else 1.0
    assert rel(oracle.brute(f), ref) < 1e-14
    assert rel(bucket_val(f), ref) < 1e-14
    w = rng.uniform(0.1, 0.9, size=n)
    g = Formula(n, [], np.stack([1 - w, w], axis=1))
    assert abs(bucket_val(g) - 1.0) < 1e-14


def test_single_clause():
    """One clause C: W = prod_all (W0+W1) - prod_{x in C} W(x, falsifying) * prod_{x not in C} (W0+W1)."""
    rng = np.random.default_rng(7)
    for trial in range(30):
        n = int(rng.integers(1, 12))
        k = int(rng.integers(1, n + 1))
        vs = rng.choice(n, size=k, replace=False) + 1
        c = [int(v) if rng.integers(0, 2) else -int(v) for v in vs]
        W = rng.uniform(0.05, 1.0, size=(n, 2))
        f = Formula(n, [c], W)
        tot = np.prod(W.sum(axis=1))
        fals = 1.0
        for l in c:
            x = abs(l)
            fals *= W[x - 1, 0] if l > 0 else W[x - 1, 1]
        for x in range(1, n + 1):
            if x not in {abs(l) for l in c}:
                fals *= W[x - 1].sum()
        ref = tot - fals
        assert rel(oracle.brute(f), ref) < 1e-13
        assert rel(bucket_val(f), ref) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 8, 20])
def test_psi_family(n):
    """psi = (OR x_i) & (OR ~x_i): every assignment but all-0 and all-1 is a
    model: W = prod(W0+W1) - prod W(x,0) - prod W(x,1); #models = 2^n - 2."""
    rng = np.random.default_rng(n)
    W = rng.uniform(0.05, 1.0, size=(n, 2))
    f = wl.psi_formula(n, W)
    ref = np.prod(W.sum(axis=1)) - np.prod(W[:, 0]) - np.prod(W[:, 1])
    if n <= 20:
        assert rel(oracle.brute(f), ref) < 1e-12
    assert rel(bucket_val(f), ref) < 1e-12
    assert oracle.exact_count(wl.psi_formula(n)) == 2 ** n - 2


def test_implication_chain_far_below_double_range():
    """Chain (~x_i | x_{i+1}), i < n: the models are 0..01..1, so
    W = sum_k prod_{i<=k} W(x_i,0) prod_{i>k} W(x_i,1).  With n = 3000 and
    weights near 0.3, W ~ 2^-5000: only a carried exponent can represent it.
    Weights are dyadic (K/256), so the reference is an exact integer sum."""
    n = 3000
    rng = np.random.default_rng(3)
    K = rng.integers(51, 103, size=(n, 2))          # ~ U(0.2, 0.4) in units of 1/256
    W = K / 256.0
    f = Formula(n, [[-i, i + 1] for i in range(1, n)], W)
    suf = [1] * (n + 1)
    for i in range(n - 1, -1, -1):
        suf[i] = suf[i + 1] * int(K[i, 1])
    tot = 0
    pre = 1
    for k in range(n + 1):
        tot += pre * suf[k]
        if k < n:
            pre *= int(K[k, 0])
    ref_log2 = (tot.bit_length() - 64 + math.log2(tot >> (tot.bit_length() - 64))) - 8 * n
    m, e = oracle.bucket(f, order=list(range(1, n + 1)))
    assert 0.5 <= m < 1.0
    assert abs(oracle.to_log2(m, e) - ref_log2) < 1e-9


# --------------------------------------------------------------- brute force vs eliminations
@pytest.mark.parametrize("negative", [False, True])
def test_bucket_matches_brute_force(negative):
    """O2 against O1 on 300 mixed small formulas (repeated literals,
    tautologies, repeated and empty clauses, unused variables)."""
    worst = 0.0
    for s in range(300):
        f = wl.random_mixed(s, negative=negative)
        ref = oracle.brute(f)
        got = bucket_val(f)
        if negative:
            scale = float(np.prod(np.abs(f.weights).sum(axis=1)))
            assert abs(got - ref) <= 1e-12 * scale, (s, got, ref)
        else:
            if ref == 0.0:
                assert got == 0.0, s
            else:
                worst = max(worst, rel(got, ref))
    assert worst < 1e-12


def test_exact_count_matches_brute_force():
    """O3 with all weights 1 counts models; brute force with weights 1.0 sums
    exact integers (counts far below 2^53)."""
    for s in range(60):
        f = wl.random_mixed(s, n_max=12)
        ones = f.with_weights(np.ones((f.n, 2)))
        assert oracle.exact_count(f) == int(oracle.brute(ones)), s


def test_exact_dyadic_weights():
    """Dyadic weights k/2^b: O3 on the integers k gives W * 2^(b n) exactly;
    O1 on the dyadic doubles agrees to rounding."""
    b = 4
    for s in range(30):
        f = wl.random_mixed(s, n_max=10)
        rng = np.random.default_rng(s)
        K = rng.integers(0, 2 ** b + 1, size=(f.n, 2))
        exact = oracle.exact_count(f, [tuple(map(int, r)) for r in K])
        g = f.with_weights(K / 2.0 ** b)
        assert rel(oracle.brute(g), exact / 2.0 ** (b * f.n)) < 1e-14 or exact == 0


def test_einsum_network_matches_brute_force():
    """O4, the literal Theorem-2 network (dense COPY tensors, one index per
    occurrence), contracted by numpy.einsum, equals O1 (Theorem 2)."""
    checked = 0
    for s in range(200):
        f = wl.random_mixed(s, n_max=8, m_max=10, k_max=3)
        _, n_idx = oracle.theorem2_network(f)
        if n_idx > 30:
            continue
        ref = oracle.brute(f)
        got = oracle.einsum_network(f)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), s
        checked += 1
    assert checked > 100


def test_config1_seed_sweep_brute_vs_bucket():
    """Random 3-CNF, 20 variables, 85 clauses: O2 equals O1 on seeds 0..39."""
    for s in range(40):
        f = wl.random_kcnf(20, 85, s)
        ref = oracle.brute(f)
        got = bucket_val(f)
        if ref == 0.0:
            assert got == 0.0
        else:
            assert rel(got, ref) < 1e-12


# --------------------------------------------------------------- invariants
def test_elimination_order_independence():
    """Any elimination order gives the same W (up to rounding)."""
    rng = np.random.default_rng(5)
    for s in range(40):
        f = wl.random_mixed(s, n_max=14)
        ref = bucket_val(f)
        for _ in range(3):
            order = rng.permutation(f.n) + 1
            got = bucket_val(f, order)
            assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300), s


def test_variable_disjoint_product():
    """W(phi1 & phi2) = W(phi1) W(phi2) when they share no variable."""
    for s in range(20):
        a = wl.random_kcnf(8, 20, s)
        b = wl.random_kcnf(7, 14, 100 + s)
        shifted = [[(abs(l) + a.n) * (1 if l > 0 else -1) for l in c] for c in b.clauses]
        ab = Formula(a.n + b.n, a.clauses + shifted, np.vstack([a.weights, b.weights]))
        ref = oracle.brute(a) * oracle.brute(b)
        got = bucket_val(ab)
        assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-300)


def test_literal_flip():
    """Negating every occurrence of x and swapping W(x,0) <-> W(x,1) leaves W unchanged."""
    rng = np.random.default_rng(9)
    for s in range(30):
        f = wl.random_mixed(s, n_max=12, allow_empty=False)
        x = int(rng.integers(1, f.n + 1))
        cl = [[-l if abs(l) == x else l for l in c] for c in f.clauses]
        W = f.weights.copy()
        W[x - 1] = W[x - 1, ::-1]
        g = Formula(f.n, cl, W)
        assert abs(bucket_val(g) - bucket_val(f)) <= 1e-13 * max(abs(bucket_val(f)), 1e-300)


def test_monotone_under_added_clause():
    """With non-negative weights, adding a clause never increases W."""
    for s in range(40):
        f = wl.random_mixed(s, n_max=12)
        g = wl.random_mixed(s + 1000, n_max=12)
        extra = [[l for l in c if abs(l) <= f.n] for c in g.clauses[:3]]
        extra = [c for c in extra if c]
        h = f.with_clauses(extra)
        assert oracle.brute(h) <= oracle.brute(f) * (1 + 1e-14)


def test_conditioning_identity():
    """Slicing identity (index slicing theorem): W(phi) = sum over eta of
    W(phi & unit clauses fixing the sliced variables to eta)."""
    rng = np.random.default_rng(11)
    for s in range(20):
        f = wl.random_kcnf(14, 40, 500 + s)
        k = 3
        vs = rng.choice(f.n, size=k, replace=False) + 1
        total = 0.0
        for eta in range(2 ** k):
            units = [[int(v) if (eta >> i) & 1 else -int(v)] for i, v in enumerate(vs)]
            total += bucket_val(f.with_clauses(units))
        ref = oracle.brute(f)
        assert abs(total - ref) <= 1e-13 * max(abs(ref), 1e-300)


def test_minfill_width_config1():
    """Min-fill on the 20-variable random 3-CNF gives a modest width (sanity)."""
    f = wl.random_kcnf(20, 85, 0)
    _, _, width = oracle.bucket(f, return_width=True)
    assert 8 <= width <= 19


def test_invalid_inputs_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.brute(Formula(2, [[3]], np.ones((2, 2))))
    with pytest.raises(oracle.OracleError):
        oracle.bucket(Formula(2, [[0, 1]], np.ones((2, 2))))
    with pytest.raises(oracle.OracleError):
        oracle.bucket(Formula(2, [[1, 2]], np.ones((2, 2))), order=[1, 1])
