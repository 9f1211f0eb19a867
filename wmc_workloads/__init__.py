"""Seeded synthetic weighted-CNF workloads.

This module only draws random formulas and weights; it holds none of the
model-counting arithmetic.  Both the GPU library's tests and the CPU oracle
consume what it produces, so it must stay free of any counting logic.

A formula is a :class:`Formula`: ``n`` Boolean variables numbered 1..n,
``clauses`` as lists of DIMACS literals (``+x`` / ``-x``), and ``weights``
as an ``(n, 2)`` float64 array with ``weights[x-1, 0] = W(x, 0)`` and
``weights[x-1, 1] = W(x, 1)``.  Literal weights follow the usual convention
W(x, 1) = w(x) for the positive literal and W(x, 0) = w(not x) = 1 - w(x)
(Definition 1 of the paper allows any real-valued W; the workloads only draw
values in (0, 1)).

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``) and
draws in a fixed, documented order so that an instance is a pure function of
its arguments.
"""

from __future__ import annotations

import dataclasses
import hashlib
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Formula",
    "random_kcnf",
    "grid_cnf",
    "banded_3cnf",
    "batch_instance",
    "serve_structure",
    "serve_queries",
    "SERVE_STRUCTURES",
    "uniform_weights",
    "row_major_order",
    "fig1_formula",
    "psi_formula",
    "random_mixed",
]


@dataclasses.dataclass
class Formula:
    n: int
    clauses: List[List[int]]
    weights: np.ndarray  # (n, 2) float64: [:, 0] = W(x,0), [:, 1] = W(x,1)
    name: str = ""

    def __post_init__(self) -> None:
        self.weights = np.ascontiguousarray(self.weights, dtype=np.float64).reshape(self.n, 2)

    @property
    def m(self) -> int:
        return len(self.clauses)

    def csr(self) -> Tuple[np.ndarray, np.ndarray]:
        """Clauses as (clause_ptr int64[m+1], lits int32[nnz])."""
        ptr = np.zeros(self.m + 1, dtype=np.int64)
        for i, c in enumerate(self.clauses):
            ptr[i + 1] = ptr[i] + len(c)
        lits = np.fromiter((l for c in self.clauses for l in c), dtype=np.int32, count=int(ptr[-1]))
        return ptr, lits

    def flat_weights(self) -> np.ndarray:
        """Weights as float64[2n]: {W(x,0), W(x,1)} for x = 1..n."""
        return np.ascontiguousarray(self.weights.reshape(-1))

    def with_weights(self, weights: np.ndarray) -> "Formula":
        return Formula(self.n, [list(c) for c in self.clauses], np.array(weights, dtype=np.float64), self.name)

    def with_clauses(self, extra: Sequence[Sequence[int]]) -> "Formula":
        return Formula(self.n, [list(c) for c in self.clauses] + [list(c) for c in extra],
                       self.weights.copy(), self.name)

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        ptr, lits = self.csr()
        h.update(ptr.tobytes())
        h.update(lits.tobytes())
        h.update(self.weights.tobytes())
        return h.hexdigest()[:16]

    def dimacs(self) -> str:
        out = [f"p cnf {self.n} {self.m}"]
        for c in self.clauses:
            out.append(" ".join(str(l) for l in c) + " 0")
        for x in range(1, self.n + 1):
            out.append(f"c weight {x} {self.weights[x-1, 1]!r} {self.weights[x-1, 0]!r}")
        return "\n".join(out) + "\n"


def uniform_weights(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """w(x) ~ U(lo, hi); returns (n, 2) with columns {1 - w, w}."""
    w = rng.uniform(lo, hi, size=n)
    return np.stack([1.0 - w, w], axis=1)


def _signed(rng: np.random.Generator, vars_: np.ndarray) -> List[int]:
    signs = rng.integers(0, 2, size=len(vars_))
    return [int(v) if s else -int(v) for v, s in zip(vars_, signs)]


def random_kcnf(n: int, m: int, seed: int, k: int = 3, wlo: float = 0.1, whi: float = 0.9) -> Formula:
    """Uniform random k-CNF: each clause picks k distinct variables without
    replacement, each sign a fair coin.  Clauses are drawn first, then weights."""
    rng = np.random.default_rng(seed)
    clauses = []
    for _ in range(m):
        vs = rng.choice(n, size=k, replace=False) + 1
        clauses.append(_signed(rng, vs))
    weights = uniform_weights(rng, n, wlo, whi)
    return Formula(n, clauses, weights, f"random{k}cnf-n{n}-m{m}-s{seed}")


def _planted_signed(rng: np.random.Generator, vars_: np.ndarray, sigma: np.ndarray) -> List[int]:
    """Signs drawn uniformly among the patterns the planted assignment sigma
    satisfies (rejection: redraw while every literal is false under sigma)."""
    while True:
        signs = rng.integers(0, 2, size=len(vars_))
        if any(int(sigma[int(v) - 1]) == int(s) for v, s in zip(vars_, signs)):
            return [int(v) if s else -int(v) for v, s in zip(vars_, signs)]


def grid_cnf(rows: int, cols: int, ternary_frac: float, seed: int,
             n_global: int = 0, wlo: float = 0.1, whi: float = 0.9, planted: bool = True) -> Formula:
    """Lattice CNF on a rows x cols variable grid, variable (i, j) = i*cols + j + 1.

    Each lattice edge (horizontal edges of a cell first, then its vertical
    edge, cells in row-major order) gives two binary clauses over its two
    endpoints with independent fair-coin signs.  Then round(ternary_frac *
    #edges) ternary clauses, each over 3 distinct corners of a uniformly drawn
    plaquette (a local reading: the clause stays inside one lattice square).
    Then ``n_global`` random 3-clauses over 3 distinct variables of the whole
    grid.  Weights last, w ~ U(wlo, whi).

    With ``planted`` (the default) a hidden assignment sigma ~ U{0,1}^n is
    drawn first and every clause's signs are drawn uniformly among the sign
    patterns sigma satisfies.  With independent fair-coin signs two binary
    clauses per edge force units that collide almost surely (e.g. (a|b) and
    (a|~b) force a), so the lattice is unsatisfiable and W = 0; the planted
    reading keeps the same structure with W > 0."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    sigma = rng.integers(0, 2, size=n) if planted else None
    sign = (lambda vs: _planted_signed(rng, vs, sigma)) if planted else (lambda vs: _signed(rng, vs))
    vid = lambda i, j: i * cols + j + 1
    clauses: List[List[int]] = []
    n_edges = 0
    for i in range(rows):
        for j in range(cols):
            nb = []
            if j + 1 < cols:
                nb.append((i, j + 1))
            if i + 1 < rows:
                nb.append((i + 1, j))
            for (a, b) in nb:
                n_edges += 1
                for _ in range(2):
                    clauses.append(sign(np.array([vid(i, j), vid(a, b)])))
    n_tern = int(round(ternary_frac * n_edges))
    for _ in range(n_tern):
        pi = int(rng.integers(0, rows - 1))
        pj = int(rng.integers(0, cols - 1))
        corners = [vid(pi, pj), vid(pi, pj + 1), vid(pi + 1, pj), vid(pi + 1, pj + 1)]
        pick = rng.choice(4, size=3, replace=False)
        clauses.append(sign(np.array([corners[p] for p in pick])))
    for _ in range(n_global):
        vs = rng.choice(n, size=3, replace=False) + 1
        clauses.append(sign(vs))
    weights = uniform_weights(rng, n, wlo, whi)
    return Formula(n, clauses, weights, f"grid{rows}x{cols}-t{ternary_frac}-g{n_global}-s{seed}")


def row_major_order(rows: int, cols: int) -> np.ndarray:
    """Elimination order sweeping the lattice row by row (variables 1..n)."""
    return np.arange(1, rows * cols + 1, dtype=np.int32)


def banded_3cnf(n: int, m: int, window: int, seed: int, wlo: float = 0.05, whi: float = 0.95) -> Formula:
    """Banded random 3-CNF: each clause draws a window start s ~ U{0..n-window}
    and then 3 distinct variables uniformly from [s, s+window), signs fair."""
    rng = np.random.default_rng(seed)
    window = min(window, n)
    clauses = []
    for _ in range(m):
        s = int(rng.integers(0, n - window + 1))
        vs = s + rng.choice(window, size=3, replace=False) + 1
        clauses.append(_signed(rng, vs))
    weights = uniform_weights(rng, n, wlo, whi)
    return Formula(n, clauses, weights, f"banded3cnf-n{n}-m{m}-W{window}-s{seed}")


def batch_instance(i: int, window: int = 20) -> Formula:
    """Instance i of the 512-instance batch: seed i; n ~ U{30..150},
    ratio ~ U(3.0, 4.2), m = round(ratio * n); banded 3-CNF with the given
    window; weights U(0.1, 0.9)."""
    rng = np.random.default_rng(i)
    n = int(rng.integers(30, 151))
    ratio = float(rng.uniform(3.0, 4.2))
    m = int(round(ratio * n))
    window = min(window, n)
    clauses = []
    for _ in range(m):
        s = int(rng.integers(0, n - window + 1))
        vs = s + rng.choice(window, size=3, replace=False) + 1
        clauses.append(_signed(rng, vs))
    weights = uniform_weights(rng, n, 0.1, 0.9)
    return Formula(n, clauses, weights, f"batch-{i}")


# (local ternary fraction, number of global 3-clauses) for the 8 serving structures
SERVE_STRUCTURES: Tuple[Tuple[float, int], ...] = (
    (0.05, 0), (0.10, 0), (0.20, 0), (0.30, 0), (0.05, 4), (0.10, 4), (0.10, 8), (0.20, 8))


def serve_structure(s: int) -> Formula:
    """Serving structure s (0..7): a 10 x 20 lattice (200 variables) with the
    lattice's edge clauses, a local ternary fraction f and k global 3-clauses,
    drawn with seed s.  Its weights are a placeholder; queries bring their own."""
    f, k = SERVE_STRUCTURES[s]
    return grid_cnf(10, 20, f, seed=s, n_global=k)


def serve_queries(n_queries: int, rate: float, seed: int = 0, n_structures: int = 8,
                  n_vars: int = 200) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Poisson stream of weight queries.

    Returns (arrival_seconds float64[q], structure int32[q], weights
    float64[q, n_vars, 2]).  Draw order: structure ids, then unit-rate
    exponential gaps (scaled by 1/rate), then the weight vectors."""
    rng = np.random.default_rng(seed)
    structure = rng.integers(0, n_structures, size=n_queries).astype(np.int32)
    gaps = rng.exponential(1.0, size=n_queries) / float(rate)
    arrivals = np.cumsum(gaps)
    w = rng.uniform(0.1, 0.9, size=(n_queries, n_vars))
    weights = np.stack([1.0 - w, w], axis=2)
    return arrivals, structure, weights


def fig1_formula(weights: Optional[np.ndarray] = None) -> Formula:
    """The four-clause formula of the paper's Figure 1 over w, x, y, z
    (numbered 1, 2, 3, 4): (w | x | ~y) & (w | y | z) & (~x | ~y) & (~y | ~z)."""
    if weights is None:
        weights = np.full((4, 2), 0.5)
    return Formula(4, [[1, 2, -3], [1, 3, 4], [-2, -3], [-3, -4]], weights, "fig1")


def psi_formula(n: int, weights: Optional[np.ndarray] = None) -> Formula:
    """psi = (x_1 | ... | x_n) & (~x_1 | ... | ~x_n), the example the paper
    uses to contrast incidence-graph and primal-graph planning."""
    if weights is None:
        weights = np.full((n, 2), 0.5)
    return Formula(n, [list(range(1, n + 1)), [-x for x in range(1, n + 1)]], weights, f"psi{n}")


def random_mixed(seed: int, n_max: int = 14, m_max: int = 30, k_max: int = 5,
                 negative: bool = False, allow_empty: bool = True) -> Formula:
    """Small formulas with the awkward cases mixed in: clause lengths 1..k_max,
    repeated literals, tautologies (x | ~x | ...), repeated clauses, variables
    in no clause, an occasional empty clause, and (if ``negative``) weights of
    either sign.  For parity sweeps on tiny inputs."""
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.integers(1, n_max + 1))
    m = int(rng.integers(0, m_max + 1))
    clauses: List[List[int]] = []
    for _ in range(m):
        r = rng.random()
        if allow_empty and r < 0.01:
            clauses.append([])
            continue
        k = int(rng.integers(1, min(k_max, n) + 1))
        vs = rng.choice(n, size=k, replace=False) + 1
        c = _signed(rng, vs)
        if r < 0.08:                      # repeated literal
            c.append(c[0])
        elif r < 0.12:                    # tautology
            c.append(-c[0])
        elif r < 0.16 and clauses:        # repeated clause
            c = list(clauses[int(rng.integers(0, len(clauses)))])
        clauses.append(c)
    if negative:
        w = rng.uniform(-1.0, 1.0, size=(n, 2))
    else:
        w = rng.uniform(0.05, 1.0, size=(n, 2))
    return Formula(n, clauses, w, f"mixed-{seed}")


def random_long(seed: int, n: int = 13, n_long: int = 2, k_lo: int = 9, k_hi: int = 12,
                n_short: int = 16) -> Formula:
    """Formulas with long clauses (k_lo..k_hi-1 distinct literals, the first
    with a repeated literal) among random 3-clauses, w ~ U(0.1, 0.9).  Long
    clauses are the ones the network builder factors into chains."""
    rng = np.random.default_rng(20_000 + seed)
    clauses: List[List[int]] = []
    for _ in range(n_long):
        k = int(rng.integers(k_lo, k_hi))
        clauses.append(_signed(rng, rng.choice(n, size=k, replace=False) + 1))
    if clauses:
        clauses[0].append(clauses[0][0])
    for _ in range(n_short):
        clauses.append(_signed(rng, rng.choice(n, size=3, replace=False) + 1))
    w = rng.uniform(0.1, 0.9, size=n)
    return Formula(n, clauses, np.stack([1 - w, w], axis=1), f"long-{seed}")
