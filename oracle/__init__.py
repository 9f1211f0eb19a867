"""CPU oracle for literal-weighted model counting -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library
(``paper_2006_15512_amd``) and never imports it.

Methods (each an exact reorganisation of Definition 1, the literal-weighted
model count W(phi) = sum_tau phi(tau) prod_x W(x, tau(x))):

* ``brute``        O1, the definition enumerated (C, n <= 30).
* ``bucket``       O2, FP64 bucket elimination with a power-of-two exponent
                   per message (C), returns (mantissa, exp2).
* ``exact_count``  O3, the same elimination over Python integers: exact for
                   integer weights (all-1 weights give the model count).
* ``einsum_network`` O4, the literal network of Theorem 2 (one index per
                   variable occurrence, dense COPY/weight tensors A_x and
                   clause tensors B_C) contracted by ``numpy.einsum``; only for
                   networks of at most 52 indices.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the C oracle with gcc (-O2 -fopenmp) into oracle/liboracle.so;
    with ``sanitize``, an AddressSanitizer + UndefinedBehaviorSanitizer build
    into oracle/liboracle_san.so (load it with WMC_ORACLE_LIBRARY and the
    sanitizer runtime preloaded)."""
    if sanitize:
        tmp = _SAN_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-result", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SAN_LIB)
        return _SAN_LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-result", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None and os.environ.get("WMC_ORACLE_LIBRARY"):
        _lib = _bind(ctypes.CDLL(os.environ["WMC_ORACLE_LIBRARY"]))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    lib.oracle_brute.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P]
    lib.oracle_brute.restype = ctypes.c_int
    lib.oracle_bucket.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P,
                                  ctypes.c_int32, P, P, P]
    lib.oracle_bucket.restype = ctypes.c_int
    lib.oracle_minfill.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P]
    lib.oracle_minfill.restype = ctypes.c_int
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _csr(clauses: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    ptr = np.zeros(len(clauses) + 1, dtype=np.int64)
    for i, c in enumerate(clauses):
        ptr[i + 1] = ptr[i] + len(c)
    lits = np.array([l for c in clauses for l in c], dtype=np.int32)
    return ptr, lits


def _check(st: int, what: str) -> None:
    if st != 0:
        raise OracleError(f"{what} failed with status {st} "
                          f"({ {1: 'invalid input', 2: 'out of memory', 3: 'too big'}.get(st, '?') })")


def brute(f) -> float:
    """O1: W(phi) by enumerating all 2^n assignments (n <= 30)."""
    lib = _load()
    ptr, lits = _csr(f.clauses)
    w = np.ascontiguousarray(np.asarray(f.weights, dtype=np.float64).reshape(-1))
    out = ctypes.c_double()
    _check(lib.oracle_brute(f.n, len(f.clauses), _ptr(ptr), _ptr(lits), _ptr(w),
                            ctypes.byref(out)), "oracle_brute")
    return out.value


def bucket(f, order: Optional[Sequence[int]] = None, max_log2: int = 30,
           return_width: bool = False):
    """O2: FP64 bucket elimination.  Returns (mantissa, exp2) with W = m * 2^e,
    |m| in [0.5, 1) or m == 0.  ``order`` is a permutation of 1..n (default:
    the oracle's own min-fill order, ties to the lowest id)."""
    lib = _load()
    ptr, lits = _csr(f.clauses)
    w = np.ascontiguousarray(np.asarray(f.weights, dtype=np.float64).reshape(-1))
    o = None
    if order is not None:
        o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        if o.size != f.n:
            raise OracleError("order must be a permutation of 1..n")
    mant = ctypes.c_double()
    ex = ctypes.c_int64()
    width = ctypes.c_int32()
    _check(lib.oracle_bucket(f.n, len(f.clauses), _ptr(ptr), _ptr(lits), _ptr(w),
                             _ptr(o) if o is not None else None, int(max_log2),
                             ctypes.byref(mant), ctypes.byref(ex), ctypes.byref(width)),
           "oracle_bucket")
    if return_width:
        return mant.value, ex.value, width.value
    return mant.value, ex.value


def bucket_value(f, order=None, max_log2: int = 30) -> float:
    m, e = bucket(f, order, max_log2)
    return math.ldexp(m, e)


def minfill_order(f) -> np.ndarray:
    """The oracle's own min-fill order (ties to the lowest variable id)."""
    lib = _load()
    ptr, lits = _csr(f.clauses)
    out = np.zeros(max(f.n, 1), dtype=np.int32)
    _check(lib.oracle_minfill(f.n, len(f.clauses), _ptr(ptr), _ptr(lits), _ptr(out)),
           "oracle_minfill")
    return out[: f.n]


def to_log2(mant: float, exp2: int) -> float:
    """log2 |m * 2^e| without forming the (possibly subnormal) double."""
    if mant == 0.0:
        return -math.inf
    return math.log2(abs(mant)) + exp2


# ---------------------------------------------------------------------------
# O3: exact elimination over Python integers
# ---------------------------------------------------------------------------
def _clause_factor(clause: Sequence[int]):
    vs = sorted({abs(l) for l in clause})
    shape = (2,) * len(vs)
    t = np.zeros(shape, dtype=object)
    for idx in np.ndindex(*shape) if vs else [()]:
        val = dict(zip(vs, idx))
        sat = any((l > 0 and val[abs(l)] == 1) or (l < 0 and val[abs(l)] == 0) for l in clause)
        t[idx] = 1 if sat else 0
    return vs, t


def _expand(vs: List[int], t: np.ndarray, union: List[int]) -> np.ndarray:
    """View factor t (axes = vs, ascending) over the union scope by broadcasting."""
    shape = [2 if v in vs else 1 for v in union]
    return t.reshape(shape)


def exact_count(f, int_weights: Optional[Sequence[Tuple[int, int]]] = None,
                order: Optional[Sequence[int]] = None) -> int:
    """O3: exact W(phi) for integer weights by bucket elimination on Python ints.

    ``int_weights[x-1] = (W(x,0), W(x,1))``; default all 1, i.e. the number
    of models.  Dyadic weights k/2^b are handled by the caller scaling every
    weight by 2^b (the result is then W * 2^(b n))."""
    n = f.n
    if int_weights is None:
        int_weights = [(1, 1)] * n
    factors = []
    for c in f.clauses:
        vs, t = _clause_factor(c)
        factors.append((vs, t))
    for x in range(1, n + 1):
        a, b = int_weights[x - 1]
        factors.append(([x], np.array([int(a), int(b)], dtype=object)))
    if order is None:
        order = minfill_order(f)
    for x in order:
        x = int(x)
        bucket_f = [fv for fv in factors if x in fv[0]]
        rest = [fv for fv in factors if x not in fv[0]]
        union = sorted({v for vs, _ in bucket_f for v in vs})
        prod = None
        for vs, t in bucket_f:
            e = _expand(vs, t, union)
            prod = e if prod is None else prod * e
        prod = np.broadcast_to(prod, (2,) * len(union))
        ax = union.index(x)
        msg = prod.sum(axis=ax)
        out_vs = [v for v in union if v != x]
        if not out_vs:
            msg = np.array(msg, dtype=object).reshape(())
        rest.append((out_vs, np.asarray(msg, dtype=object)))
        factors = rest
    total = 1
    for vs, t in factors:
        assert not vs
        total *= int(t.item() if isinstance(t, np.ndarray) else t)
    return int(total)


# ---------------------------------------------------------------------------
# O4: the literal Theorem-2 network, contracted by numpy.einsum
# ---------------------------------------------------------------------------
def theorem2_network(f):
    """Build the dense network of Theorem 2: one index per (x, C) occurrence
    (duplicate literals collapse to one index per clause), A_x over the
    occurrences of x (W(x,0) on all-0, W(x,1) on all-1, else 0), B_C over the
    occurrences in C (1 iff the assignment satisfies C).  Returns a list of
    (tensor, [index ids]) and the number of indices."""
    occ: Dict[Tuple[int, int], int] = {}
    tensors = []
    for ci, c in enumerate(f.clauses):
        vs = sorted({abs(l) for l in c})
        ids = []
        for v in vs:
            occ[(v, ci)] = len(occ)
            ids.append(occ[(v, ci)])
        shape = (2,) * len(vs)
        t = np.zeros(shape)
        for idx in (np.ndindex(*shape) if vs else [()]):
            val = dict(zip(vs, idx))
            t[idx] = 1.0 if any((l > 0 and val[abs(l)] == 1) or (l < 0 and val[abs(l)] == 0)
                                for l in c) else 0.0
        tensors.append((t, ids))
    for x in range(1, f.n + 1):
        ids = [occ[k] for k in sorted(occ) if k[0] == x]
        d = len(ids)
        if d == 0:
            tensors.append((np.array(f.weights[x - 1, 0] + f.weights[x - 1, 1]), []))
            continue
        t = np.zeros((2,) * d)
        t[(0,) * d] = f.weights[x - 1, 0]
        t[(1,) * d] = f.weights[x - 1, 1]
        tensors.append((t, ids))
    return tensors, len(occ)


def einsum_network(f) -> float:
    """O4: contract the literal Theorem-2 network with numpy.einsum."""
    tensors, n_idx = theorem2_network(f)
    if n_idx > 52:
        raise OracleError("einsum_network supports at most 52 indices")
    args = []
    for t, ids in tensors:
        args.append(t)
        args.append(list(ids))
    args.append([])
    return float(np.einsum(*args, optimize="greedy"))
