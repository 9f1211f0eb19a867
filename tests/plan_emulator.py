"""Replays a plan's raw device descriptors on the CPU with numpy.

Test infrastructure for the host planner: it interprets the leaf and node
descriptors, launch list and arena offsets exactly as the HIP kernels do
(run-list bit extraction, kappa-lowest operand layouts, shared arena,
power-of-two operand scaling), so a wrong layout, run list, slice bit or
arena overlap shows up on a machine without a GPU.  It is not the oracle:
it mirrors the GPU path and is itself checked against the oracle.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

LEAF = np.dtype([("out", "<i8"), ("work_begin", "<i8"), ("tensor", "<i4"), ("kind", "<i4"),
                 ("rank", "<i4"), ("k", "<i4"), ("var", "<i4"), ("falsify", "<u4"), ("taut", "<i4"),
                 ("pad", "<i4"), ("pos", "<i2", (24,))])
NODE = np.dtype({"names": ["a", "b", "c", "work_begin", "ta", "tb", "tc", "rc", "nk", "nra", "nrb", "cls",
                           "ra", "rb"],
                 "formats": ["<i8", "<i8", "<i8", "<i8", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4",
                             ("<u4", (20,)), ("<u4", (20,))],
                 "offsets": [0, 8, 16, 24, 32, 36, 40, 44, 48, 52, 56, 60, 64, 144],
                 "itemsize": 224})
LAUNCH = np.dtype([("type", "<i4"), ("first", "<i4"), ("count", "<i4"), ("pad", "<i4"), ("work", "<i8")])
GEMM = np.dtype({"names": ["a", "b", "c", "ta", "tb", "tc", "nk", "nm", "nn", "nb", "nrun", "run"],
                 "formats": ["<i8", "<i8", "<i8", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4", ("<i4", (7,)),
                             ("u1", (7, 12, 3))],
                 "offsets": [0, 8, 16, 24, 28, 32, 36, 40, 44, 48, 52, 80],
                 "itemsize": 336})
GR_MU_A, GR_BETA_A, GR_NU_B, GR_BETA_B, GR_MU_C, GR_NU_C, GR_BETA_C = range(7)
STREAM = np.dtype({"names": ["s", "o", "c", "ts", "to", "tc", "rc", "np", "nq", "pbit", "qbit", "nlrun", "nsrun",
                             "norun", "lrun", "srun", "orun", "ro", "o_lds", "block_begin"],
                   "formats": ["<i8", "<i8", "<i8", "<i4", "<i4", "<i4", "<i4", "<i4", "<i4", ("<i4", (2,)),
                               ("<i4", (2,)), "<i4", "<i4", "<i4", ("<u4", (16,)), ("<u4", (16,)), ("<u4", (16,)),
                               "<i4", "<i4", "<i8"],
                   "offsets": [0, 8, 16, 24, 28, 32, 36, 40, 44, 48, 56, 64, 68, 72, 76, 140, 204, 268, 272, 280],
                   "itemsize": 288})


def parse(plan):
    img, info = plan.image()
    assert info["leaf_desc_bytes"] == LEAF.itemsize
    assert info["node_desc_bytes"] == NODE.itemsize
    assert info["launch_bytes"] == LAUNCH.itemsize
    assert info["gemm_desc_bytes"] == GEMM.itemsize
    nl, nn, nla, ng = info["n_leaves"], info["n_nodes"], info["n_launches"], info["n_gemms"]
    leaves = np.frombuffer(img, LEAF, count=nl, offset=0)
    nodes = np.frombuffer(img, NODE, count=nn, offset=nl * LEAF.itemsize)
    off = nl * LEAF.itemsize + nn * NODE.itemsize
    launches = np.frombuffer(img, LAUNCH, count=nla, offset=off)
    gemms = np.frombuffer(img, GEMM, count=ng, offset=off + nla * LAUNCH.itemsize)
    return leaves, nodes, launches, gemms, info


def _pext(r: np.ndarray, runs, nr: int) -> np.ndarray:
    """Bit extraction along runs given as (src, len, dst) triples or packed
    words src | len << 8 | dst << 16."""
    out = np.zeros_like(r)
    for q in range(nr):
        run = runs[q]
        if np.ndim(run) == 0:
            w = int(run)
            s, l, d = w & 255, (w >> 8) & 255, w >> 16
        else:
            s, l, d = (int(x) for x in run)
        out |= ((r >> np.uint64(s)) & np.uint64((1 << l) - 1)) << np.uint64(d)
    return out


def _sexp(m: float) -> int:
    if not m > 0.0:
        return 0
    return math.frexp(m)[1]


def _stream_task_as_node(t, nk):
    """A streaming task (S, O and their C-bit run lists) rewritten as
    (a, b, c, ta, tb, tc, rc, nk, A-runs, B-runs) so the generic replay below
    can execute it (the product is symmetric in its operands)."""
    return dict(a=int(t["s"]), b=int(t["o"]), c=int(t["c"]), ta=int(t["ts"]), tb=int(t["to"]), tc=int(t["tc"]),
                rc=int(t["rc"]), nk=nk, ra=np.array(t["srun"][: int(t["nsrun"])], dtype=np.uint32),
                nra=int(t["nsrun"]), rb=np.array(t["orun"][: int(t["norun"])], dtype=np.uint32), nrb=int(t["norun"]))


def _replay(leaves, nodes, launches, gemms, arena_elems, nt, w, store, eta, roots, root_offs, tasks_of=None):
    """One pass of the launch list; returns the exact value of each root."""
    arena = np.zeros(max(arena_elems, 1), dtype=store)
    maxv = np.zeros(max(nt, 1))
    ex = np.zeros(max(nt, 1), dtype=np.int64)
    for d in leaves:
        size = 1 << int(d["rank"])
        e = np.arange(size, dtype=np.int64)
        if d["kind"] == 0:
            a = np.zeros(size, dtype=np.int64)
            for q in range(int(d["k"])):
                p = int(d["pos"][q])
                bit = (e >> p) & 1 if p >= 0 else np.full(size, (eta >> (-p - 1)) & 1)
                a |= bit << q
            v = np.where((a != int(d["falsify"])) | bool(d["taut"]), 1.0, 0.0)
        elif d["kind"] == 1:
            p = int(d["pos"][0])
            bit = (e >> p) & 1 if p >= 0 else np.full(size, (eta >> (-p - 1)) & 1)
            v = w[2 * int(d["var"]) + bit]
        else:
            v = np.array([w[2 * int(d["var"])] + w[2 * int(d["var"]) + 1]])
        s = v.astype(store)
        arena[int(d["out"]): int(d["out"]) + size] = s
        maxv[int(d["tensor"])] = float(np.max(np.abs(s.astype(np.float64))))
    for li in range(1, len(launches)):
        L = launches[li]
        results = []
        if int(L["type"]) == 2:
            g = gemms[int(L["pad"])]
            nk, nm, nn, nb = (int(g[k]) for k in ("nk", "nm", "nn", "nb"))
            runs = lambda q: (g["run"][q], int(g["nrun"][q]))
            mu = np.arange(1 << nm, dtype=np.uint64)
            nu = np.arange(1 << nn, dtype=np.uint64)
            sA, sB = _sexp(maxv[int(g["ta"])]), _sexp(maxv[int(g["tb"])])
            outs = []
            for beta in range(1 << nb):
                bt = np.array([beta], dtype=np.uint64)
                # A is stored [4 lowest mu bits | kappa | rest]
                rows = (mu & np.uint64(15)) | \
                    ((_pext(mu >> np.uint64(4), *runs(GR_MU_A)) | _pext(bt, *runs(GR_BETA_A))) << np.uint64(4 + nk))
                cols = (_pext(nu, *runs(GR_NU_B)) | _pext(bt, *runs(GR_BETA_B))) << np.uint64(nk)
                kk = np.arange(1 << nk, dtype=np.uint64)
                Am = arena[int(g["a"]) + (rows[:, None] + (kk[None, :] << np.uint64(4))).astype(np.int64)].astype(np.float64)
                Bm = arena[int(g["b"]) + (cols[:, None] + kk[None, :]).astype(np.int64)].astype(np.float64)
                Cm = np.ldexp(Am @ Bm.T, -(sA + sB)).astype(store)
                addr = (_pext(mu, *runs(GR_MU_C))[:, None] | _pext(nu, *runs(GR_NU_C))[None, :] |
                        _pext(bt, *runs(GR_BETA_C)))
                outs.append((addr.astype(np.int64).ravel(), Cm.ravel()))
            mx = 0.0
            for addr, val in outs:
                arena[int(g["c"]) + addr] = val
                mx = max(mx, float(np.max(np.abs(val.astype(np.float64)))))
            maxv[int(g["tc"])] = mx
            ex[int(g["tc"])] = ex[int(g["ta"])] + ex[int(g["tb"])] + sA + sB
            continue
        step = list(nodes[int(L["first"]): int(L["first"]) + int(L["count"])])
        if tasks_of is not None:
            step += tasks_of(li)
        for d in step:
            rc, nk = int(d["rc"]), int(d["nk"])
            r = np.arange(1 << rc, dtype=np.uint64)
            pa = _pext(r, d["ra"], int(d["nra"])) << np.uint64(nk)
            pb = _pext(r, d["rb"], int(d["nrb"])) << np.uint64(nk)
            sA, sB = _sexp(maxv[int(d["ta"])]), _sexp(maxv[int(d["tb"])])
            acc = np.zeros(1 << rc)
            for j in range(1 << nk):
                acc += arena[int(d["a"]) + (pa + np.uint64(j)).astype(np.int64)].astype(np.float64) * \
                       arena[int(d["b"]) + (pb + np.uint64(j)).astype(np.int64)].astype(np.float64)
            out = np.ldexp(acc, -(sA + sB)).astype(store)
            results.append((d, out, int(ex[int(d["ta"])] + ex[int(d["tb"])] + sA + sB)))
        for d, out, e in results:
            arena[int(d["c"]): int(d["c"]) + out.size] = out
            maxv[int(d["tc"])] = float(np.max(np.abs(out.astype(np.float64))))
            ex[int(d["tc"])] = e
    vals = []
    for root, off in zip(roots, root_offs):
        if root < 0:
            vals.append(Fraction(1))
            continue
        v = float(arena[int(off)])
        vals.append(Fraction(v) * (Fraction(2) ** int(ex[int(root)])))
    return vals


def full_weights(plan, weights) -> np.ndarray:
    """The device weight array: the caller's 2*n weights, then (1, 1) for
    each auxiliary variable of a factored long clause."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    return np.concatenate([w, np.ones(2 * plan.stats()["n_aux_vars"])])


def emulate(plan, weights, store=np.float64, slices=None):
    """Contract ``plan`` on the CPU exactly as the kernels would.  Returns the
    exact rational sum over the requested slices (default: all) of the slice
    values as they would be produced, plus the list of per-slice values."""
    leaves, nodes, launches, gemms, info = parse(plan)
    w = full_weights(plan, weights)
    root = info["root"]
    if root < 0:
        return Fraction(1), [Fraction(1)]
    n_slices = 1 << len(plan.stats()["sliced_vars"])
    total = Fraction(0)
    per = []
    for eta in (range(n_slices) if slices is None else slices):
        (val,) = _replay(leaves, nodes, launches, gemms, info["arena_elems"], info["n_tensors"], w, store, eta,
                         [root], [info["root_off"]])
        per.append(val)
        total += val
    return total, per


def emulate_batch(batch, weights, store=np.float64):
    """Replay a batch's merged descriptors; returns one exact value per instance."""
    img, info = batch.image()
    nl, nn, nla, ng, n = info["n_leaves"], info["n_nodes"], info["n_launches"], info["n_gemms"], info["n_instances"]
    off = 0
    leaves = np.frombuffer(img, LEAF, count=nl, offset=off)
    off += nl * LEAF.itemsize
    nodes = np.frombuffer(img, NODE, count=nn, offset=off)
    off += nn * NODE.itemsize
    launches = np.frombuffer(img, LAUNCH, count=nla, offset=off)
    off += nla * LAUNCH.itemsize
    gemms = np.frombuffer(img, GEMM, count=ng, offset=off)
    off += ng * GEMM.itemsize
    roots = np.frombuffer(img, "<i4", count=n, offset=off)
    off += 4 * n
    root_offs = np.frombuffer(img, "<i8", count=n, offset=off)
    off += 8 * n
    nt = info["n_tasks"]
    tasks = np.frombuffer(img, STREAM, count=nt, offset=off)
    off += nt * STREAM.itemsize
    groups = np.frombuffer(img, "<i4", count=6 * nla, offset=off).reshape(nla, 6)

    def tasks_of(k):
        tf = int(groups[k, 0])
        out = []
        for nk in range(4):
            for t in tasks[tf + int(groups[k, 1 + nk]): tf + int(groups[k, 2 + nk])]:
                out.append(_stream_task_as_node(t, nk))
        return out
    wu = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    parts, u = [], 0
    for p in batch.plans:
        k = 2 * p.stats()["n_vars"]
        parts.append(full_weights(p, wu[u:u + k]))
        u += k
    w = np.concatenate(parts) if parts else wu
    return _replay(leaves, nodes, launches, gemms, info["arena_elems"], info["meta_total"], w, store, 0,
                   list(roots), list(root_offs), tasks_of)


def to_float(x: Fraction) -> float:
    if x == 0:
        return 0.0
    try:
        return float(x)
    except OverflowError:
        return math.inf


def rel_err(a: Fraction, b: Fraction) -> float:
    if a == b:
        return 0.0
    d = abs(a - b) / max(abs(a), abs(b))
    return float(d)
