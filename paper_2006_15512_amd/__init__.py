"""Python binding of libwmc (the MI355X tensor-network weighted model counter).

Argument marshalling only: every step of the reduction, planning and
contraction runs in the C/HIP library.  PyTorch is used for device memory
(the caller-owned workspace) and streams.  The functions keep the C-ABI
names: ``wmc_build_network``, ``wmc_plan``, ``wmc_contract``; ``Network``,
``Plan`` and ``contract`` are convenience wrappers around them.

If the library has not been built the import still succeeds (so the build
step can run), but every call raises :class:`WmcLibraryMissing`: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, NamedTuple, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WMC_LIBRARY names another build of the same library (the sanitizer build
# of the host code: python -m paper_2006_15512_amd.build --sanitize)
LIB_PATH = os.environ.get("WMC_LIBRARY") or os.path.join(_HERE, "libwmc.so")

WMC_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "OUT_OF_MEMORY", 3: "CAP_UNREACHABLE",
                4: "DEVICE", 5: "BUSY", 6: "UNSUPPORTED", 7: "CANCELLED"}
CANCELLED = 7
FP64, FP32_SCALED = 0, 1
TREE_MINFILL, TREE_ORDER, TREE_EXPLICIT, TREE_NETWORK = 0, 1, 2, 3
SLICE_BY_MEMORY, SLICE_BY_FLOPS = 0, 1
_PREC = {"fp64": 0, "fp32": 1, "fp32_scaled": 1}
MAX_RANK = 34
MAX_SLICED = 40
N_CLASSES = 4
CLASS_NAMES = ["small", "stream", "gemm", "other"]


class WmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class WmcLibraryMissing(RuntimeError):
    pass


class wmc_value(ctypes.Structure):
    _fields_ = [("mantissa", ctypes.c_double), ("exp2", ctypes.c_int64),
                ("value", ctypes.c_double), ("log2_abs", ctypes.c_double)]


class wmc_plan_options(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("order", ctypes.POINTER(ctypes.c_int32)), ("order_len", ctypes.c_int32),
                ("block", ctypes.c_int32), ("parent", ctypes.POINTER(ctypes.c_int64)),
                ("n_tree_nodes", ctypes.c_int64), ("mem_cap_bytes", ctypes.c_uint64),
                ("rank_cap", ctypes.c_int32), ("slice_objective", ctypes.c_int32), ("slice_group", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class wmc_tuning(ctypes.Structure):
    _fields_ = [("stream2_grid_cap", ctypes.c_int32), ("stream_mfma_grid_cap", ctypes.c_int32),
                ("stream_mfma_min_bits", ctypes.c_int32), ("stream2_tile_bits", ctypes.c_int32),
                ("stream2_min_thread_bits", ctypes.c_int32), ("stream2_low_bits", ctypes.c_int32),
                ("split_lanes", ctypes.c_int32), ("multi_min_rank", ctypes.c_int32),
                ("gemm_tpw_max_nt", ctypes.c_int32), ("gemm_orient", ctypes.c_int32),
                ("stream2_vec", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


TUNING_FIELDS = [name for name, _ in wmc_tuning._fields_ if name != "reserved"]


def tuning_get(precision: str = "fp64") -> Dict[str, int]:
    """The executor tuning table that plans of this precision made now copy."""
    t = wmc_tuning()
    _check(lib().wmc_tuning_get(_PREC[precision], ctypes.byref(t)))
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


def tuning_set(precision: str = "fp64", table: Optional[Dict[str, int]] = None) -> None:
    """Replace the table for plans made afterwards (None: built-in defaults);
    missing keys keep their current values."""
    if table is None:
        _check(lib().wmc_tuning_set(_PREC[precision], None))
        return
    cur = tuning_get(precision)
    cur.update({k: int(v) for k, v in table.items() if k in TUNING_FIELDS})
    t = wmc_tuning()
    for k, v in cur.items():
        setattr(t, k, v)
    _check(lib().wmc_tuning_set(_PREC[precision], ctypes.byref(t)))


class wmc_slice_state(ctypes.Structure):
    _fields_ = [("s", ctypes.c_double), ("c", ctypes.c_double), ("e", ctypes.c_int64),
                ("next_slice", ctypes.c_int64), ("n_slices", ctypes.c_int64), ("reserved", ctypes.c_int64)]


class wmc_plan_info(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_clauses", ctypes.c_int64),
                ("n_tensors", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("max_rank", ctypes.c_int32),
                ("max_rank_unsliced", ctypes.c_int32), ("max_index_rank", ctypes.c_int32),
                ("n_sliced", ctypes.c_int32), ("n_slices", ctypes.c_int64),
                ("sliced_vars", ctypes.c_int32 * MAX_SLICED), ("flops_per_slice", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("peak_live_bytes", ctypes.c_double),
                ("arena_bytes", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("class_hist", ctypes.c_int64 * N_CLASSES), ("n_launches", ctypes.c_int64),
                ("max_node_bytes", ctypes.c_double), ("n_aux_vars", ctypes.c_int32), ("slice_group", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libwmc.so (raises WmcLibraryMissing if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise WmcLibraryMissing(f"{LIB_PATH} not built: run `python -m paper_2006_15512_amd.build`")
        # torch ships its own HIP runtime under the same soname.  Loading torch
        # first makes libwmc.so bind to that runtime, so device buffers and
        # streams created by torch are valid in library calls; loading the
        # library first would put a second HIP runtime in the process.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sigs = {
            "wmc_build_network": [i32, i64, P, P, P, P],
            "wmc_network_info": [P, P, P],
            "wmc_plan": [P, ctypes.POINTER(wmc_plan_options), P],
            "wmc_plan_stats": [P, ctypes.POINTER(wmc_plan_info)],
            "wmc_order_from_td": [P, ctypes.c_char_p, i64, P, P],
            "wmc_plan_tensor": [P, i64, P, P, P, P],
            "wmc_plan_node": [P, i64, P, P, P, P],
            "wmc_plan_image": [P, P, u64, P, P],
            "wmc_contract": [P, P, P, u64, P, ctypes.POINTER(wmc_value)],
            "wmc_contract_slices": [P, P, P, u64, P, i64, i64, ctypes.POINTER(wmc_value), P],
            "wmc_contract_resume": [P, P, P, u64, P, i64, ctypes.POINTER(wmc_slice_state), ctypes.POINTER(wmc_value)],
            "wmc_plan_launches": [P, P, P, P, i64, P],
            "wmc_batch_create": [P, i64, P],
            "wmc_batch_info": [P, P, P, P],
            "wmc_batch_contract": [P, P, P, u64, P, ctypes.c_uint32, P],
            "wmc_batch_image": [P, P, u64, P, P],
            "wmc_serve_create": [P, P, u64, P, P],
            "wmc_serve_register": [P, P, P],
            "wmc_serve_submit": [P, i32, P, u64],
            "wmc_serve_step": [P, P, P],
            "wmc_serve_poll": [P, P, i32, P],
            "wmc_serve_wait": [P, P, i32, P, i64],
            "wmc_serve_cancel": [P, u64],
            "wmc_serve_submit_deadline": [P, i32, P, u64, ctypes.c_double],
            "wmc_serve": [P, P, i64, P],
            "wmc_serve_stats": [P, P],
            "wmc_contract_profile": [P, P, P, u64, P, P, i64, ctypes.POINTER(wmc_value)],
            "wmc_plan_kernels": [P, P, i64, P],
            "wmc_contract_noalloc": [P, P, P, ctypes.POINTER(wmc_value)],
            "wmc_build_network_td": [i32, i64, P, P, P, ctypes.c_char_p, i64, P, P],
            "wmc_tuning_get": [i32, P],
            "wmc_tuning_set": [i32, P],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name in ("wmc_network_destroy", "wmc_plan_destroy", "wmc_batch_destroy", "wmc_serve_destroy"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = None
        L.wmc_last_error.restype = ctypes.c_char_p
        L.wmc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != WMC_OK:
        raise WmcError(st, lib().wmc_last_error().decode())


def _p(a: Optional[np.ndarray]):
    return None if a is None or a.size == 0 else a.ctypes.data_as(ctypes.c_void_p)


class Value(NamedTuple):
    mantissa: float
    exp2: int
    value: float
    log2_abs: float

    @staticmethod
    def of(v: wmc_value) -> "Value":
        return Value(v.mantissa, int(v.exp2), v.value, v.log2_abs)


# ---------------------------------------------------------------------------
# reduction
# ---------------------------------------------------------------------------
class Network:
    """wmc_build_network over a CNF (list of DIMACS clauses) and weights (n, 2)."""

    def __init__(self, n: int, clauses: Sequence[Sequence[int]], weights):
        ptr = np.zeros(len(clauses) + 1, dtype=np.int64)
        for i, c in enumerate(clauses):
            ptr[i + 1] = ptr[i] + len(c)
        lits = np.array([l for c in clauses for l in c], dtype=np.int32)
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if w.size != 2 * n:
            raise ValueError("weights must have 2*n entries")
        h = ctypes.c_void_p()
        _check(lib().wmc_build_network(int(n), len(clauses), _p(ptr) if len(clauses) else None,
                                       _p(lits), _p(w), ctypes.byref(h)))
        self._h = h
        self.n = int(n)
        self.m = len(clauses)
        # kept for checkpoint identities (the library holds its own copies)
        self.clauses = [list(map(int, c)) for c in clauses]
        self.weights = w.copy()

    @classmethod
    def from_formula(cls, f) -> "Network":
        return cls(f.n, f.clauses, f.weights)

    @classmethod
    def from_td(cls, f, td: str, root_bag: int = 0) -> "Network":
        """wmc_build_network_td (FactorTree): the network factored along a
        tree decomposition ``td`` (PACE text) of the formula's incidence graph
        (variables 1..n, clause c as vertex n + 1 + c); plan it with
        kind="network".  The decomposition's width is in ``.td_width``."""
        self = cls.__new__(cls)
        clauses = f.clauses
        ptr = np.zeros(len(clauses) + 1, dtype=np.int64)
        for i, c in enumerate(clauses):
            ptr[i + 1] = ptr[i] + len(c)
        lits = np.array([l for c in clauses for l in c], dtype=np.int32)
        w = np.ascontiguousarray(np.asarray(f.weights, dtype=np.float64).reshape(-1))
        if w.size != 2 * f.n:
            raise ValueError("weights must have 2*n entries")
        h = ctypes.c_void_p()
        wd = ctypes.c_int32()
        _check(lib().wmc_build_network_td(int(f.n), len(clauses), _p(ptr) if len(clauses) else None, _p(lits), _p(w),
                                          td.encode(), int(root_bag), ctypes.byref(h), ctypes.byref(wd)))
        self._h = h
        self.n = int(f.n)
        self.m = len(clauses)
        self.clauses = [list(map(int, c)) for c in clauses]
        self.weights = w.copy()
        self.td_width = int(wd.value)
        return self

    def info(self) -> Dict[str, int]:
        nt, ni = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wmc_network_info(self._h, ctypes.byref(nt), ctypes.byref(ni)))
        return {"n_tensors": nt.value, "n_indices": ni.value}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wmc_network_destroy(h)
            self._h = None


def wmc_build_network(n, clauses, weights) -> Network:
    return Network(n, clauses, weights)


def order_from_td(net: Network, td: str, root_bag: int = 0):
    """wmc_order_from_td: (elimination order over 1..n, width) from a tree
    decomposition of the primal graph given as PACE .td text; pass the order
    to Plan(net, kind="order", order=...)."""
    order = np.zeros(max(net.n, 1), dtype=np.int32)
    width = ctypes.c_int32()
    _check(lib().wmc_order_from_td(net._h, td.encode(), int(root_bag), _p(order), ctypes.byref(width)))
    return order[: net.n], width.value


# ---------------------------------------------------------------------------
# planning
# ---------------------------------------------------------------------------
_TUNING_LOADED = False


def _auto_tuning() -> None:
    """Once per process, before the first plan: install the executor tuning
    measured for this device, if one is stored (``autotune.load_tuning``);
    WMC_NO_TUNING=1 keeps the built-in defaults."""
    global _TUNING_LOADED
    if _TUNING_LOADED:
        return
    _TUNING_LOADED = True
    if os.environ.get("WMC_NO_TUNING"):
        return
    from .autotune import load_tuning
    load_tuning()


class Plan:
    """wmc_plan: contraction tree + slicing + layouts for one network."""

    def __init__(self, net: Network, kind: str = "minfill", seed: int = 0,
                 order: Optional[Sequence[int]] = None, parent: Optional[Sequence[int]] = None,
                 mem_cap_bytes: int = 0, rank_cap: int = 0, precision: str = "fp64", block: int = 1,
                 slice_objective: str = "memory", slice_group: int = 1):
        o = wmc_plan_options()
        o.kind = {"minfill": TREE_MINFILL, "order": TREE_ORDER, "explicit": TREE_EXPLICIT,
                  "network": TREE_NETWORK}[kind]
        o.precision = {"fp64": FP64, "fp32": FP32_SCALED, "fp32_scaled": FP32_SCALED}[precision]
        o.seed = int(seed)
        o.block = int(block)
        self._order = self._parent = None
        if order is not None:
            self._order = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
            o.order = self._order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            o.order_len = int(self._order.size)
        if parent is not None:
            self._parent = np.ascontiguousarray(np.asarray(parent, dtype=np.int64))
            o.parent = self._parent.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            o.n_tree_nodes = int(self._parent.size)
        o.mem_cap_bytes = int(mem_cap_bytes)
        o.rank_cap = int(rank_cap)
        _auto_tuning()
        o.slice_group = int(slice_group)
        o.slice_objective = {"memory": SLICE_BY_MEMORY, "flops": SLICE_BY_FLOPS}[slice_objective]
        h = ctypes.c_void_p()
        _check(lib().wmc_plan(net._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.net = net
        self.precision = precision
        self._info = wmc_plan_info()
        _check(lib().wmc_plan_stats(self._h, ctypes.byref(self._info)))

    def stats(self) -> Dict:
        i = self._info
        d = {name: getattr(i, name) for name, _ in wmc_plan_info._fields_}
        d["sliced_vars"] = list(i.sliced_vars)[: i.n_sliced]
        d["class_hist"] = {CLASS_NAMES[k]: int(i.class_hist[k]) for k in range(N_CLASSES)}
        return d

    @property
    def workspace_bytes(self) -> int:
        return int(self._info.workspace_bytes)

    @property
    def n_slices(self) -> int:
        return int(self._info.n_slices)

    def tensor(self, t: int):
        kind, src, rank = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        vars_ = (ctypes.c_int32 * (MAX_RANK + 1))()
        _check(lib().wmc_plan_tensor(self._h, int(t), ctypes.byref(kind), ctypes.byref(src),
                                     ctypes.byref(rank), vars_))
        return kind.value, src.value, list(vars_)[: rank.value]

    def node(self, i: int):
        a, b, c, cls = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().wmc_plan_node(self._h, int(i), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                   ctypes.byref(cls)))
        return a.value, b.value, c.value, cls.value

    def export(self):
        """(tensors, nodes, sliced_vars): tensors[t] = (kind, src, layout),
        nodes[i] = (a, b, c, class) in launch order."""
        s = self.stats()
        tensors = [self.tensor(t) for t in range(s["n_tensors"])]
        nodes = [self.node(i) for i in range(s["n_nodes"])]
        return tensors, nodes, s["sliced_vars"]

    def image(self):
        """Raw descriptor image: (bytes, info dict) as uploaded to the device."""
        need = ctypes.c_uint64()
        info = (ctypes.c_int64 * 13)()
        _check(lib().wmc_plan_image(self._h, None, 0, ctypes.byref(need), info))
        buf = (ctypes.c_uint8 * max(int(need.value), 1))()
        _check(lib().wmc_plan_image(self._h, buf, int(need.value), ctypes.byref(need), info))
        keys = ["n_leaves", "n_nodes", "n_launches", "arena_elems", "root", "root_off", "n_tensors",
                "elem", "leaf_desc_bytes", "node_desc_bytes", "launch_bytes", "n_gemms", "gemm_desc_bytes"]
        return bytes(buf)[: int(need.value)], dict(zip(keys, list(info)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wmc_plan_destroy(h)
            self._h = None


def wmc_plan(net: Network, **kw) -> Plan:
    return Plan(net, **kw)


# ---------------------------------------------------------------------------
# execution
# ---------------------------------------------------------------------------
def workspace(plan: Plan, device: str = "cuda:0"):
    """A caller-owned device workspace for ``plan`` (a torch uint8 tensor)."""
    import torch
    n = max(plan.workspace_bytes, 256)
    return torch.empty(n, dtype=torch.uint8, device=device)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def wmc_contract(plan: Plan, weights=None, ws=None, stream=None) -> Value:
    """Contract ``plan`` on the GPU; ``ws`` is a device tensor of at least
    plan.workspace_bytes (allocated here if omitted)."""
    if ws is None:
        ws = workspace(plan)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if w.size != 2 * plan.net.n:
            raise ValueError("weights must have 2*n entries")
    out = wmc_value()
    _check(lib().wmc_contract(plan._h, _p(w), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                              _stream_ptr(stream), ctypes.byref(out)))
    return Value.of(out)


NOALLOC_SCRATCH_BYTES = 64 << 20


def wmc_contract_noalloc(plan: Plan, weights=None, stream=None) -> Value:
    """wmc_contract on the library's static device scratch (no device
    allocation; plans up to NOALLOC_SCRATCH_BYTES of workspace)."""
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if w.size != 2 * plan.net.n:
            raise ValueError("weights must have 2*n entries")
    out = wmc_value()
    _check(lib().wmc_contract_noalloc(plan._h, _p(w), _stream_ptr(stream), ctypes.byref(out)))
    return Value.of(out)


def wmc_contract_slices(plan: Plan, begin: int, end: int, weights=None, ws=None, stream=None,
                        per_slice: bool = False):
    """Sum of slices [begin, end); with per_slice=True also each slice's value."""
    if ws is None:
        ws = workspace(plan)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    out = wmc_value()
    arr = (wmc_value * max(end - begin, 1))() if per_slice else None
    _check(lib().wmc_contract_slices(plan._h, _p(w), ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel() * ws.element_size(), _stream_ptr(stream), int(begin), int(end),
                                     ctypes.byref(out), arr))
    if per_slice:
        return Value.of(out), [Value.of(arr[i]) for i in range(end - begin)]
    return Value.of(out)


contract = wmc_contract


def wmc_contract_resume(plan: Plan, state: wmc_slice_state, count: int, weights=None, ws=None, stream=None) -> Value:
    """Run the next ``count`` slices after ``state.next_slice``, continuing
    the running sum in ``state`` (updated in place); returns the sum so far."""
    if ws is None:
        ws = workspace(plan)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    out = wmc_value()
    _check(lib().wmc_contract_resume(plan._h, _p(w), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                     _stream_ptr(stream), int(count), ctypes.byref(state), ctypes.byref(out)))
    return Value.of(out)


def checkpoint_identity(plan: Plan, weights=None) -> Dict:
    """What a checkpointed slice loop's running sum depends on: the plan's
    slices and precision, the formula's clauses and the weights used."""
    import hashlib
    st = plan.stats()
    h = hashlib.sha256()
    for c in plan.net.clauses:
        h.update(np.asarray(c, dtype=np.int32).tobytes() + b";")
    wsrc = plan.net.weights if weights is None else weights
    wd = hashlib.sha256(np.ascontiguousarray(np.asarray(wsrc, dtype=np.float64).reshape(-1)).tobytes()).hexdigest()
    return {"n_slices": int(st["n_slices"]), "sliced_vars": [int(x) for x in st["sliced_vars"]],
            "n_vars": int(st["n_vars"]), "n_clauses": int(st["n_clauses"]), "precision": plan.precision,
            "clauses_sha256": h.hexdigest(), "weights_sha256": wd}


def contract_checkpointed(plan: Plan, path: str, chunk: int = 1, weights=None, ws=None, stream=None,
                          stop_after: Optional[int] = None) -> Optional[Value]:
    """The slice loop in chunks of ``chunk`` slices with its running sum saved
    to ``path`` (JSON, written atomically) after every chunk; an existing file
    resumes the loop where it stopped.  ``stop_after`` ends the call after
    that many chunks (returns None if slices remain).  The file records what
    the running sum depends on (slice count, sliced variables, precision, a
    digest of the clauses and of the weights actually used) and is refused
    for any other plan, formula or weight vector."""
    import json
    ident = checkpoint_identity(plan, weights)
    state = wmc_slice_state()
    if os.path.exists(path):
        with open(path) as fh:
            saved = json.load(fh)
        if saved["plan"] != ident:
            raise ValueError(f"{path} holds a checkpoint of another plan")
        state.s, state.c = float.fromhex(saved["s"]), float.fromhex(saved["c"])
        state.e, state.next_slice, state.n_slices = int(saved["e"]), int(saved["next_slice"]), int(saved["n_slices"])
    done = 0
    v = None
    while True:
        v = wmc_contract_resume(plan, state, chunk, weights, ws, stream)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({"plan": ident, "s": state.s.hex(), "c": state.c.hex(), "e": int(state.e),
                       "next_slice": int(state.next_slice), "n_slices": int(state.n_slices)}, fh)
        os.replace(tmp, path)
        done += 1
        if state.next_slice >= state.n_slices:
            return v
        if stop_after is not None and done >= stop_after:
            return None


def plan_launches(plan: Plan):
    """Per-launch algorithmic (bytes, flops, class) of one slice, in issue order."""
    n = ctypes.c_int64()
    _check(lib().wmc_plan_launches(plan._h, None, None, None, 0, ctypes.byref(n)))
    k = int(n.value)
    b = np.zeros(k)
    f = np.zeros(k)
    c = np.zeros(k, dtype=np.int32)
    _check(lib().wmc_plan_launches(plan._h, _p(b), _p(f), _p(c), k, ctypes.byref(n)))
    return b, f, c


KERNEL_NAMES = ["k_begin", "k_leaves", "k_nodes", "k_gemm_p", "k_gemm", "k_stream_mfma", "k_stream2",
                "k_stream2_split", "k_finish", "k_stream2_vec"]


def plan_kernels(plan: Plan) -> np.ndarray:
    """Kernel family (index into KERNEL_NAMES) of each launch of one slice,
    in the order of plan_launches."""
    n = ctypes.c_int64()
    _check(lib().wmc_plan_kernels(plan._h, None, 0, ctypes.byref(n)))
    k = np.zeros(int(n.value), dtype=np.int32)
    _check(lib().wmc_plan_kernels(plan._h, _p(k), int(n.value), ctypes.byref(n)))
    return k


def wmc_contract_profile(plan: Plan, weights=None, ws=None, stream=None):
    """wmc_contract with HIP events between launches: (value, ms per launch)."""
    if ws is None:
        ws = workspace(plan)
    b, _, _ = plan_launches(plan)
    ms = np.zeros(len(b), dtype=np.float32)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    out = wmc_value()
    _check(lib().wmc_contract_profile(plan._h, _p(w), ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel() * ws.element_size(), _stream_ptr(stream), _p(ms), len(ms),
                                      ctypes.byref(out)))
    return Value.of(out), ms


def version() -> str:
    return lib().wmc_version().decode()


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------
BATCH_RESIDENT = 1  # descriptors already in this workspace from an earlier call
BATCH_GRAPH = 2  # capture the launches once per workspace and replay the HIP graph
BATCH_PERSISTENT = 4  # every merged step in one cooperative launch (exact; slower on small formulas)


class Batch:
    """wmc_batch_create over a list of plans of one precision (sliced plans
    enter as one instance per slice)."""

    def __init__(self, plans: Sequence[Plan]):
        arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
        h = ctypes.c_void_p()
        _check(lib().wmc_batch_create(arr, len(plans), ctypes.byref(h)))
        self._h = h
        self.plans = list(plans)
        wsb, nl, ni = ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wmc_batch_info(self._h, ctypes.byref(wsb), ctypes.byref(nl), ctypes.byref(ni)))
        self.workspace_bytes = int(wsb.value)
        self.n_launches = int(nl.value)
        self.n = int(ni.value)

    def workspace(self, device: str = "cuda:0"):
        import torch
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)

    def image(self):
        """Raw descriptor image: (bytes, info dict)."""
        need = ctypes.c_uint64()
        info = (ctypes.c_int64 * 10)()
        _check(lib().wmc_batch_image(self._h, None, 0, ctypes.byref(need), info))
        buf = (ctypes.c_uint8 * max(int(need.value), 1))()
        _check(lib().wmc_batch_image(self._h, buf, int(need.value), ctypes.byref(need), info))
        keys = ["n_leaves", "n_nodes", "n_launches", "arena_elems", "n_instances", "meta_total", "elem",
                "n_gemms", "n_vars_total", "n_tasks"]
        return bytes(buf)[: int(need.value)], dict(zip(keys, list(info)))

    def contract(self, weights=None, ws=None, stream=None, flags: int = 0) -> List[Value]:
        if ws is None:
            ws = self.workspace()
        w = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        out = (wmc_value * self.n)()
        _check(lib().wmc_batch_contract(self._h, _p(w), ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel() * ws.element_size(), _stream_ptr(stream), int(flags), out))
        return [Value.of(out[i]) for i in range(self.n)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wmc_batch_destroy(h)
            self._h = None


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class wmc_serve_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64), ("step_bytes", ctypes.c_uint64)]


class wmc_response(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("structure", ctypes.c_int32), ("status", ctypes.c_int32),
                ("value", wmc_value), ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class wmc_request(ctypes.Structure):
    _fields_ = [("t_arrive", ctypes.c_double), ("structure", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("request_id", ctypes.c_uint64), ("weights", ctypes.c_void_p)]


class wmc_serve_info(ctypes.Structure):
    _fields_ = [("region_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64),
                ("peak_used_bytes", ctypes.c_uint64), ("peak_active", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("n_active", ctypes.c_int64), ("n_queued", ctypes.c_int64), ("n_structures", ctypes.c_int64)]


class Response(NamedTuple):
    request_id: int
    structure: int
    status: int
    value: Value
    t_arrive: float
    t_admit: float
    t_done: float

    @staticmethod
    def of(r: wmc_response) -> "Response":
        return Response(int(r.request_id), int(r.structure), int(r.status), Value.of(r.value), r.t_arrive,
                        r.t_admit, r.t_done)


class Server:
    """wmc_serve_create over a caller-owned device buffer (a torch tensor)."""

    def __init__(self, precision: str = "fp64", max_slots: int = 64, max_queue: int = 1 << 20,
                 hbm_budget_bytes: int = 0, buffer_bytes: int = 1 << 30, step_bytes: int = 0,
                 device: str = "cuda:0", stream=None):
        import torch
        o = wmc_serve_options()
        o.precision = {"fp64": FP64, "fp32": FP32_SCALED, "fp32_scaled": FP32_SCALED}[precision]
        o.max_slots = int(max_slots)
        o.max_queue = int(max_queue)
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.step_bytes = int(step_bytes)
        self.buf = torch.empty(int(buffer_bytes), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().wmc_serve_create(ctypes.byref(o), ctypes.c_void_p(self.buf.data_ptr()), int(buffer_bytes),
                                      _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.plans = []

    def register(self, plan: Plan) -> int:
        sid = ctypes.c_int32()
        _check(lib().wmc_serve_register(self._h, plan._h, ctypes.byref(sid)))
        self.plans.append(plan)
        return int(sid.value)

    def submit(self, structure: int, weights, request_id: int) -> None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        _check(lib().wmc_serve_submit(self._h, int(structure), _p(w), int(request_id)))

    def submit_deadline(self, structure: int, weights, request_id: int, timeout_s: float) -> None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        _check(lib().wmc_serve_submit_deadline(self._h, int(structure), _p(w), int(request_id), float(timeout_s)))

    def cancel(self, request_id: int) -> None:
        _check(lib().wmc_serve_cancel(self._h, int(request_id)))

    def wait(self, timeout_s: float, max_n: int = 1 << 16) -> List[Response]:
        arr = (wmc_response * max_n)()
        n = ctypes.c_int32()
        _check(lib().wmc_serve_wait(self._h, arr, int(max_n), ctypes.byref(n), int(timeout_s * 1e6)))
        return [Response.of(arr[i]) for i in range(n.value)]

    def step(self):
        na, nq = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().wmc_serve_step(self._h, ctypes.byref(na), ctypes.byref(nq)))
        return int(na.value), int(nq.value)

    def poll(self, max_n: int = 1 << 16) -> List[Response]:
        arr = (wmc_response * max_n)()
        n = ctypes.c_int32()
        _check(lib().wmc_serve_poll(self._h, arr, int(max_n), ctypes.byref(n)))
        return [Response.of(arr[i]) for i in range(n.value)]

    def drain(self) -> List[Response]:
        out = []
        while True:
            na, nq = self.step()
            out += self.poll()
            if na == 0 and nq == 0:
                return out

    def run(self, arrivals, structures, weights, ids=None) -> List[Response]:
        """Replay timed arrivals (wmc_serve): arrivals sorted (seconds),
        structures (ints), weights (list of arrays)."""
        n = len(arrivals)
        ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1)) for w in weights]
        reqs = (wmc_request * max(n, 1))()
        for i in range(n):
            reqs[i].t_arrive = float(arrivals[i])
            reqs[i].structure = int(structures[i])
            reqs[i].request_id = int(ids[i]) if ids is not None else i
            reqs[i].weights = ws[i].ctypes.data_as(ctypes.c_void_p)
        out = (wmc_response * max(n, 1))()
        _check(lib().wmc_serve(self._h, reqs, n, out))
        return [Response.of(out[i]) for i in range(n)]

    def stats(self) -> Dict:
        i = wmc_serve_info()
        _check(lib().wmc_serve_stats(self._h, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in wmc_serve_info._fields_}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.wmc_serve_destroy(h)
            self._h = None
