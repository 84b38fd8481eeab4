"""Python binding of libgsw (ctypes).  Argument marshalling only: every step of
the traversal runs in the library's HIP kernels.  PyTorch supplies device
memory and streams when results should stay on the GPU.

The library must have been built (``python -m paper_1708_01159_amd.build``);
loading fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsw.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, ERANGE, EBUSY, ENOTREE, ENOTSYM = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ERANGE", -5: "EBUSY",
                -6: "ENOTREE", -7: "ENOTSYM"}

# kernels (values of GSW_K_* in include/gsw.h)
PUSH_VERTEX, PUSH_WAVE4, PUSH_WAVE8, PUSH_WAVE16, PUSH_WAVE32, PUSH_WAVE64 = 0, 1, 2, 3, 4, 5
PUSH_EDGE, PULL_BITMAP, VERTEX_SCAN, EDGE_SCAN = 6, 7, 8, 9
N_KERNELS = 10
KERNEL_NAMES = ("push_vertex", "push_wave4", "push_wave8", "push_wave16", "push_wave32",
                "push_wave64", "push_edge", "pull_bitmap", "vertex_scan", "edge_scan")
DEFAULT_KERNEL = PUSH_EDGE
N_FEATURES = 12
FEATURE_NAMES = ("n_vertices", "n_edges", "deg_min", "deg_q1", "deg_median", "deg_q3", "deg_max",
                 "deg_std", "frontier", "frontier_frac", "discovered", "discovered_frac")

ASSUME_SYMMETRIC, WITH_ORIGIN, TRUSTED = 0x1, 0x2, 0x4
POLICY_TREE, POLICY_FIXED, POLICY_SCHEDULE = 0, 1, 2


class GswError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class LevelTrace(ctypes.Structure):
    _fields_ = [("source_idx", ctypes.c_int32), ("level", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("n_frontier", ctypes.c_int64), ("discovered", ctypes.c_int64),
                ("n_next", ctypes.c_int64), ("ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


class BfsOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("fixed_kernel", ctypes.c_int32),
                ("schedule", ctypes.c_void_p), ("schedule_len", ctypes.c_int32),
                ("tree", ctypes.c_void_p), ("time_levels", ctypes.c_int32),
                ("canonical_parents", ctypes.c_int32), ("device_ptrs", ctypes.c_int32),
                ("max_workgroups", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class MsbfsOpts(ctypes.Structure):
    _fields_ = [("push_to_pull", ctypes.c_float), ("pull_to_push", ctypes.c_float),
                ("device_ptrs", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


MSBFS_MAX_SOURCES = 1024
MSBFS_LEVEL_CAP = 127

_lib = None


def lib():
    """The loaded libgsw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgsw.so is not built (%s); run python -m paper_1708_01159_amd.build"
                           % LIB_PATH)
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname).  Loading torch first lets libgsw bind to that copy; the other
    # order would load two runtimes, and the second cannot open the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    P = ctypes.POINTER
    sig = {
        "gsw_last_error": (ctypes.c_char_p, []),
        "gsw_kernel_name": (ctypes.c_char_p, [i32]),
        "gsw_abi_version": (i32, []),
        "gsw_bfs_opts_default": (None, [P(BfsOpts)]),
        "gsw_graph_validate": (i32, [i64, i64, vp, vp, P(i32)]),
        "gsw_graph_create_host": (i32, [i64, i64, vp, vp, u32, P(vp)]),
        "gsw_graph_create_device": (i32, [i64, i64, vp, vp, u32, vp, P(vp)]),
        "gsw_graph_destroy": (None, [vp]),
        "gsw_graph_info": (i32, [vp, P(i64), P(i64), vp, P(ctypes.c_size_t)]),
        "gsw_level_features": (i32, [vp, i64, i64, vp]),
        "gsw_degree_stats": (i32, [i64, vp, vp]),
        "gsw_tree_create": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, P(vp)]),
        "gsw_tree_destroy": (None, [vp]),
        "gsw_tree_predict": (i32, [vp, vp, i32, i32, P(i32), P(i32)]),
        "gsw_bfs": (i32, [vp, vp, i32, vp, vp, vp, i32, P(i32), P(BfsOpts)]),
        "gsw_bfs_profile": (i32, [vp, i32, vp, i32, i32, i32, vp, vp, i32, P(i32), vp]),
        "gsw_msbfs_opts_default": (None, [P(MsbfsOpts)]),
        "gsw_msbfs": (i32, [vp, vp, i32, vp, P(i32), P(MsbfsOpts)]),
        "gsw_session_create": (i32, [vp, i32, P(vp)]),
        "gsw_session_destroy": (None, [vp]),
        "gsw_session_admit": (i32, [vp, i32, P(i32)]),
        "gsw_session_step": (i32, [vp, i32, vp, i32, P(i32), P(i32)]),
        "gsw_session_fetch": (i32, [vp, i32, vp, i32]),
        "gsw_session_info": (i32, [vp, P(i32), P(i32), P(i64), P(ctypes.c_size_t)]),
        "gsw_session_set_thresholds": (i32, [vp, ctypes.c_float, ctypes.c_float]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st):
    if st != OK:
        raise GswError(st, (lib().gsw_last_error() or b"").decode())


def last_error() -> str:
    return (lib().gsw_last_error() or b"").decode()


def kernel_name(k: int) -> str:
    return lib().gsw_kernel_name(k).decode()


def _ptr(a) -> int:
    """Data pointer of a numpy array or torch tensor."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def validate(offs, cols):
    """Host-side CSR check; returns True when the graph is symmetric."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    sym = ctypes.c_int32(0)
    _check(lib().gsw_graph_validate(offs.shape[0] - 1, cols.shape[0], offs.ctypes.data,
                                    cols.ctypes.data, ctypes.byref(sym)))
    return bool(sym.value)


def degree_stats(offs) -> np.ndarray:
    """The library's {min, q1, median, q3, max, std} of a host CSR's degrees."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    out = np.empty(6, dtype=np.float64)
    _check(lib().gsw_degree_stats(offs.shape[0] - 1, offs.ctypes.data, out.ctypes.data))
    return out


class Graph:
    """A graph resident in device memory."""

    def __init__(self, handle, n, nnz, keep=None):
        self._h = ctypes.c_void_p(handle)
        self.n = int(n)
        self.nnz = int(nnz)
        self._keep = keep  # borrowed device tensors

    @classmethod
    def from_csr(cls, offs, cols, flags: int = 0, stream=None):
        """numpy arrays are copied to the device; torch CUDA tensors are
        borrowed (kept alive by this object)."""
        out = ctypes.c_void_p()
        if hasattr(offs, "is_cuda") and offs.is_cuda:
            import torch

            offs = offs.to(torch.int64).contiguous()
            cols = cols.to(torch.int32).contiguous()
            n, nnz = offs.shape[0] - 1, cols.shape[0]
            s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
            _check(lib().gsw_graph_create_device(n, nnz, offs.data_ptr(), cols.data_ptr(), flags, s,
                                                 ctypes.byref(out)))
            return cls(out.value, n, nnz, keep=(offs, cols))
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n, nnz = offs.shape[0] - 1, cols.shape[0]
        _check(lib().gsw_graph_create_host(n, nnz, offs.ctypes.data, cols.ctypes.data, flags,
                                           ctypes.byref(out)))
        return cls(out.value, n, nnz)

    @property
    def handle(self):
        return self._h

    def info(self):
        n, nnz, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        st = (ctypes.c_double * 6)()
        _check(lib().gsw_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz), st, ctypes.byref(b)))
        return dict(n=n.value, nnz=nnz.value, deg_stats=list(st), dev_bytes=b.value)

    def level_features(self, n_frontier: int, discovered: int) -> np.ndarray:
        out = np.empty(N_FEATURES, dtype=np.float64)
        _check(lib().gsw_level_features(self._h, n_frontier, discovered, out.ctypes.data))
        return out

    def close(self):
        if self._h is not None and self._h.value:
            lib().gsw_graph_destroy(self._h)
        self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Decision tree (flat CART arrays) mapping features to a kernel."""

    def __init__(self, arrays: dict):
        self.arrays = arrays
        feat = np.ascontiguousarray(arrays["feature"], dtype=np.int32)
        thr = np.ascontiguousarray(arrays["threshold"], dtype=np.float64)
        left = np.ascontiguousarray(arrays["left"], dtype=np.int32)
        right = np.ascontiguousarray(arrays["right"], dtype=np.int32)
        val = np.ascontiguousarray(arrays["value"], dtype=np.float64)
        ck = np.ascontiguousarray(arrays["class_kernel"], dtype=np.int32)
        n_nodes, n_classes = val.shape
        # inner nodes only carry a feature index; leaves carry -2 in sklearn
        feat = np.where(left == -1, 0, feat).astype(np.int32)
        out = ctypes.c_void_p()
        _check(lib().gsw_tree_create(n_nodes, n_classes, feat.ctypes.data, thr.ctypes.data,
                                     left.ctypes.data, right.ctypes.data, val.ctypes.data,
                                     ck.ctypes.data, ctypes.byref(out)))
        self._h = out
        self.n_nodes, self.n_classes = n_nodes, n_classes

    @classmethod
    def load(cls, path: str) -> "Tree":
        with open(path) as f:
            return cls(json.load(f))

    @classmethod
    def constant(cls, kernel: int) -> "Tree":
        """A one-leaf tree that always picks ``kernel``."""
        return cls(dict(feature=[0], threshold=[-2.0], left=[-1], right=[-1], value=[[1.0]],
                        class_kernel=[kernel]))

    def predict(self, x, prev_kernel: int, level: int):
        x = np.ascontiguousarray(x, dtype=np.float64)
        k, u = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gsw_tree_predict(self._h, x.ctypes.data, prev_kernel, level, ctypes.byref(k),
                                      ctypes.byref(u)))
        return k.value, bool(u.value)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if self._h is not None and self._h.value:
                lib().gsw_tree_destroy(self._h)
            self._h = None
        except Exception:
            pass


@dataclass
class TraceRow:
    source_idx: int
    level: int
    kernel: int
    flags: int
    n_frontier: int
    discovered: int
    n_next: int
    ms: float

    @property
    def kernel_name(self):
        return KERNEL_NAMES[self.kernel]


def _opts(policy, kernel, schedule, tree, time_levels, canonical_parents, device_ptrs, stream):
    o = BfsOpts()
    lib().gsw_bfs_opts_default(ctypes.byref(o))
    keep = None
    if policy == "tree":
        if tree is None:
            raise ValueError("tree policy needs a tree")
        o.policy = POLICY_TREE
        o.tree = tree.handle.value
    elif policy == "fixed":
        o.policy = POLICY_FIXED
        o.fixed_kernel = int(kernel)
    elif policy == "schedule":
        keep = np.ascontiguousarray(schedule, dtype=np.int32)
        o.policy = POLICY_SCHEDULE
        o.schedule = keep.ctypes.data
        o.schedule_len = keep.shape[0]
    else:
        raise ValueError("policy must be tree, fixed or schedule")
    o.time_levels = int(bool(time_levels))
    o.canonical_parents = int(bool(canonical_parents))
    o.device_ptrs = int(bool(device_ptrs))
    o.stream = stream
    return o, keep


def bfs(graph: Graph, sources, policy: str = "tree", kernel: int = PUSH_VERTEX, schedule=None,
        tree: Tree = None, parents: bool = True, time_levels: bool = False,
        canonical_parents: bool = False, device: bool = False, stream=None, out=None,
        trace_cap: int = None, max_workgroups: int = 0):
    """Level-switched BFS from each source.

    Returns ``(levels, parents, trace)``: ``levels`` is ``[len(sources), n]``
    int32 (numpy on the host, or a torch CUDA tensor when ``device``),
    ``parents`` likewise or None, ``trace`` a list of TraceRow.
    ``out`` may supply preallocated ``(levels, parents)`` device tensors.
    ``max_workgroups`` > 0 caps every level launch (for tests of the
    striding paths; 0 lets the library size launches).
    """
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    S, n = src.shape[0], graph.n
    if device:
        import torch

        if out is not None:
            lv, pa = out
        else:
            lv = torch.empty((S, n), dtype=torch.int32, device="cuda")
            pa = torch.empty((S, n), dtype=torch.int32, device="cuda") if parents else None
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
    else:
        lv = np.empty((S, n), dtype=np.int32)
        pa = np.empty((S, n), dtype=np.int32) if parents else None
    o, keep = _opts(policy, kernel, schedule, tree, time_levels, canonical_parents, device, stream)
    o.max_workgroups = int(max_workgroups)
    cap = trace_cap if trace_cap is not None else 64 * max(S, 1)
    while True:
        tr = (LevelTrace * max(cap, 1))()
        tlen = ctypes.c_int32(0)
        _check(lib().gsw_bfs(graph.handle, src.ctypes.data, S, _ptr(lv),
                             _ptr(pa) if pa is not None else None, tr, cap, ctypes.byref(tlen),
                             ctypes.byref(o)))
        if tlen.value <= cap or trace_cap is not None:
            break
        cap = tlen.value  # rerun once with room for every row
    rows = [TraceRow(t.source_idx, t.level, t.kernel, t.flags, t.n_frontier, t.discovered,
                     t.n_next, t.ms) for t in tr[:min(tlen.value, cap)]]
    del keep
    return lv, pa, rows


class Runner:
    """Repeated single-source BFS on one graph with arguments marshalled once.

    ``run(source)`` calls gsw_bfs directly (levels/parents in the given
    device tensors, trace rows in a reusable buffer) and returns the number
    of trace rows; ``rows()`` decodes them on demand.
    """

    def __init__(self, graph: Graph, levels, parents=None, policy: str = "tree", kernel=PUSH_VERTEX,
                 schedule=None, tree: Tree = None, time_levels: bool = False, stream=None,
                 trace_cap: int = 4096):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.graph, self.levels, self.parents, self.tree = graph, levels, parents, tree
        self.opts, self._keep = _opts(policy, kernel, schedule, tree, time_levels, False, True, stream)
        self.trace = (LevelTrace * trace_cap)()
        self.cap = trace_cap
        self.tlen = ctypes.c_int32(0)
        self.src = np.zeros(1, dtype=np.int32)
        self._args = None

    def set_schedule(self, schedule):
        self._keep = np.ascontiguousarray(schedule, dtype=np.int32)
        self.opts.schedule = self._keep.ctypes.data
        self.opts.schedule_len = self._keep.shape[0]

    def run(self, source: int) -> int:
        self.src[0] = source
        _check(lib().gsw_bfs(self.graph.handle, self.src.ctypes.data, 1, _ptr(self.levels),
                             _ptr(self.parents) if self.parents is not None else None, self.trace,
                             self.cap, ctypes.byref(self.tlen), ctypes.byref(self.opts)))
        return self.tlen.value

    def rows(self):
        return [TraceRow(t.source_idx, t.level, t.kernel, t.flags, t.n_frontier, t.discovered,
                         t.n_next, t.ms) for t in self.trace[:min(self.tlen.value, self.cap)]]


def msbfs(graph: Graph, sources, push_to_pull: float = None, pull_to_push: float = None,
          device: bool = False, stream=None, out=None, use_graph: bool = True):
    """Batched BFS of up to 1024 sources.  Returns ``(levels int8 [S][n], n_levels)``;
    levels are a torch CUDA tensor when ``device`` (or ``out`` is given).
    ``use_graph`` replays the captured two-level HIP graph instead of
    launching each kernel."""
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    S, n = src.shape[0], graph.n
    o = MsbfsOpts()
    lib().gsw_msbfs_opts_default(ctypes.byref(o))
    o.graph = 1 if use_graph else 0
    if push_to_pull is not None:
        o.push_to_pull = push_to_pull
    if pull_to_push is not None:
        o.pull_to_push = pull_to_push
    if device or out is not None:
        import torch

        lv = out if out is not None else torch.empty((S, n), dtype=torch.int8, device="cuda")
        o.device_ptrs = 1
        o.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    else:
        lv = np.empty((S, n), dtype=np.int8)
        o.stream = stream
    nl = ctypes.c_int32(0)
    _check(lib().gsw_msbfs(graph.handle, src.ctypes.data, S, _ptr(lv), ctypes.byref(nl),
                           ctypes.byref(o)))
    return lv, nl.value


class Session:
    """Continuously batched single-source queries on one graph (gsw_session_*)."""

    def __init__(self, graph: Graph, slots: int = 64):
        out = ctypes.c_void_p()
        _check(lib().gsw_session_create(graph.handle, slots, ctypes.byref(out)))
        self._h = out
        self.graph = graph
        self.slots = slots
        self._fin = np.zeros(slots, dtype=np.int32)

    def admit(self, source: int):
        """Slot index, or None when every slot is busy."""
        k = ctypes.c_int32(-1)
        st = lib().gsw_session_admit(self._h, int(source), ctypes.byref(k))
        if st == EBUSY:
            return None
        _check(st)
        return k.value

    def step(self, max_levels: int = 8):
        """Runs levels until a slot finishes, ``max_levels`` have run or nothing
        is admitted or running; queries admitted meanwhile (from any thread)
        join at level boundaries.  Returns (finished slots, levels run)."""
        nf, lr = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().gsw_session_step(self._h, max_levels, self._fin.ctypes.data, self.slots,
                                      ctypes.byref(nf), ctypes.byref(lr)))
        return self._fin[:nf.value].tolist(), lr.value

    def fetch(self, slot: int, out=None):
        """The slot's int32 levels (into ``out``, a torch CUDA tensor or numpy
        array, when given) and frees the slot."""
        if out is None:
            out = np.empty(self.graph.n, dtype=np.int32)
        dev = 1 if hasattr(out, "data_ptr") else 0
        _check(lib().gsw_session_fetch(self._h, int(slot), _ptr(out), dev))
        return out

    def info(self):
        s, b, it, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().gsw_session_info(self._h, ctypes.byref(s), ctypes.byref(b), ctypes.byref(it),
                                      ctypes.byref(nb)))
        return dict(slots=s.value, busy=b.value, iteration=it.value, dev_bytes=nb.value)

    def set_thresholds(self, push_to_pull: float, pull_to_push: float):
        _check(lib().gsw_session_set_thresholds(self._h, push_to_pull, pull_to_push))

    def close(self):
        if self._h is not None and self._h.value:
            lib().gsw_session_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bfs_profile(graph: Graph, source: int, kernels=None, reps: int = 5,
                advance_kernel: int = PUSH_EDGE, max_levels: int = 100000, stream=None):
    """Per-level median time (ms) of each kernel from the same saved state.

    Returns ``(times [levels][len(kernels)], frontier [levels], kernels)``.
    """
    ks = np.ascontiguousarray(kernels if kernels is not None else range(N_KERNELS), dtype=np.int32)
    cap = max_levels
    times = np.empty((cap, ks.shape[0]), dtype=np.float32)
    fr = np.empty(cap, dtype=np.int64)
    nl = ctypes.c_int32(0)
    _check(lib().gsw_bfs_profile(graph.handle, int(source), ks.ctypes.data, ks.shape[0], reps,
                                 advance_kernel, times.ctypes.data, fr.ctypes.data, cap,
                                 ctypes.byref(nl), stream))
    return times[:nl.value].copy(), fr[:nl.value].copy(), ks.tolist()
