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

# base kernels (values of GSW_K_* in include/gsw.h)
PUSH_VERTEX, PUSH_WAVE4, PUSH_WAVE8, PUSH_WAVE16, PUSH_WAVE32, PUSH_WAVE64 = 0, 1, 2, 3, 4, 5
PUSH_EDGE, PULL_BITMAP, VERTEX_SCAN, EDGE_SCAN, REV_EDGE_SCAN = 6, 7, 8, 9, 10
N_BASE_KERNELS = 11
BASE_NAMES = ("push_vertex", "push_wave4", "push_wave8", "push_wave16", "push_wave32",
              "push_wave64", "push_edge", "pull_bitmap", "vertex_scan", "edge_scan", "rev_edge_scan")
# frontier-count variants (GSW_COUNT_*); a kernel id = base + N_BASE_KERNELS * variant
COUNT_WORKGROUP, COUNT_WAVE, COUNT_THREAD = 0, 1, 2
COUNT_NAMES = ("", ".wave", ".thread")
N_KERNELS = N_BASE_KERNELS * 3
KERNEL_NAMES = tuple(b + c for c in COUNT_NAMES for b in BASE_NAMES)
DEFAULT_KERNEL = PUSH_EDGE


def kernel_id(base: int, variant: int = COUNT_WORKGROUP) -> int:
    return base + N_BASE_KERNELS * variant


def kernel_base(k: int) -> int:
    return k % N_BASE_KERNELS


def kernel_count(k: int) -> int:
    return k // N_BASE_KERNELS


N_FEATURES = 24
N_GRAPH_FEATURES = 20
FEATURE_NAMES = ("n_vertices", "n_edges",
                 "out_deg_min", "out_deg_q1", "out_deg_median", "out_deg_q3", "out_deg_max", "out_deg_std",
                 "in_deg_min", "in_deg_q1", "in_deg_median", "in_deg_q3", "in_deg_max", "in_deg_std",
                 "abs_deg_min", "abs_deg_q1", "abs_deg_median", "abs_deg_q3", "abs_deg_max", "abs_deg_std",
                 "frontier", "frontier_frac", "discovered", "discovered_frac")

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
                ("n_next", ctypes.c_int64), ("e_frontier", ctypes.c_int64),
                ("ms", ctypes.c_float), ("launch", ctypes.c_int32)]


class BfsOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("fixed_kernel", ctypes.c_int32),
                ("schedule", ctypes.c_void_p), ("schedule_len", ctypes.c_int32),
                ("tree", ctypes.c_void_p), ("time_levels", ctypes.c_int32),
                ("canonical_parents", ctypes.c_int32), ("device_ptrs", ctypes.c_int32),
                ("max_workgroups", ctypes.c_int32), ("count_arcs", ctypes.c_int32),
                ("no_solo", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class MsbfsOpts(ctypes.Structure):
    _fields_ = [("push_to_pull", ctypes.c_float), ("pull_to_push", ctypes.c_float),
                ("device_ptrs", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("wide_levels", ctypes.c_void_p), ("wide_index", ctypes.c_void_p),
                ("wide_cap", ctypes.c_int32), ("n_wide", ctypes.c_void_p),
                ("tree", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class CcTrace(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int32), ("kernel", ctypes.c_int32), ("n_active", ctypes.c_int64),
                ("e_active", ctypes.c_int64), ("changed", ctypes.c_int64), ("ms", ctypes.c_float),
                ("pad", ctypes.c_int32)]


class CcOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("bfs_first", ctypes.c_int32), ("tree", ctypes.c_void_p),
                ("pull_above", ctypes.c_float), ("device_ptrs", ctypes.c_int32), ("stream", ctypes.c_void_p)]


CC_SWITCH, CC_PUSH, CC_PULL = 0, 1, 2          # gsw_cc_opts.policy
CC_K_BFS, CC_K_PUSH, CC_K_PULL = 0, 1, 2       # gsw_cc_trace.kernel
CC_KERNEL_NAMES = ("bfs", "push", "pull")

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
        "gsw_source_digest": (ctypes.c_char_p, []),
        "gsw_bfs_opts_default": (None, [P(BfsOpts)]),
        "gsw_graph_validate": (i32, [i64, i64, vp, vp, P(i32)]),
        "gsw_graph_create_host": (i32, [i64, i64, vp, vp, u32, P(vp)]),
        "gsw_graph_create_device": (i32, [i64, i64, vp, vp, u32, vp, P(vp)]),
        "gsw_graph_destroy": (None, [vp]),
        "gsw_graph_info": (i32, [vp, P(i64), P(i64), vp, P(ctypes.c_size_t)]),
        "gsw_graph_symmetric": (i32, [vp]),
        "gsw_graph_features_host": (i32, [i64, i64, vp, vp, vp]),
        "gsw_feature_name": (ctypes.c_char_p, [i32]),
        "gsw_tree_load": (i32, [ctypes.c_char_p, P(vp)]),
        "gsw_session_bytes": (ctypes.c_size_t, [vp, i32]),
        "gsw_graph_workspace_bytes": (ctypes.c_size_t, [vp]),
        "gsw_session_rebase": (i32, [vp, i64]),
        "gsw_level_features": (i32, [vp, i64, i64, vp]),
        "gsw_degree_stats": (i32, [i64, vp, vp]),
        "gsw_tree_create": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, P(vp)]),
        "gsw_tree_destroy": (None, [vp]),
        "gsw_tree_predict": (i32, [vp, vp, i32, i32, P(i32), P(i32)]),
        "gsw_bfs": (i32, [vp, vp, i32, vp, vp, vp, i32, P(i32), P(BfsOpts)]),
        "gsw_bfs_noalloc": (i32, [vp, vp, i32, vp, vp, vp, i32, P(i32), P(BfsOpts)]),
        "gsw_bfs_profile": (i32, [vp, i32, vp, i32, i32, i32, vp, vp, i32, P(i32), vp]),
        "gsw_msbfs_opts_default": (None, [P(MsbfsOpts)]),
        "gsw_msbfs": (i32, [vp, vp, i32, vp, P(i32), P(MsbfsOpts)]),
        "gsw_session_create": (i32, [vp, i32, P(vp)]),
        "gsw_session_destroy": (None, [vp]),
        "gsw_session_admit": (i32, [vp, i32, P(i32)]),
        "gsw_session_step": (i32, [vp, i32, vp, i32, P(i32), P(i32)]),
        "gsw_session_fetch": (i32, [vp, i32, vp, i32]),
        "gsw_session_cancel": (i32, [vp, i32]),
        "gsw_session_info": (i32, [vp, P(i32), P(i32), P(i64), P(ctypes.c_size_t)]),
        "gsw_session_set_thresholds": (i32, [vp, ctypes.c_float, ctypes.c_float]),
        "gsw_cc_opts_default": (None, [P(CcOpts)]),
        "gsw_cc": (i32, [vp, vp, P(i64), vp, i32, P(i32), P(CcOpts)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    from .build import source_digest

    built, here = L.gsw_source_digest().decode(), source_digest()
    if built != here:
        raise RuntimeError("libgsw.so was built from other sources (stamp %s, sources %s); rebuild with "
                           "python -m paper_1708_01159_amd.build" % (built, here))
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


_NP_DTYPES = {"int32": np.int32, "int8": np.int8}


def check_out(t, dtype: str, numel: int, device: bool, what: str):
    """Rejects an output buffer the library would write out of bounds or to the
    wrong memory: a torch tensor must be a CUDA tensor (when ``device``) of
    exactly ``dtype``, contiguous, with at least ``numel`` elements; a numpy
    array (host output) likewise.  Raises ValueError."""
    if t is None:
        raise ValueError("%s: no buffer" % what)
    if hasattr(t, "data_ptr"):  # torch
        import torch

        if not device:
            raise ValueError("%s: a torch tensor was given for host output" % what)
        if not t.is_cuda:
            raise ValueError("%s: expected a CUDA tensor, got one on %s" % (what, t.device))
        if t.dtype != getattr(torch, dtype):
            raise ValueError("%s: expected torch.%s, got %s" % (what, dtype, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s: tensor is not contiguous" % what)
        if t.numel() < numel:
            raise ValueError("%s: %d elements, need %d" % (what, t.numel(), numel))
        return
    if device:
        raise ValueError("%s: expected a CUDA tensor, got %s" % (what, type(t).__name__))
    if not isinstance(t, np.ndarray):
        raise ValueError("%s: expected a numpy array or torch tensor, got %s" % (what, type(t).__name__))
    if t.dtype != _NP_DTYPES[dtype]:
        raise ValueError("%s: expected %s, got %s" % (what, dtype, t.dtype))
    if not t.flags["C_CONTIGUOUS"] or not t.flags["WRITEABLE"]:
        raise ValueError("%s: array is not contiguous and writeable" % what)
    if t.size < numel:
        raise ValueError("%s: %d elements, need %d" % (what, t.size, numel))


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

    @property
    def symmetric(self) -> bool:
        return bool(lib().gsw_graph_symmetric(self._h))

    def workspace_bytes(self) -> int:
        """Device bytes of the single-source workspace (allocated on first use)."""
        return int(lib().gsw_graph_workspace_bytes(self._h))

    def session_bytes(self, slots: int) -> int:
        """Device bytes a serving session of ``slots`` slots on this graph allocates."""
        return int(lib().gsw_session_bytes(self._h, int(slots)))

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
        """Reads the JSON export with the library's own reader (gsw_tree_load)."""
        with open(path) as f:
            arrays = json.load(f)
        out = ctypes.c_void_p()
        _check(lib().gsw_tree_load(os.fsencode(path), ctypes.byref(out)))
        t = cls.__new__(cls)
        t.arrays = arrays
        t._h = out
        t.n_nodes = len(arrays["left"])
        t.n_classes = len(arrays["class_kernel"])
        return t

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
    e_frontier: int = -1
    launch: int = -1

    @property
    def kernel_name(self):
        return KERNEL_NAMES[self.kernel]


def _row(t):
    return TraceRow(t.source_idx, t.level, t.kernel, t.flags, t.n_frontier, t.discovered, t.n_next, t.ms,
                    t.e_frontier, t.launch)


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
    o.time_levels = int(time_levels)  # 0, 1 (device clock) or 2 (HIP events)
    o.canonical_parents = int(bool(canonical_parents))
    o.device_ptrs = int(bool(device_ptrs))
    o.stream = stream
    return o, keep


def bfs(graph: Graph, sources, policy: str = "tree", kernel: int = PUSH_VERTEX, schedule=None,
        tree: Tree = None, parents: bool = True, time_levels: bool = False,
        canonical_parents: bool = False, device: bool = False, stream=None, out=None,
        trace_cap: int = None, max_workgroups: int = 0, count_arcs: bool = False, solo: bool = True):
    """Level-switched BFS from each source.

    Returns ``(levels, parents, trace)``: ``levels`` is ``[len(sources), n]``
    int32 (numpy on the host, or a torch CUDA tensor when ``device``),
    ``parents`` likewise or None, ``trace`` a list of TraceRow.
    ``out`` may supply preallocated ``(levels, parents)`` device tensors.
    ``max_workgroups`` > 0 caps every level launch (for tests of the
    striding paths; 0 lets the library size launches).  ``count_arcs``
    fills each trace row's ``e_frontier``.  ``solo`` allows the
    single-workgroup multi-level launches for small frontiers.
    """
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    S, n = src.shape[0], graph.n
    if device:
        import torch

        if out is not None:
            lv, pa = out
            check_out(lv, "int32", S * n, True, "bfs levels")
            if pa is not None:
                check_out(pa, "int32", S * n, True, "bfs parents")
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
    o.count_arcs = int(bool(count_arcs))
    o.no_solo = int(not solo)
    cap = trace_cap if trace_cap is not None else 64 * max(S, 1)
    while True:
        tr = (LevelTrace * max(cap, 1))()
        tlen = ctypes.c_int32(0)
        _check(lib().gsw_bfs(graph.handle, src.ctypes.data, S, _ptr(lv), _ptr(pa) if pa is not None else None,
                             tr, cap, ctypes.byref(tlen), ctypes.byref(o)))
        if tlen.value <= cap or trace_cap is not None:
            break
        cap = tlen.value  # rerun once with room for every row
    rows = [_row(t) for t in tr[:min(tlen.value, cap)]]
    del keep
    return lv, pa, rows


def bfs_noalloc(graph: Graph, sources, levels, parents=None, policy: str = "tree", kernel: int = PUSH_VERTEX,
                schedule=None, tree: Tree = None, time_levels: bool = False, canonical_parents: bool = False,
                stream=None, trace_cap: int = None, max_workgroups: int = 0, count_arcs: bool = False):
    """gsw_bfs_noalloc: the search of ``bfs`` into caller-allocated device
    tensors (``levels``, optional ``parents``: int32, ``[len(sources), n]``)
    without any allocation in the library.  Returns the trace rows."""
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    S, n = src.shape[0], graph.n
    check_out(levels, "int32", S * n, True, "bfs_noalloc levels")
    if parents is not None:
        check_out(parents, "int32", S * n, True, "bfs_noalloc parents")
    if stream is None:
        import torch

        stream = torch.cuda.current_stream().cuda_stream
    o, keep = _opts(policy, kernel, schedule, tree, time_levels, canonical_parents, True, stream)
    o.max_workgroups = int(max_workgroups)
    o.count_arcs = int(bool(count_arcs))
    cap = trace_cap if trace_cap is not None else 64 * max(S, 1)
    tr = (LevelTrace * max(cap, 1))()
    tlen = ctypes.c_int32(0)
    _check(lib().gsw_bfs_noalloc(graph.handle, src.ctypes.data, S, _ptr(levels),
                                 _ptr(parents) if parents is not None else None, tr, cap, ctypes.byref(tlen),
                                 ctypes.byref(o)))
    del keep
    return [_row(t) for t in tr[:min(tlen.value, cap)]]


def components(graph: Graph, policy: str = "switch", bfs_first: bool = True, tree: Tree = None,
               pull_above: float = None, device: bool = False, stream=None, out=None, trace_cap: int = 4096):
    """Weakly connected components (gsw_cc).  Returns ``(labels, n_components,
    trace)``: ``labels`` int32 ``[n]``, the smallest vertex id of each
    vertex's component (numpy, or a torch CUDA tensor when ``device``;
    ``out`` may supply it, a CUDA tensor when ``device``, else a numpy
    array), ``trace`` a list of dicts, one per iteration.
    ``policy``: "switch" (push or pull per iteration), "push" or "pull";
    ``tree`` picks the kernels of the phase-1 BFS (None: the default kernel)."""
    pol = {"switch": CC_SWITCH, "push": CC_PUSH, "pull": CC_PULL}[policy]
    n = graph.n
    o = CcOpts()
    lib().gsw_cc_opts_default(ctypes.byref(o))
    o.policy = pol
    o.bfs_first = int(bool(bfs_first))
    o.tree = tree.handle if tree is not None else None
    if pull_above is not None:
        o.pull_above = float(pull_above)
    if device:
        import torch

        if out is not None:
            check_out(out, "int32", n, True, "components labels")
            lab = out
        else:
            lab = torch.empty(n, dtype=torch.int32, device="cuda")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
    elif out is not None:
        check_out(out, "int32", n, False, "components labels")
        lab = out
    else:
        lab = np.empty(n, dtype=np.int32)
    o.device_ptrs = int(bool(device))
    o.stream = stream
    tr = (CcTrace * max(trace_cap, 1))()
    tlen = ctypes.c_int32(0)
    nc = ctypes.c_int64(0)
    _check(lib().gsw_cc(graph.handle, _ptr(lab), ctypes.byref(nc), tr, trace_cap, ctypes.byref(tlen),
                        ctypes.byref(o)))
    rows = [dict(iteration=t.iteration, kernel=CC_KERNEL_NAMES[t.kernel], n_active=t.n_active,
                 e_active=t.e_active, changed=t.changed, ms=t.ms) for t in tr[:min(tlen.value, trace_cap)]]
    return lab, int(nc.value), rows


class Runner:
    """Repeated single-source BFS on one graph with arguments marshalled once.

    ``run(source)`` calls gsw_bfs directly (levels/parents in the given
    device tensors, trace rows in a reusable buffer) and returns the number
    of trace rows; ``rows()`` decodes them on demand.
    """

    def __init__(self, graph: Graph, levels, parents=None, policy: str = "tree", kernel=PUSH_VERTEX,
                 schedule=None, tree: Tree = None, time_levels: bool = False, stream=None,
                 trace_cap: int = 4096, solo: bool = True):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        check_out(levels, "int32", graph.n, True, "Runner levels")
        if parents is not None:
            check_out(parents, "int32", graph.n, True, "Runner parents")
        self.graph, self.levels, self.parents, self.tree = graph, levels, parents, tree
        self.opts, self._keep = _opts(policy, kernel, schedule, tree, time_levels, False, True, stream)
        self.opts.no_solo = int(not solo)
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
        return [_row(t) for t in self.trace[:min(self.tlen.value, self.cap)]]


def msbfs(graph: Graph, sources, push_to_pull: float = None, pull_to_push: float = None,
          device: bool = False, stream=None, out=None, use_graph: bool = True, block_size: int = 0,
          fallback: bool = False, tree: Tree = None, wide_cap: int = None):
    """Batched BFS of up to 1024 sources.  Returns ``(levels int8 [S][n], n_levels)``;
    levels are a torch CUDA tensor when ``device`` (or ``out`` is given).
    ``use_graph`` replays the captured two-level HIP graph instead of
    launching each kernel; ``block_size`` (128/256/512, 0 = default) sets
    the level kernels' workgroup size.  With ``fallback`` the result is
    ``(levels, n_levels, wide)``, ``wide`` a dict {source index: int32 row}
    of the sources rerun on the single-source path because they go deeper
    than 127 (their int8 rows hold -128 beyond 127)."""
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    S, n = src.shape[0], graph.n
    o = MsbfsOpts()
    lib().gsw_msbfs_opts_default(ctypes.byref(o))
    o.graph = 1 if use_graph else 0
    o.block_size = int(block_size)
    if push_to_pull is not None:
        o.push_to_pull = push_to_pull
    if pull_to_push is not None:
        o.pull_to_push = pull_to_push
    dev = bool(device or out is not None)
    if dev:
        import torch

        if out is not None:
            check_out(out, "int8", S * n, True, "msbfs levels")
        lv = out if out is not None else torch.empty((S, n), dtype=torch.int8, device="cuda")
        o.device_ptrs = 1
        o.stream = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    else:
        lv = np.empty((S, n), dtype=np.int8)
        o.stream = stream
    keep = []
    nw = ctypes.c_int32(0)
    if fallback:
        cap = S if wide_cap is None else int(wide_cap)
        if dev:
            import torch

            wl = torch.empty((max(cap, 1), n), dtype=torch.int32, device="cuda")
        else:
            wl = np.empty((max(cap, 1), n), dtype=np.int32)
        wi = np.zeros(max(cap, 1), dtype=np.int32)
        keep += [wl, wi]
        o.fallback = 1
        o.wide_levels = _ptr(wl)
        o.wide_index = wi.ctypes.data
        o.wide_cap = cap
        o.n_wide = ctypes.addressof(nw)
        o.tree = tree.handle.value if tree is not None else None
    nl = ctypes.c_int32(0)
    _check(lib().gsw_msbfs(graph.handle, src.ctypes.data, S, _ptr(lv), ctypes.byref(nl),
                           ctypes.byref(o)))
    if not fallback:
        return lv, nl.value
    wide = {int(wi[k]): wl[k] for k in range(nw.value)}
    return lv, nl.value, wide


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
        check_out(out, "int32", self.graph.n, bool(dev), "session fetch")
        _check(lib().gsw_session_fetch(self._h, int(slot), _ptr(out), dev))
        return out

    def cancel(self, slot: int) -> bool:
        """Cancels the slot's admitted or running query (see gsw_session_cancel);
        False when the slot holds none (e.g. its query already finished)."""
        st = lib().gsw_session_cancel(self._h, int(slot))
        if st == EINVAL:
            return False
        _check(st)
        return True

    def rebase(self, iteration: int):
        """Sets the level counter (only while nothing runs; see gsw_session_rebase)."""
        _check(lib().gsw_session_rebase(self._h, int(iteration)))

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


def graph_features_host(offs, cols) -> np.ndarray:
    """The library's 20 graph features of a host CSR (no GPU)."""
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.empty(N_GRAPH_FEATURES, dtype=np.float64)
    _check(lib().gsw_graph_features_host(offs.shape[0] - 1, cols.shape[0], offs.ctypes.data,
                                         cols.ctypes.data, out.ctypes.data))
    return out


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
