"""Python binding of the gt C ABI (``include/gt.h``): argument marshalling only.

Every step of the traversal runs in the HIP kernels of ``libgt.so``; this
module passes device pointers (torch CUDA tensors) and HIP streams through
ctypes and turns status codes into exceptions. There is no CPU fallback: if
the library cannot be loaded or no GPU is present, calls raise.

The traversal follows C. Zhang, arXiv 2009.07463: degree-0 and degree-1
vertices are split off (Algorithm 8, MH = 0), direction-optimizing BFS
(Algorithm 1) runs on the relabelled core, and a sequential leaf pass
(Algorithm 7) completes the parent and level arrays (driver: Algorithm 9).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgt.so")

GT_OK, GT_E_INVALID, GT_E_NOMEM, GT_E_HIP, GT_E_DEPTH, GT_E_BUSY, GT_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
GT_BUILD_PLAIN, GT_BUILD_SPLIT, GT_BUILD_KEEP_LEAVES, GT_BUILD_RMZERO = 0, 1, 2, 3
GT_BUILD_HUBS_FIRST = 4
GT_BUILD_KEEP_ZERO, GT_BUILD_RELABELLED = 8, 11


def GT_BUILD_HUB_SHARE(k: int) -> int:
    """Hubs-first build flag field: at most n_core / 2**k hubs (0: k = 4)."""
    return (int(k) & 0xF) << 16


def GT_BUILD_MH(h: int) -> int:
    """Maximum edge-tree height bits of the build flags (255: unlimited)."""
    return (int(h) & 0xFF) << 8
GT_DIR_TOP_DOWN, GT_DIR_BOTTOM_UP = 0, 1
GT_LOOP_HOST, GT_LOOP_GRAPH, GT_LOOP_DEVICE = 1, 2, 3
KERNEL_NAMES = {0: "td_edges", 1: "td_flat", 2: "bu_words", 3: "bu_list"}
GT_MAX_LEVELS = 512
UNREACHED_U8 = 255

_STATUS_NAMES = {GT_E_INVALID: "GT_E_INVALID", GT_E_NOMEM: "GT_E_NOMEM", GT_E_HIP: "GT_E_HIP",
                 GT_E_DEPTH: "GT_E_DEPTH", GT_E_BUSY: "GT_E_BUSY", GT_E_UNSUPPORTED: "GT_E_UNSUPPORTED"}


class GTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_input_edges", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("n_core", ctypes.c_int64), ("n_leaf", ctypes.c_int64), ("n_zero", ctypes.c_int64),
                ("n_core_entries", ctypes.c_int64), ("n_leaf_pairs", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("tree_height", ctypes.c_uint32),
                ("n_tree_internal", ctypes.c_int64), ("n_core_edge", ctypes.c_int64),
                ("n_edge_trees", ctypes.c_int64), ("edge_tree_vertices", ctypes.c_int64),
                ("edge_tree_max", ctypes.c_int64), ("edge_tree_min", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class LevelStats(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int32), ("kernel", ctypes.c_int32), ("frontier", ctypes.c_int64),
                ("scanned", ctypes.c_int64), ("examined", ctypes.c_int64), ("found", ctypes.c_int64),
                ("ms", ctypes.c_float), ("ms_main", ctypes.c_float),
                ("examined_long", ctypes.c_int64), ("found_long", ctypes.c_int64)]


class RunStats(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("root_class", ctypes.c_int32),
                ("ms_init", ctypes.c_float), ("ms_output", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("level", LevelStats * GT_MAX_LEVELS)]

    def levels(self):
        out = []
        for i in range(min(self.n_levels, GT_MAX_LEVELS)):
            l = self.level[i]
            out.append(dict(dir="BU" if l.dir == GT_DIR_BOTTOM_UP else "TD", kernel=KERNEL_NAMES.get(l.kernel, "?"),
                            frontier=l.frontier,
                            scanned=l.scanned, examined=l.examined, found=l.found, ms=l.ms,
                            ms_main=l.ms_main, examined_long=l.examined_long, found_long=l.found_long))
        return out


class Tuning(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("beta", ctypes.c_int32), ("bu_lane_edges", ctypes.c_int32),
                ("bu_hub_deg", ctypes.c_int32), ("bu_blocks", ctypes.c_int32),
                ("bu_hub_blocks", ctypes.c_int32), ("td_small_edges", ctypes.c_int32),
                ("td_blocks", ctypes.c_int32), ("ms_blocks", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("bu_hint", ctypes.c_int32), ("loop", ctypes.c_int32), ("graph_levels", ctypes.c_int32),
                ("td_hub_deg", ctypes.c_int32), ("bu_list_div", ctypes.c_int32), ("td_flat", ctypes.c_int32),
                ("ms_alpha", ctypes.c_int32), ("bu_gamma", ctypes.c_int32), ("ms_loop", ctypes.c_int32),
                ("bu_lds", ctypes.c_int32),
                ("bu_form", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TuneReport(ctypes.Structure):
    _fields_ = [("signature", ctypes.c_uint64), ("from_cache", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("ms_start", ctypes.c_double), ("ms_best", ctypes.c_double),
                ("ms_batch_start", ctypes.c_double), ("ms_batch_best", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["signature"] = "%016x" % self.signature
        return d


class DeviceProps(ctypes.Structure):
    _fields_ = [("arch", ctypes.c_char * 64), ("name", ctypes.c_char * 64), ("compute_units", ctypes.c_int32),
                ("clock_khz", ctypes.c_int32), ("memory_clock_khz", ctypes.c_int32),
                ("memory_bus_bits", ctypes.c_int32), ("l2_bytes", ctypes.c_int64), ("total_bytes", ctypes.c_int64),
                ("peak_hbm_gbs", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["arch"] = self.arch.decode(errors="replace")
        d["name"] = self.name.decode(errors="replace")
        return d


GT_TUNE_FORCE, GT_TUNE_BATCH = 1, 2

_lib = None


def load_library(build_if_missing: bool = True):
    """Load libgt.so (building it in-tree only if no build exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError("libgt.so is not built (python -m paper_2009_07463_amd.build_lib)")
        from . import build_lib
        build_lib.build()
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "gt_build_graph": [P, P, I64, I64, U32, P, ctypes.POINTER(P)],
        "gt_graph_destroy": [P],
        "gt_graph_info_get": [P, ctypes.POINTER(GraphInfo)],
        "gt_graph_degrees": [P, P, P],
        "gt_bfs": [P, I32, P, P, P],
        "gt_bfs_static": [P, I32, P, P, P],
        "gt_last_run_stats": [P, ctypes.POINTER(RunStats)],
        "gt_get_tuning": [P, ctypes.POINTER(Tuning)],
        "gt_set_tuning": [P, ctypes.POINTER(Tuning)],
        "gt_bfs_batch": [P, P, I32, P, P],
        "gt_reconstruct_parent": [P, I32, P, P, P],
        "gt_levels_to_u8": [P, I64, P, P],
        "gt_session_create": [P, I32, P, ctypes.POINTER(P)],
        "gt_session_admit": [P, I32, P, ctypes.POINTER(I32)],
        "gt_session_step": [P, ctypes.POINTER(ctypes.c_uint64)],
        "gt_session_active": [P, ctypes.POINTER(I32)],
        "gt_session_destroy": [P],
        "gt_autotune": [P, P, I32, ctypes.c_char_p, U32, P, ctypes.POINTER(Tuning), ctypes.POINTER(TuneReport)],
        "gt_device_props_get": [I32, ctypes.POINTER(DeviceProps)],
        "gt_memory_in_use": [ctypes.POINTER(I64)],
        "gt_set_memory_limit": [I64],
        "gt_stream_copy": [P, P, I64, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.gt_last_error.argtypes = []
    lib.gt_last_error.restype = ctypes.c_char_p
    lib.gt_version.argtypes = []
    lib.gt_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code: int):
    if code != GT_OK:
        msg = load_library().gt_last_error().decode(errors="replace")
        raise GTError(code, msg)


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype: torch.dtype, numel: int, name: str) -> int:
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError("%s must be contiguous %s with >= %d elements" % (name, dtype, numel))
    return t.data_ptr()


def version() -> str:
    return load_library().gt_version().decode()


def levels_to_u8(level: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """int32 levels (-1 = unreached) to the uint8 batch encoding (255 =
    unreached), by the library (gt_levels_to_u8)."""
    n = level.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=level.device)
    _check(load_library().gt_levels_to_u8(_dev_ptr(level, torch.int32, n, "level") if n else None, n,
                                          _dev_ptr(out, torch.uint8, n, "out") if n else None,
                                          _stream_ptr(stream)))
    return out


def device_props(device: int = 0) -> dict:
    """hipDeviceProp_t fields of a device, with the double-data-rate HBM peak
    they imply (gt_device_props_get)."""
    out = DeviceProps()
    _check(load_library().gt_device_props_get(int(device), ctypes.byref(out)))
    return out.as_dict()


def memory_in_use() -> int:
    """Device bytes the library holds (gt_memory_in_use)."""
    out = ctypes.c_int64(0)
    _check(load_library().gt_memory_in_use(ctypes.byref(out)))
    return out.value


def set_memory_limit(nbytes: int):
    """Cap on the library's device memory (0: none; gt_set_memory_limit)."""
    _check(load_library().gt_set_memory_limit(int(nbytes)))


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """dst[:] = src[:] by the library's streaming copy kernel (gt_stream_copy);
    byte sizes must match and be a multiple of 16."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst differ in size")
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors")
    _check(load_library().gt_stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream_ptr(stream)))


class Graph:
    """A graph resident in HBM (``gt_build_graph``).

    src, dst: int32 CUDA tensors of equal length (undirected edges).
    split=True builds the edge-leaf view (core CSR + leaf list); False keeps
    the whole graph for plain direction-optimizing BFS. rmzero=True (with
    split=True) builds the ablation that only removes isolated vertices.
    mh > 0 (with split=True) builds the edge-tree view of maximum tree height
    mh (Algorithm 8; -1 or 255: unlimited). hubs_first=True (with
    split=True) numbers the highest-degree core vertices first, at most
    n_core / 2**hub_share of them (hub_share 0: 1/16). keep_all=True (with
    split=True) splits nothing off: the whole graph, relabelled (hubs first
    if asked), through the split machinery -- plain BFS on that numbering.
    """

    def __init__(self, src: torch.Tensor, dst: torch.Tensor, n_vertices: int, split: bool = True,
                 stream=None, rmzero: bool = False, mh: int = 0, hubs_first: bool = False, hub_share: int = 0,
                 keep_all: bool = False):
        lib = load_library()
        m = src.numel()
        if dst.numel() != m:
            raise ValueError("src and dst differ in length")
        h = ctypes.c_void_p()
        sp = _dev_ptr(src, torch.int32, m, "src") if m else None
        dp = _dev_ptr(dst, torch.int32, m, "dst") if m else None
        if keep_all:
            kind = GT_BUILD_RELABELLED if split else GT_BUILD_KEEP_ZERO
        elif split:
            kind = GT_BUILD_RMZERO if rmzero else GT_BUILD_SPLIT
        else:
            kind = GT_BUILD_KEEP_LEAVES if rmzero else GT_BUILD_PLAIN
        _check(lib.gt_build_graph(sp, dp, m, int(n_vertices), kind |
                                  GT_BUILD_MH(255 if mh < 0 else mh) |
                                  ((GT_BUILD_HUBS_FIRST | GT_BUILD_HUB_SHARE(hub_share)) if hubs_first else 0),
                                  _stream_ptr(stream),
                                  ctypes.byref(h)))
        self._h = h
        self.n = int(n_vertices)
        self.split = bool(split)
        self.rmzero = bool(rmzero)
        self.keep_all = bool(keep_all)
        self.mh = int(mh)
        self.device = src.device if m else torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            load_library().gt_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph is closed")
        return self._h

    def info(self) -> dict:
        out = GraphInfo()
        _check(load_library().gt_graph_info_get(self.handle, ctypes.byref(out)))
        return out.as_dict()

    def degrees(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(load_library().gt_graph_degrees(self.handle, _dev_ptr(out, torch.int32, self.n, "out"),
                                               _stream_ptr(stream)))
        return out

    def bfs(self, root: int, parent: torch.Tensor | None = None, level: torch.Tensor | None = None,
            stream=None):
        """(parent, level) int32 CUDA tensors of a BFS from root (caller ids)."""
        if parent is None:
            parent = torch.empty(self.n, dtype=torch.int32, device=self.device)
        if level is None:
            level = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(load_library().gt_bfs(self.handle, int(root), _dev_ptr(parent, torch.int32, self.n, "parent"),
                                     _dev_ptr(level, torch.int32, self.n, "level"), _stream_ptr(stream)))
        return parent, level

    def bfs_static(self, root: int, parent: torch.Tensor, level: torch.Tensor, stream=None):
        """BFS from root into caller-provided (parent, level) int32 CUDA
        tensors, with the library's static working memory (gt_bfs_static:
        no device allocation in the call)."""
        _check(load_library().gt_bfs_static(self.handle, int(root), _dev_ptr(parent, torch.int32, self.n, "parent"),
                                            _dev_ptr(level, torch.int32, self.n, "level"), _stream_ptr(stream)))
        return parent, level

    def last_stats(self) -> RunStats:
        out = RunStats()
        _check(load_library().gt_last_run_stats(self.handle, ctypes.byref(out)))
        return out

    def tuning(self) -> Tuning:
        out = Tuning()
        _check(load_library().gt_get_tuning(self.handle, ctypes.byref(out)))
        return out

    def set_tuning(self, **kw):
        t = Tuning()
        for name, _ in Tuning._fields_:
            if name != "reserved":
                setattr(t, name, -1 if name == "timing" else 0)
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(load_library().gt_set_tuning(self.handle, ctypes.byref(t)))

    def autotune(self, roots, cache_path: str | None = None, force: bool = False, batch: bool = False,
                 stream=None):
        """Tune this handle's knobs by timed trials (gt_autotune); returns
        (tuning dict, report dict)."""
        roots = [int(r) for r in roots]
        arr = (ctypes.c_int32 * max(len(roots), 1))(*roots)
        t, rep = Tuning(), TuneReport()
        flags = (GT_TUNE_FORCE if force else 0) | (GT_TUNE_BATCH if batch else 0)
        _check(load_library().gt_autotune(self.handle, ctypes.cast(arr, ctypes.c_void_p), len(roots),
                                          cache_path.encode() if cache_path else None, flags,
                                          _stream_ptr(stream), ctypes.byref(t), ctypes.byref(rep)))
        return t.as_dict(), rep.as_dict()

    def bfs_batch(self, roots, levels: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """uint8 CUDA tensor [k, n]: levels from each root (255 = unreached)."""
        roots = [int(r) for r in roots]
        k = len(roots)
        if levels is None:
            levels = torch.empty((k, self.n), dtype=torch.uint8, device=self.device)
        arr = (ctypes.c_int32 * max(k, 1))(*roots)
        _check(load_library().gt_bfs_batch(self.handle, ctypes.cast(arr, ctypes.c_void_p), k,
                                           _dev_ptr(levels, torch.uint8, k * self.n, "levels"),
                                           _stream_ptr(stream)))
        return levels

    def reconstruct_parent(self, root: int, level_u8: torch.Tensor, parent: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
        if parent is None:
            parent = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(load_library().gt_reconstruct_parent(
            self.handle, int(root), _dev_ptr(level_u8, torch.uint8, self.n, "level"),
            _dev_ptr(parent, torch.int32, self.n, "parent"), _stream_ptr(stream)))
        return parent


class Session:
    """Continuous-batching session over one graph (``gt_session_*``)."""

    def __init__(self, graph: Graph, slots: int = 64, stream=None):
        self.graph = graph
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(load_library().gt_session_create(graph.handle, int(slots), _stream_ptr(self.stream),
                                                ctypes.byref(h)))
        self._h = h
        self.slots = int(slots)

    def admit(self, root: int, level_out: torch.Tensor) -> int:
        slot = ctypes.c_int32(-1)
        _check(load_library().gt_session_admit(self._h, int(root),
                                               _dev_ptr(level_out, torch.uint8, self.graph.n, "level_out"),
                                               ctypes.byref(slot)))
        return slot.value

    def try_admit(self, root: int, level_out: torch.Tensor):
        try:
            return self.admit(root, level_out)
        except GTError as e:
            if e.code == GT_E_BUSY:
                return None
            raise

    def step(self) -> int:
        done = ctypes.c_uint64(0)
        _check(load_library().gt_session_step(self._h, ctypes.byref(done)))
        return done.value

    def active(self) -> int:
        a = ctypes.c_int32(0)
        _check(load_library().gt_session_active(self._h, ctypes.byref(a)))
        return a.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().gt_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
