"""Python binding of libhpm (ctypes).  Argument marshalling only.

Every step of matching runs in the HIP library; this module converts numpy
arrays and torch device buffers/streams into the pointers the C ABI
(include/hpm.h) takes.  torch supplies device memory for mapping output and
the current stream; nothing else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# HPM_LIBRARY: load another build of the same sources (e.g. a sanitizer build)
LIB_PATH = os.environ.get("HPM_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libhpm.so")

OK, E_ARG, E_GRAPH, E_PATTERN, E_NOMEM, E_TRUNCATED, E_OVERFLOW, E_DEVICE, E_UNSUPPORTED, \
    E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
PENDING = 1
ISO, MONO = 0, 1
ANY, EQ, GE = 0, 1, 2
F_NO_REORDER = 0x1
ABI_VERSION = 9  # HPM_ABI_VERSION of include/hpm.h
F_TIMING = 0x2
F_NO_FILTER = 0x4
F_OVERLAP = 0x8
F_LOOKAHEAD = 0x10
F_COUNT_FROM_MAX = 0x20
F_NO_ARC_INDEX = 0x40


def F_TIMING_KINDS(*names):
    """Flag bits that limit F_TIMING to the named kernel families (KERNELS)."""
    mask = 0
    for n in names:
        mask |= 1 << KERNELS.index(n)
    return (mask & 0x1FF) << 16
MAX_K = 16
KERNELS = ("vertex_validator", "edge_scan", "row_pivot", "prefix_sum", "expand", "last_level",
           "reduce", "filter", "index")

# Every function include/hpm.h declares.
EXPORTS = ("hpm_graph_create", "hpm_graph_destroy", "hpm_graph_info", "hpm_match",
           "hpm_match_noalloc", "hpm_scan_survivors", "hpm_match_batch",
           "hpm_batch_tune", "hpm_match_batch_persistent", "hpm_batch_autotune",
           "hpm_last_batch_stats",
           "hpm_server_create", "hpm_server_submit", "hpm_server_poll", "hpm_server_read_stats",
           "hpm_server_destroy", "hpm_plan_order", "hpm_last_stats", "hpm_status_string",
           "hpm_last_error", "hpm_abi_version")


class HpmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class _Pattern(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_arcs", ctypes.c_int32),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("vop", ctypes.c_void_p), ("vval", ctypes.c_void_p),
                ("eop", ctypes.c_void_p), ("eval", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("max_matches", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("arcs_scanned", ctypes.c_uint64), ("survivors", ctypes.c_uint64),
                ("rows", ctypes.c_uint64 * (MAX_K + 1)), ("work", ctypes.c_uint64 * (MAX_K + 1)),
                ("chunks", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64),
                ("kernel_launches", ctypes.c_uint64 * len(KERNELS)),
                ("kernel_ms", ctypes.c_double * len(KERNELS)), ("ms_total", ctypes.c_double),
                ("filtered_lists", ctypes.c_uint64), ("raw_work", ctypes.c_uint64 * (MAX_K + 1)),
                ("overlap_removed", ctypes.c_uint64), ("counted_rows", ctypes.c_uint64),
                ("counted_work", ctypes.c_uint64), ("filter_rows", ctypes.c_uint64),
                ("filter_entries", ctypes.c_uint64), ("filter_pieces", ctypes.c_uint64),
                ("lookahead_removed", ctypes.c_uint64), ("index_arcs", ctypes.c_uint64)]


X_MAPPED, X_SHORTER = 0, 1


class _BatchConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("items_per_lane", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int32), ("strategy", ctypes.c_int32),
                ("task_work", ctypes.c_int64), ("blocks_per_cu", ctypes.c_int32),
                ("idle_us", ctypes.c_int32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("error_bits", ctypes.c_uint32),
                ("tasks", ctypes.c_uint64 * 4), ("launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("queue_slots", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64),
                ("fixed_bytes", ctypes.c_uint64), ("arena_capacity", ctypes.c_uint64),
                ("grid", ctypes.c_int32), ("fallback_patterns", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("ms_total", ctypes.c_double)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("workers", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


class _QueryResult(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("count", ctypes.c_uint64), ("est_bytes", ctypes.c_uint64),
                ("granted_bytes", ctypes.c_uint64), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("workers", ctypes.c_int32),
                ("running", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64),
                ("grant_pool_bytes", ctypes.c_uint64), ("granted_bytes", ctypes.c_uint64),
                ("peak_granted_bytes", ctypes.c_uint64), ("admitted", ctypes.c_uint64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libhpm.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2507_04130_amd.build`")
    # torch ships its own HIP runtime with the same soname as ROCm's; loading it
    # first makes libhpm bind to that one copy, so streams and device pointers
    # from torch are valid inside the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.hpm_graph_create.argtypes = [ctypes.POINTER(P), I32, I64, P, P, P, P, I32, P, I32, P, P]
    lib.hpm_graph_destroy.argtypes = [P]
    lib.hpm_graph_info.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I64),
                                   ctypes.POINTER(U64)]
    lib.hpm_match.argtypes = [P, ctypes.POINTER(_Pattern), ctypes.c_int, P,
                              ctypes.POINTER(_Opts), ctypes.POINTER(U64), P, U64]
    lib.hpm_scan_survivors.argtypes = [P, ctypes.POINTER(_Pattern), ctypes.c_int, P,
                                       ctypes.POINTER(_Opts), ctypes.POINTER(U64), P, U64]
    lib.hpm_match_noalloc.argtypes = [P, ctypes.POINTER(_Pattern), ctypes.c_int, P,
                                      ctypes.POINTER(_Opts), ctypes.POINTER(U64), P, U64]
    lib.hpm_match_batch.argtypes = [P, I32, ctypes.POINTER(_Pattern), P, P, ctypes.POINTER(_Opts),
                                    I32, P, P]
    lib.hpm_batch_tune.argtypes = [P, I32, ctypes.POINTER(_Pattern), P, P, ctypes.POINTER(_Opts),
                                   ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]
    lib.hpm_match_batch_persistent.argtypes = [P, I32, ctypes.POINTER(_Pattern), P, P,
                                               ctypes.POINTER(_Opts),
                                               ctypes.POINTER(_BatchConfig), P, P]
    lib.hpm_batch_autotune.argtypes = [P, I32, ctypes.POINTER(_Pattern), P, P,
                                       ctypes.POINTER(_Opts), ctypes.POINTER(_BatchConfig),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.hpm_last_batch_stats.argtypes = [ctypes.POINTER(_BatchStats)]
    lib.hpm_server_create.argtypes = [ctypes.POINTER(P), P, ctypes.POINTER(_ServerOpts)]
    lib.hpm_server_submit.argtypes = [P, ctypes.POINTER(_Pattern), ctypes.c_int, P, U64,
                                      ctypes.POINTER(U64)]
    lib.hpm_server_poll.argtypes = [P, U64, I32, ctypes.POINTER(_QueryResult)]
    lib.hpm_server_read_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.hpm_server_destroy.argtypes = [P]
    lib.hpm_plan_order.argtypes = [ctypes.POINTER(_Pattern), I32, I32, ctypes.c_uint32, P]
    lib.hpm_last_stats.argtypes = [ctypes.POINTER(_Stats)]
    lib.hpm_status_string.argtypes = [ctypes.c_int]
    lib.hpm_status_string.restype = ctypes.c_char_p
    lib.hpm_last_error.restype = ctypes.c_char_p
    lib.hpm_abi_version.restype = ctypes.c_int
    for name in ("hpm_graph_create", "hpm_graph_destroy", "hpm_graph_info", "hpm_match",
                 "hpm_match_noalloc", "hpm_scan_survivors",
                 "hpm_match_batch", "hpm_batch_tune", "hpm_match_batch_persistent",
                 "hpm_batch_autotune", "hpm_last_batch_stats",
                 "hpm_server_create", "hpm_server_submit", "hpm_server_poll",
                 "hpm_server_read_stats", "hpm_server_destroy", "hpm_plan_order",
                 "hpm_last_stats"):
        getattr(lib, name).restype = ctypes.c_int
    if lib.hpm_abi_version() != ABI_VERSION:
        # the struct mirrors in this module follow this ABI; a stale build
        # would write past them
        raise ImportError(f"{LIB_PATH} implements ABI {lib.hpm_abi_version()}, this binding "
                          f"expects {ABI_VERSION}: rebuild it with "
                          "`python -m paper_2507_04130_amd.build`")
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        lib = load()
        msg = lib.hpm_last_error().decode() or lib.hpm_status_string(status).decode()
        raise HpmError(status, msg)


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Graph:
    """A target graph resident in device memory (hpm_graph_create)."""

    def __init__(self, out_off, out_nbrs, in_off, in_nbrs, vcols=(), ecols=(), stream=None):
        lib = load()
        self._keep = [np.ascontiguousarray(out_off, dtype=np.int64),
                      _i32(out_nbrs), np.ascontiguousarray(in_off, dtype=np.int64),
                      _i32(in_nbrs)]
        n = self._keep[0].shape[0] - 1
        m = self._keep[1].shape[0]
        vc = [_i32(c) for c in vcols]
        ec = [_i32(c) for c in ecols]
        vptrs = (ctypes.c_void_p * max(1, len(vc)))(*[c.ctypes.data for c in vc])
        eptrs = (ctypes.c_void_p * max(1, len(ec)))(*[c.ctypes.data for c in ec])
        h = ctypes.c_void_p()
        _check(lib.hpm_graph_create(ctypes.byref(h), n, m, _ptr(self._keep[0]),
                                    _ptr(self._keep[1]), _ptr(self._keep[2]),
                                    _ptr(self._keep[3]), len(vc), vptrs if vc else None,
                                    len(ec), eptrs if ec else None, _stream_handle(stream)))
        self._h = h
        self._keep = None
        self.n_vcols = len(vc)
        self.n_ecols = len(ec)

    @classmethod
    def from_host(cls, hg, stream=None) -> "Graph":
        """From any object with out_off/out_nbrs/in_off/in_nbrs/vcols/ecols arrays."""
        return cls(hg.out_off, hg.out_nbrs, hg.in_off, hg.in_nbrs, hg.vcols, hg.ecols, stream)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph is closed")
        return self._h

    def info(self):
        n, m, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_uint64()
        _check(load().hpm_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                     ctypes.byref(b)))
        return {"n": n.value, "m": m.value, "device_bytes": b.value}

    def close(self):
        if getattr(self, "_h", None):
            load().hpm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _pattern_struct(p):
    arrs = {name: _i32(getattr(p, name)) for name in ("src", "dst", "vop", "vval", "eop", "eval")}
    s = _Pattern(int(p.k), int(arrs["src"].shape[0]), *[_ptr(arrs[n]) for n in
                 ("src", "dst", "vop", "vval", "eop", "eval")])
    return s, arrs


def plan_order(p, n_vcols: int = 1, n_ecols: int = 1, flags: int = 0) -> list:
    """Matching order (position -> pattern vertex) the library uses; host only."""
    s, keep = _pattern_struct(p)
    out = np.zeros(int(p.k), dtype=np.int32)
    _check(load().hpm_plan_order(ctypes.byref(s), n_vcols, n_ecols, flags, _ptr(out)))
    return out.tolist()


def _check_columns(g, p):
    nv = 0 if p.vop is None else np.asarray(p.vop).shape[-1]
    ne = 0 if p.eop is None else np.asarray(p.eop).shape[-1]
    if (p.vop is not None and nv != g.n_vcols) or (p.eop is not None and ne != g.n_ecols):
        raise HpmError(E_PATTERN, f"pattern has {nv} vertex / {ne} arc predicate columns, "
                                  f"graph has {g.n_vcols} / {g.n_ecols}")


def match(g: Graph, p, mode: int, mappings: bool = False, cap: int | None = None, stream=None,
          budget: int | None = None, flags: int = 0, max_matches: int = 0):
    """Count embeddings of pattern p in g; optionally return them.

    Returns (count, rows) where rows is None or an int32 torch tensor [count, k]
    on the current device (original pattern-vertex order, unspecified row
    order).  With mappings=True and cap=None the count is taken first and the
    buffer sized to it (two calls).  max_matches > 0 stops the search once that
    many embeddings are found (first-k): the count is then at most max_matches.
    """
    lib = load()
    _check_columns(g, p)
    s, keep = _pattern_struct(p)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), int(max_matches))
    cnt = ctypes.c_uint64()
    sh = _stream_handle(stream)
    if not mappings:
        _check(lib.hpm_match(g.handle, ctypes.byref(s), int(mode), sh, ctypes.byref(opts),
                             ctypes.byref(cnt), None, 0))
        return int(cnt.value), None
    import torch
    if cap is None:
        _check(lib.hpm_match(g.handle, ctypes.byref(s), int(mode), sh, ctypes.byref(opts),
                             ctypes.byref(cnt), None, 0))
        cap = int(cnt.value)
    buf = torch.empty((max(int(cap), 1), int(p.k)), dtype=torch.int32, device="cuda")
    st = lib.hpm_match(g.handle, ctypes.byref(s), int(mode), sh, ctypes.byref(opts),
                       ctypes.byref(cnt), ctypes.c_void_p(buf.data_ptr()), int(cap))
    _check(st)
    return int(cnt.value), buf[: int(cnt.value)]


def match_noalloc(g: Graph, p, mode: int, out=None, stream=None, budget: int | None = None,
                  flags: int = 0, max_matches: int = 0):
    """hpm_match_noalloc: as match(), for callers that cannot allocate device
    memory.  out: None (count only) or a caller-owned int32 device tensor
    [cap, k] that receives the rows.  Returns (count, out[:count] or None);
    the count may exceed cap (then HpmError with E_TRUNCATED is raised)."""
    lib = load()
    _check_columns(g, p)
    s, keep = _pattern_struct(p)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), int(max_matches))
    cnt = ctypes.c_uint64()
    ptr, cap = None, 0
    if out is not None:
        if out.dim() != 2 or out.shape[1] != p.k or not out.is_contiguous():
            raise ValueError("out must be a contiguous [cap, k] int32 device tensor")
        ptr, cap = ctypes.c_void_p(out.data_ptr()), int(out.shape[0])
    _check(lib.hpm_match_noalloc(g.handle, ctypes.byref(s), int(mode), _stream_handle(stream),
                                 ctypes.byref(opts), ctypes.byref(cnt), ptr, cap))
    return int(cnt.value), (out[: int(cnt.value)] if out is not None else None)


def scan_survivors(g: Graph, p, mode: int, stream=None, flags: int = 0):
    """hpm_scan_survivors: the depth-2 rows (image of position 0, image of
    position 1) that pass the validators (deterministic but unspecified
    order), as an int32 [s2, 2] torch tensor on the current device."""
    import torch
    lib = load()
    _check_columns(g, p)
    s, keep = _pattern_struct(p)
    opts = _Opts(ctypes.sizeof(_Opts), flags, 0, 0)
    cnt = ctypes.c_uint64()
    sh = _stream_handle(stream)
    _check(lib.hpm_scan_survivors(g.handle, ctypes.byref(s), int(mode), sh, ctypes.byref(opts),
                                  ctypes.byref(cnt), None, 0))
    buf = torch.empty((max(int(cnt.value), 1), 2), dtype=torch.int32, device="cuda")
    _check(lib.hpm_scan_survivors(g.handle, ctypes.byref(s), int(mode), sh, ctypes.byref(opts),
                                  ctypes.byref(cnt), ctypes.c_void_p(buf.data_ptr()),
                                  int(buf.shape[0])))
    return buf[: int(cnt.value)]


def match_batch(g: Graph, patterns, modes, workers: int = 0, stream=None,
                budget: int | None = None, flags: int = 0, max_matches: int = 0):
    """Counts of many patterns on one graph (hpm_match_batch).

    Returns (counts, statuses) as lists; raises HpmError if any pattern failed
    (its status is in the exception's message).
    """
    lib = load()
    n = len(patterns)
    for p in patterns:
        _check_columns(g, p)
    structs = (_Pattern * max(n, 1))()
    keep = []
    for i, p in enumerate(patterns):
        st, arrs = _pattern_struct(p)
        structs[i] = st
        keep.append(arrs)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    status = np.zeros(max(n, 1), dtype=np.int32)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), int(max_matches))
    _check(lib.hpm_match_batch(g.handle, n, structs, _ptr(md), _stream_handle(stream),
                               ctypes.byref(opts), int(workers), _ptr(counts), _ptr(status)))
    return [int(c) for c in counts[:n]], [int(x) for x in status[:n]]


def batch_tune(g: Graph, patterns, modes, stream=None, budget: int | None = None,
               flags: int = 0, max_matches: int = 0):
    """Fastest worker count for match_batch on this batch (hpm_batch_tune):
    returns (workers, milliseconds)."""
    lib = load()
    n = len(patterns)
    for p in patterns:
        _check_columns(g, p)
    structs = (_Pattern * max(n, 1))()
    keep = []
    for i, p in enumerate(patterns):
        st, arrs = _pattern_struct(p)
        structs[i] = st
        keep.append(arrs)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), int(max_matches))
    w, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib.hpm_batch_tune(g.handle, n, structs, _ptr(md), _stream_handle(stream),
                              ctypes.byref(opts), ctypes.byref(w), ctypes.byref(ms)))
    return int(w.value), float(ms.value)


def _batch_structs(g, patterns):
    for p in patterns:
        _check_columns(g, p)
    structs = (_Pattern * max(len(patterns), 1))()
    keep = []
    for i, p in enumerate(patterns):
        st, arrs = _pattern_struct(p)
        structs[i] = st
        keep.append(arrs)
    return structs, keep


def _config(cfg):
    if cfg is None:
        return None
    c = _BatchConfig(ctypes.sizeof(_BatchConfig), int(cfg.get("items_per_lane", 0)),
                     int(cfg.get("chunk_rows", 0)), int(cfg.get("strategy", X_MAPPED)),
                     int(cfg.get("task_work", 0)), int(cfg.get("blocks_per_cu", 0)),
                     int(cfg.get("idle_us", 0)))
    return ctypes.byref(c), c


def match_batch_persistent(g: Graph, patterns, modes, config=None, stream=None,
                           budget: int | None = None, flags: int = 0, max_matches: int = 0):
    """Counts of many patterns in one persistent launch (hpm_match_batch_persistent).

    config: None or a dict with any of items_per_lane, chunk_rows, strategy,
    task_work, blocks_per_cu, idle_us.  Returns (counts, statuses); raises HpmError if
    any pattern failed.
    """
    lib = load()
    n = len(patterns)
    structs, keep = _batch_structs(g, patterns)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    status = np.zeros(max(n, 1), dtype=np.int32)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), int(max_matches))
    cfg = _config(config)
    _check(lib.hpm_match_batch_persistent(g.handle, n, structs, _ptr(md), _stream_handle(stream),
                                          ctypes.byref(opts), cfg[0] if cfg else None,
                                          _ptr(counts), _ptr(status)))
    return [int(c) for c in counts[:n]], [int(x) for x in status[:n]]


def batch_autotune(g: Graph, patterns, modes, stream=None, budget: int | None = None,
                   flags: int = 0):
    """Fastest persistent-launch configuration for this batch (hpm_batch_autotune):
    returns (config dict, milliseconds)."""
    lib = load()
    n = len(patterns)
    structs, keep = _batch_structs(g, patterns)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    opts = _Opts(ctypes.sizeof(_Opts), flags, int(budget or 0), 0)
    best = _BatchConfig(ctypes.sizeof(_BatchConfig), 0, 0, 0, 0, 0, 0)
    ms = ctypes.c_double()
    _check(lib.hpm_batch_autotune(g.handle, n, structs, _ptr(md), _stream_handle(stream),
                                  ctypes.byref(opts), ctypes.byref(best), ctypes.byref(ms)))
    return ({"items_per_lane": best.items_per_lane, "chunk_rows": best.chunk_rows,
             "strategy": best.strategy, "task_work": best.task_work,
             "blocks_per_cu": best.blocks_per_cu}, float(ms.value))


def last_batch_stats() -> dict:
    """Statistics of this thread's last match_batch_persistent call."""
    lib = load()
    st = _BatchStats()
    _check(lib.hpm_last_batch_stats(ctypes.byref(st)))
    return {"error_bits": st.error_bits, "launches": st.launches, "tasks_scan": st.tasks[2],
            "tasks_expand": st.tasks[3], "queue_slots": st.queue_slots,
            "arena_bytes": st.arena_bytes, "scratch_bytes": st.scratch_bytes,
            "fixed_bytes": st.fixed_bytes, "arena_capacity": st.arena_capacity, "grid": st.grid,
            "fallback_patterns": st.fallback_patterns, "kernel_ms": st.kernel_ms,
            "ms_total": st.ms_total}


class Server:
    """A resident graph answering queued queries (hpm_server_*).

    submit() returns a ticket at once; poll(ticket) returns None while the
    query runs (or blocks with wait=True) and then a dict with count, status,
    queue_ms, run_ms, est_bytes and granted_bytes.  Mapping buffers passed to
    submit are torch int32 device tensors [cap, k] kept alive until polled.
    """

    def __init__(self, g: Graph, workers: int = 0, budget: int | None = None, flags: int = 0):
        lib = load()
        opts = _ServerOpts(ctypes.sizeof(_ServerOpts), int(workers), int(budget or 0), flags)
        h = ctypes.c_void_p()
        _check(lib.hpm_server_create(ctypes.byref(h), g.handle, ctypes.byref(opts)))
        self._h = h
        self._g = g
        self._bufs = {}

    def submit(self, p, mode: int, mappings=None) -> int:
        _check_columns(self._g, p)
        s, keep = _pattern_struct(p)
        t = ctypes.c_uint64()
        ptr, cap = (None, 0) if mappings is None else (ctypes.c_void_p(mappings.data_ptr()),
                                                       int(mappings.shape[0]))
        _check(load().hpm_server_submit(self._h, ctypes.byref(s), int(mode), ptr, cap,
                                        ctypes.byref(t)))
        if mappings is not None:
            self._bufs[t.value] = mappings
        return int(t.value)

    def poll(self, ticket: int, wait: bool = False):
        r = _QueryResult()
        st = load().hpm_server_poll(self._h, int(ticket), int(bool(wait)), ctypes.byref(r))
        if st == PENDING:
            return None
        _check(st)
        buf = self._bufs.pop(int(ticket), None)
        out = {"status": r.status, "count": int(r.count), "queue_ms": r.queue_ms,
               "run_ms": r.run_ms, "est_bytes": int(r.est_bytes),
               "granted_bytes": int(r.granted_bytes)}
        if r.status not in (OK, E_TRUNCATED):
            out["error"] = load().hpm_last_error().decode()
        if buf is not None and r.status == OK:
            out["rows"] = buf[: int(r.count)]
        return out

    def stats(self) -> dict:
        s = _ServerStats()
        _check(load().hpm_server_read_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _ServerStats._fields_ if name != "struct_size"}

    def close(self):
        if getattr(self, "_h", None):
            load().hpm_server_destroy(self._h)
            self._h = None
            self._bufs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_stats() -> dict:
    """Statistics of this thread's most recent successful match."""
    s = _Stats()
    _check(load().hpm_last_stats(ctypes.byref(s)))
    return {
        "count": s.count, "arcs_scanned": s.arcs_scanned, "survivors": s.survivors,
        "rows": list(s.rows), "work": list(s.work), "chunks": s.chunks,
        "scratch_bytes": s.scratch_bytes,
        "kernel_launches": dict(zip(KERNELS, list(s.kernel_launches))),
        "kernel_ms": dict(zip(KERNELS, list(s.kernel_ms))), "ms_total": s.ms_total,
        "filtered_lists": s.filtered_lists, "raw_work": list(s.raw_work),
        "overlap_removed": s.overlap_removed,
        "counted_rows": s.counted_rows, "counted_work": s.counted_work,
        "filter_rows": s.filter_rows, "filter_entries": s.filter_entries,
        "filter_pieces": s.filter_pieces, "lookahead_removed": s.lookahead_removed,
        "index_arcs": s.index_arcs,
    }


def status_string(status: int) -> str:
    return load().hpm_status_string(status).decode()


def abi_version() -> int:
    return load().hpm_abi_version()
