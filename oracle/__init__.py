"""CPU oracle for edge-centric subgraph matching -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The library under paper_2507_04130_amd/ never imports it, and
the two share no code.

`match()` returns every embedding of a pattern in a target graph by plain
backtracking from the empty mapping (the problem definition of Sec. II-A,
Eq. (1)-(3), with the monomorphism relaxation); see hpm_oracle.cpp.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hpm_oracle.cpp")
# HPM_ORACLE_LIB: load another build of the same source (the sanitizer test's)
_LIB = os.environ.get("HPM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O3 -fopenmp into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("fp1", ctypes.c_uint64),
                ("fp2", ctypes.c_uint64), ("rows", ctypes.POINTER(ctypes.c_int32))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.og_match.restype = ctypes.c_int
    lib.og_match.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, ctypes.c_int32, P,
                             ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P,
                             ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Result)]
    lib.og_check_rows.restype = ctypes.c_int64
    lib.og_check_rows.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, ctypes.c_int32, P,
                                  ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, P, P, P, P,
                                  P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_uint64, P]
    lib.og_free.argtypes = [P]
    lib.og_sort_rows.argtypes = [P, ctypes.c_uint64, ctypes.c_int32]
    lib.og_fingerprint.argtypes = [P, ctypes.c_uint64, ctypes.c_int32, P]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleResult:
    def __init__(self, count, fp, rows, seconds, threads, tested=0, capped=False):
        self.count = count
        self.tested = tested      # candidate images tested (all depths, roots included)
        self.capped = capped      # the max_tested bound was passed: count is None
        self.fingerprint = fp
        self.rows = rows
        self.seconds = seconds
        self.threads = threads


def match(g, p, mode: int, threads: int = 1, rows: bool = True, root_mask=None,
          max_tested: int = 0) -> OracleResult:
    """All embeddings of pattern p in graph g (mode 0 = induced iso, 1 = mono).

    g: synth.graphs.HostGraph; p: synth.patterns.Pattern.  rows=True returns the
    sorted int32 [count, k] array (original pattern ids).  root_mask: optional
    uint8[n]; only embeddings with f(0) in the mask are enumerated.
    max_tested: if nonzero, the search stops once it has tested more candidate
    images than this; the result then has capped=True and count None.
    """
    lib = _load()
    out_off = np.ascontiguousarray(g.out_off, dtype=np.int64)
    in_off = np.ascontiguousarray(g.in_off, dtype=np.int64)
    out_nbrs, in_nbrs = _c32(g.out_nbrs), _c32(g.in_nbrs)
    nv, ne = len(g.vcols), len(g.ecols)
    vcols = _c32(np.stack(g.vcols)) if nv else np.zeros(1, np.int32)
    ecols = _c32(np.stack(g.ecols)) if ne else np.zeros(1, np.int32)
    src, dst = _c32(p.src), _c32(p.dst)
    vop, vval = _c32(p.vop), _c32(p.vval)
    eop, evl = _c32(p.eop), _c32(p.eval)
    if vop.size != p.k * nv or eop.size != p.n_arcs * ne:
        raise ValueError("pattern predicate arrays do not match the graph's column counts")
    mask = None if root_mask is None else np.ascontiguousarray(root_mask, dtype=np.uint8)
    res = _Result()
    tested = ctypes.c_uint64(0)
    t0 = time.perf_counter()
    rc = lib.og_match(g.n, g.m, _p(out_off), _p(out_nbrs), _p(in_off), _p(in_nbrs), nv, _p(vcols),
                      ne, _p(ecols), p.k, p.n_arcs, _p(src), _p(dst), _p(vop), _p(vval), _p(eop),
                      _p(evl), int(mode), int(threads), _p(mask), int(bool(rows)),
                      int(max_tested), ctypes.byref(tested), ctypes.byref(res))
    dt = time.perf_counter() - t0
    nthr = threads if threads > 0 else os.cpu_count()
    if rc == 1:
        return OracleResult(None, None, None, dt, nthr, int(tested.value), True)
    if rc != 0:
        raise RuntimeError(f"og_match failed: {rc}")
    out_rows = None
    if rows:
        cnt = int(res.count)
        buf = np.ctypeslib.as_array(res.rows, shape=(max(cnt, 1) * p.k,)) if cnt else None
        out_rows = (buf[: cnt * p.k].reshape(cnt, p.k).copy() if cnt
                    else np.zeros((0, p.k), dtype=np.int32))
        lib.og_free(ctypes.cast(res.rows, ctypes.c_void_p))
    return OracleResult(int(res.count), (int(res.fp1), int(res.fp2)), out_rows, dt, nthr,
                        int(tested.value))


def check_rows(g, p, mode: int, rows: np.ndarray, threads: int = 1) -> np.ndarray:
    """uint8 flag per row of an int32 [count, k] array (original pattern ids):
    1 when the row is an embedding of p in g under `mode`, 0 otherwise."""
    lib = _load()
    out_off = np.ascontiguousarray(g.out_off, dtype=np.int64)
    in_off = np.ascontiguousarray(g.in_off, dtype=np.int64)
    out_nbrs, in_nbrs = _c32(g.out_nbrs), _c32(g.in_nbrs)
    nv, ne = len(g.vcols), len(g.ecols)
    vcols = _c32(np.stack(g.vcols)) if nv else np.zeros(1, np.int32)
    ecols = _c32(np.stack(g.ecols)) if ne else np.zeros(1, np.int32)
    r = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, p.k)
    ok = np.zeros(r.shape[0], dtype=np.uint8)
    rc = lib.og_check_rows(g.n, g.m, _p(out_off), _p(out_nbrs), _p(in_off), _p(in_nbrs), nv,
                           _p(vcols), ne, _p(ecols), p.k, p.n_arcs, _p(_c32(p.src)),
                           _p(_c32(p.dst)), _p(_c32(p.vop)), _p(_c32(p.vval)), _p(_c32(p.eop)),
                           _p(_c32(p.eval)), int(mode), int(threads), _p(r), r.shape[0], _p(ok))
    if rc < 0:
        raise RuntimeError("og_check_rows failed")
    return ok


def sort_rows(rows: np.ndarray) -> np.ndarray:
    """Lexicographically sorted copy of an int32 [count, k] row array."""
    r = np.ascontiguousarray(rows, dtype=np.int32).copy()
    if r.shape[0]:
        _load().og_sort_rows(_p(r), r.shape[0], r.shape[1])
    return r


def fingerprint(rows: np.ndarray) -> tuple:
    """Order-independent 128-bit fingerprint of a row set (same as match())."""
    r = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros(2, dtype=np.uint64)
    _load().og_fingerprint(_p(r), r.shape[0], r.shape[1] if r.ndim == 2 else 0, _p(out))
    return int(out[0]), int(out[1])
