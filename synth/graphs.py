"""Seeded synthetic property graphs (directed, simple, no self-loops).

This module only draws random inputs and lays them out as CSR; it holds none
of the matching arithmetic, so both the CPU oracle and the HIP path can be fed
from it.  Every generator is a pure function of its arguments: the same seed
gives byte-identical arrays (checked by sha256 in the tests).

Families follow the paper's experimental section (Sec. IV-A, "Synthetic Graph
Generation"): Erdos-Renyi graphs with uniformly assigned attributes, plus two
skewed families standing in for the scale-free and connectome datasets
(Sec. IV-D/IV-G): R-MAT and a directed Chung-Lu graph with power-law in/out
weights and a fixed fraction of reciprocal arcs.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import numpy as np


@dataclass
class HostGraph:
    """A directed graph as out-CSR + in-CSR with SoA int32 attribute columns.

    out_off int64[n+1], out_nbrs int32[m]: row u lists the heads of u's out-arcs,
    strictly ascending.  in_off/in_nbrs: the transpose.  vcols: list of int32[n].
    ecols: list of int32[m] in out-CSR arc order (arc id e = position in out_nbrs).
    """
    n: int
    m: int
    out_off: np.ndarray
    out_nbrs: np.ndarray
    in_off: np.ndarray
    in_nbrs: np.ndarray
    vcols: list = field(default_factory=list)
    ecols: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    def src(self) -> np.ndarray:
        """Tail of every arc, in out-CSR order (int32[m])."""
        deg = np.diff(self.out_off)
        return np.repeat(np.arange(self.n, dtype=np.int32), deg)

    def arrays(self):
        out = {"out_off": self.out_off, "out_nbrs": self.out_nbrs,
               "in_off": self.in_off, "in_nbrs": self.in_nbrs}
        for i, c in enumerate(self.vcols):
            out[f"vcol{i}"] = c
        for i, c in enumerate(self.ecols):
            out[f"ecol{i}"] = c
        return out

    def sha256(self) -> dict:
        return {k: hashlib.sha256(np.ascontiguousarray(v).tobytes()).hexdigest()
                for k, v in self.arrays().items()}


def _first_unique(keys: np.ndarray) -> np.ndarray:
    """Distinct values of `keys` in order of first occurrence."""
    _, idx = np.unique(keys, return_index=True)
    idx.sort()
    return keys[idx]


def csr_from_keys(n: int, keys: np.ndarray) -> tuple:
    """Build out- and in-CSR from distinct arc keys src*n+dst (any order)."""
    keys = np.sort(keys.astype(np.int64, copy=False))
    src = keys // n
    dst = keys - src * n
    m = keys.shape[0]
    out_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=out_off[1:])
    out_nbrs = dst.astype(np.int32)
    del keys
    tkeys = np.sort(dst * n + src)
    del src, dst
    t_src = tkeys // n                       # head of the arc (row of the in-CSR)
    in_nbrs = (tkeys - t_src * n).astype(np.int32)
    in_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(t_src, minlength=n), out=in_off[1:])
    assert out_off[-1] == m and in_off[-1] == m
    return out_off, out_nbrs, in_off, in_nbrs


def graph_from_arcs(n, src, dst, vcols=(), ecol_fn=None, meta=None) -> HostGraph:
    """CSR graph from parallel arc arrays (must be distinct, no self-loops).

    ecol_fn(m) -> list of int32[m] arrays, drawn in out-CSR order.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keys = src * n + dst
    out_off, out_nbrs, in_off, in_nbrs = csr_from_keys(n, keys)
    m = out_nbrs.shape[0]
    ecols = list(ecol_fn(m)) if ecol_fn is not None else []
    return HostGraph(n, m, out_off, out_nbrs, in_off, in_nbrs,
                     [np.ascontiguousarray(c, dtype=np.int32) for c in vcols],
                     [np.ascontiguousarray(c, dtype=np.int32) for c in ecols],
                     dict(meta or {}))


# ---------------------------------------------------------------- label draws

def zipf_probs(s: float, nvals: int) -> np.ndarray:
    """P(i) proportional to (i+1)^-s on 0..nvals-1."""
    w = np.arange(1, nvals + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def draw_labels(rng, size, dist) -> np.ndarray:
    """dist: ("uniform", nvals) | ("zipf", s, nvals) | ("lognormal_int", mu, sigma)."""
    kind = dist[0]
    if kind == "uniform":
        return rng.integers(0, dist[1], size=size, dtype=np.int32)
    if kind == "zipf":
        p = zipf_probs(dist[1], dist[2])
        return rng.choice(dist[2], size=size, p=p).astype(np.int32)
    if kind == "lognormal_int":
        z = rng.standard_normal(size)
        return (1 + np.floor(np.exp(dist[1] + dist[2] * z))).astype(np.int32)
    raise ValueError(dist)


# ---------------------------------------------------------------- families

def erdos_renyi(n: int, m: int, seed: int, vlabels=("uniform", 4),
                elabels=("uniform", 2), batch: int | None = None) -> HostGraph:
    """Directed G(n, m): m distinct ordered pairs (u, v), u != v, uniform.

    Pairs are drawn in batches; self-loops are dropped and the first m distinct
    pairs in draw order are kept.
    """
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of ordered pairs")
    rng = np.random.default_rng(seed)
    batch = batch or max(2 * m, 1024)
    pool = np.empty(0, dtype=np.int64)
    while True:
        u = rng.integers(0, n, size=batch, dtype=np.int64)
        v = rng.integers(0, n, size=batch, dtype=np.int64)
        keep = u != v
        pool = _first_unique(np.concatenate([pool, u[keep] * n + v[keep]]))
        if pool.shape[0] >= m:
            break
    keys = pool[:m]
    vl = draw_labels(rng, n, vlabels)
    g = graph_from_arcs(n, keys // n, keys % n, [vl],
                        lambda mm: [draw_labels(rng, mm, elabels)],
                        meta={"family": "er", "n": n, "m": m, "seed": seed})
    return g


def rmat(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19,
         vlabels=("zipf", 1.2, 16), elabels=("uniform", 4),
         batch: int = 1 << 22, permute: bool = True) -> HostGraph:
    """R-MAT (Chakrabarti et al. 2004) with quadrant probabilities a, b, c, d=1-a-b-c.

    Each arc descends `scale` levels, choosing a quadrant per level.  Self-loops
    and repeats are dropped; the first m distinct arcs in draw order are kept;
    vertex ids are then relabelled by a seeded random permutation.
    """
    n = 1 << scale
    rng = np.random.default_rng(seed)
    pool = np.empty(0, dtype=np.int64)
    t1, t2, t3 = a, a + b, a + b + c
    while pool.shape[0] < m:
        src = np.zeros(batch, dtype=np.int64)
        dst = np.zeros(batch, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(batch, dtype=np.float32)
            sbit = r >= t2
            dbit = ((r >= t1) & (r < t2)) | (r >= t3)
            src = (src << 1) | sbit
            dst = (dst << 1) | dbit
        keep = src != dst
        pool = _first_unique(np.concatenate([pool, (src[keep] << scale) | dst[keep]]))
    keys = pool[:m]
    s = keys >> scale
    d = keys & (n - 1)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        s, d = perm[s], perm[d]
    vl = draw_labels(rng, n, vlabels)
    return graph_from_arcs(n, s, d, [vl], lambda mm: [draw_labels(rng, mm, elabels)],
                           meta={"family": "rmat", "scale": scale, "m": m, "seed": seed,
                                 "abcd": [a, b, c, round(1 - a - b - c, 6)]})


def truncated_pareto(rng, size, gamma: float, xmin: float, xmax: float) -> np.ndarray:
    """Weights with density proportional to x^-gamma on [xmin, xmax] (inverse CDF)."""
    al = gamma - 1.0
    u = rng.random(size)
    lo = (xmax / xmin) ** (-al)
    return xmin * (1.0 - u * (1.0 - lo)) ** (-1.0 / al)


_CL_LIB = None


def build_native(force: bool = True) -> str:
    """Compile the Chung-Lu helper (g++ -O3 -fopenmp) into synth/libchunglu.so."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    lib = os.path.join(here, "libchunglu.so")
    if force or not os.path.exists(lib):
        subprocess.run(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o",
                        lib + ".tmp", os.path.join(here, "chung_lu.cpp")], check=True)
        os.replace(lib + ".tmp", lib)
    return lib


def _cl_lib():
    global _CL_LIB
    if _CL_LIB is None:
        import ctypes
        lib = ctypes.CDLL(build_native(force=False))
        P = ctypes.POINTER
        lib.cl_generate.restype = ctypes.c_int64
        lib.cl_generate.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_int32, P(P(ctypes.c_int64)), P(P(ctypes.c_int32)),
                                    P(P(ctypes.c_int64)), P(P(ctypes.c_int32)),
                                    P(P(ctypes.c_int32)), P(P(ctypes.c_int32))]
        lib.cl_free.argtypes = [ctypes.c_void_p]
        _CL_LIB = lib
    return _CL_LIB


def connectome(n: int, m: int, seed: int, gamma: float = 2.1, xmax: float = 50_000,
               recip: float = 0.30, nlab: int = 8, mu: float = 1.0, sigma: float = 1.0,
               threads: int = 0) -> HostGraph:
    """Directed Chung-Lu graph with power-law in/out weights and reciprocity.

    Built by synth/chung_lu.cpp (see its header for the recipe): out- and
    in-weights i.i.d. truncated Pareto(gamma, 1, xmax); Poisson arc draws per
    tail, heads proportional to w_in; self-loops and repeats dropped; reverse
    arcs added so that a `recip` fraction of arcs is reciprocal; vertex labels
    U{0..nlab-1}; arc weight 1 + floor(exp(mu + sigma Z)).  About m arcs.
    Counter-based random streams: the output does not depend on `threads`.
    """
    import ctypes
    lib = _cl_lib()
    P64, P32 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    oo, on, io, inn, vl, ew = P64(), P32(), P64(), P32(), P32(), P32()
    M = lib.cl_generate(n, m, gamma, xmax, recip, nlab, mu, sigma, seed, threads,
                        ctypes.byref(oo), ctypes.byref(on), ctypes.byref(io), ctypes.byref(inn),
                        ctypes.byref(vl), ctypes.byref(ew))
    if M < 0:
        raise ValueError("bad Chung-Lu parameters")

    def take(ptr, count, dtype):
        arr = np.ctypeslib.as_array(ptr, shape=(max(count, 1),))[:count].astype(dtype, copy=True)
        lib.cl_free(ctypes.cast(ptr, ctypes.c_void_p))
        return arr

    out_off = take(oo, n + 1, np.int64)
    out_nbrs = take(on, M, np.int32)
    in_off = take(io, n + 1, np.int64)
    in_nbrs = take(inn, M, np.int32)
    vlab = take(vl, n, np.int32)
    wts = take(ew, M, np.int32)
    return HostGraph(n, int(M), out_off, out_nbrs, in_off, in_nbrs, [vlab], [wts],
                     {"family": "chung_lu", "n": n, "m_target": m, "m": int(M), "seed": seed,
                      "gamma": gamma, "xmax": xmax, "recip": recip})


def reciprocal_fraction(g: HostGraph) -> float:
    """Fraction of arcs (u,v) whose reverse (v,u) is also an arc."""
    n = g.n
    src = g.src().astype(np.int64)
    keys = src * n + g.out_nbrs
    rev = g.out_nbrs.astype(np.int64) * n + src
    pos = np.searchsorted(keys, rev)           # keys are sorted (CSR order)
    pos[pos >= keys.shape[0]] = 0
    return float((keys[pos] == rev).mean()) if g.m else 0.0


def permute_vertices(g: HostGraph, perm: np.ndarray) -> HostGraph:
    """Relabel vertex v as perm[v]; attributes travel with their vertex/arc."""
    n = g.n
    src = g.src().astype(np.int64)
    dst = g.out_nbrs.astype(np.int64)
    ns, nd = perm[src].astype(np.int64), perm[dst].astype(np.int64)
    order = np.argsort(ns * n + nd, kind="stable")
    vcols = []
    for c in g.vcols:
        nc = np.empty_like(c)
        nc[perm] = c
        vcols.append(nc)
    ecols = [c[order] for c in g.ecols]
    out = graph_from_arcs(n, ns, nd, vcols, None, meta=dict(g.meta, permuted=True))
    out.ecols = [np.ascontiguousarray(c, dtype=np.int32) for c in ecols]
    return out


def from_dense(adj: np.ndarray, vcols=(), ecols_dense=()) -> HostGraph:
    """Graph from a dense 0/1 adjacency matrix (diagonal must be zero).

    ecols_dense: int matrices giving the attribute of arc (u,v) at [u,v].
    """
    adj = np.asarray(adj)
    n = adj.shape[0]
    assert not np.any(np.diag(adj)), "self-loops"
    u, v = np.nonzero(adj)                       # row-major: out-CSR order
    g = graph_from_arcs(n, u, v, vcols, None, meta={"family": "dense"})
    g.ecols = [np.ascontiguousarray(np.asarray(e)[u, v], dtype=np.int32) for e in ecols_dense]
    return g
