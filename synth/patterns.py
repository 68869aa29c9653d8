"""Pattern (query) graphs: fixed motifs and seeded random patterns.

A pattern has vertices 0..k-1, a list of arcs (src[i] -> dst[i]), and for each
vertex and each arc one predicate per attribute column: (op, value) with op in
{ANY=0, EQ=1, GE=2}.  EQ is the label equality of the problem definition
(Sec. II-A, Eq. (2)-(3)); GE expresses a weight threshold; ANY leaves a column
unconstrained.  This module only describes and draws patterns.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

ANY, EQ, GE = 0, 1, 2
ISO, MONO = 0, 1


@dataclass
class Pattern:
    k: int
    src: np.ndarray            # int32[n_arcs]
    dst: np.ndarray            # int32[n_arcs]
    vop: np.ndarray            # int32[k][n_vcols]
    vval: np.ndarray           # int32[k][n_vcols]
    eop: np.ndarray            # int32[n_arcs][n_ecols]
    eval: np.ndarray           # int32[n_arcs][n_ecols]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_arcs(self) -> int:
        return int(self.src.shape[0])

    def arcs(self):
        return list(zip(self.src.tolist(), self.dst.tolist()))


def make_pattern(k, arcs, n_vcols=1, n_ecols=1, vpred=None, epred=None, name=""):
    """vpred: list (per vertex) of list (per column) of (op, val), or None = ANY.
    epred: list (per arc) of list (per column) of (op, val), or None = ANY."""
    arcs = list(arcs)
    src = np.array([a for a, _ in arcs], dtype=np.int32)
    dst = np.array([b for _, b in arcs], dtype=np.int32)
    vop = np.zeros((k, n_vcols), dtype=np.int32)
    vval = np.zeros((k, n_vcols), dtype=np.int32)
    eop = np.zeros((len(arcs), n_ecols), dtype=np.int32)
    evl = np.zeros((len(arcs), n_ecols), dtype=np.int32)
    if vpred is not None:
        for v, cols in enumerate(vpred):
            for c, pv in enumerate(cols or []):
                if pv is not None:
                    vop[v, c], vval[v, c] = pv
    if epred is not None:
        for i, cols in enumerate(epred):
            for c, pv in enumerate(cols or []):
                if pv is not None:
                    eop[i, c], evl[i, c] = pv
    return Pattern(k, src, dst, vop, vval, eop, evl, name)


def relabel_pattern(p: Pattern, perm) -> Pattern:
    """Vertex v becomes perm[v]; predicates travel with their vertex/arc."""
    perm = np.asarray(perm)
    vop = np.empty_like(p.vop)
    vval = np.empty_like(p.vval)
    vop[perm] = p.vop
    vval[perm] = p.vval
    return Pattern(p.k, perm[p.src].astype(np.int32), perm[p.dst].astype(np.int32),
                   vop, vval, p.eop.copy(), p.eval.copy(), p.name + "_perm")


# Arc lists of the fixed motifs used by the benchmark workloads.
MOTIFS = {
    "cycle3": (3, [(0, 1), (1, 2), (2, 0)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "ffl_tail": (4, [(0, 1), (1, 2), (0, 2), (2, 3)]),
    "star3_back": (4, [(0, 1), (0, 2), (0, 3), (1, 0)]),
    # transitive tournament on 4 vertices (i -> j for i < j) minus the arc 0 -> 3
    "clique4_minus1": (4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]),
    # three sources each pointing at both of two targets, plus nothing else
    "bifan_plus1": (5, [(0, 3), (0, 4), (1, 3), (1, 4), (2, 3), (2, 4)]),
    "ff_chain": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 2), (1, 3), (2, 4)]),
    "recip_triad_plus": (5, [(0, 1), (1, 0), (1, 2), (2, 1), (2, 0), (0, 2), (2, 3), (3, 4)]),
}


def motif(name, vlabels=None, elabels=None, eop=EQ, vop=EQ, name_suffix=""):
    """Motif with per-vertex label predicates (vop, label) and one arc predicate
    (eop, value) per arc; None entries mean ANY."""
    k, arcs = MOTIFS[name]
    vpred = None if vlabels is None else [[None if x is None else (vop, int(x))] for x in vlabels]
    epred = None if elabels is None else [[None if x is None else (eop, int(x))] for x in elabels]
    return make_pattern(k, arcs, 1, 1, vpred, epred, name + name_suffix)


def _zipf_choice(rng, size, s, nvals):
    w = np.arange(1, nvals + 1, dtype=np.float64) ** (-s)
    return rng.choice(nvals, size=size, p=w / w.sum())


def random_pattern(rng, kmin=3, kmax=8, max_density=0.6, p_recip=0.1,
                   vlabels=("zipf", 1.2, 16), elabels=("uniform", 4),
                   eop=EQ, eval_const=None, name=""):
    """Random weakly connected pattern.

    k ~ U{kmin..kmax}; a uniform random spanning tree (Pruefer sequence) with
    random orientation; then random extra unordered pairs until the pair
    density reaches rho ~ U[(k-1)/C(k,2), max_density]; each added pair gets a
    random orientation and is made reciprocal with probability p_recip.
    """
    k = int(rng.integers(kmin, kmax + 1))
    pairs = set()
    if k == 2:
        pairs.add((0, 1))
    else:
        seq = rng.integers(0, k, size=k - 2).tolist()
        degree = [1] * k
        for x in seq:
            degree[x] += 1
        for x in seq:
            leaf = min(i for i in range(k) if degree[i] == 1)
            pairs.add((min(leaf, x), max(leaf, x)))
            degree[leaf] -= 1
            degree[x] -= 1
        u, w = [i for i in range(k) if degree[i] == 1]
        pairs.add((u, w))
    npairs = k * (k - 1) // 2
    rho_lo = (k - 1) / npairs
    rho = rng.uniform(rho_lo, max(rho_lo, max_density))
    target = max(k - 1, int(round(rho * npairs)))
    all_pairs = [p for p in itertools.combinations(range(k), 2) if p not in pairs]
    rng.shuffle(all_pairs)
    arcs = []
    for (a, b) in sorted(pairs):
        arcs.append((a, b) if rng.random() < 0.5 else (b, a))
    for (a, b) in all_pairs[: max(0, target - len(pairs))]:
        if rng.random() < 0.5:
            a, b = b, a
        arcs.append((a, b))
        if rng.random() < p_recip:
            arcs.append((b, a))
    if vlabels[0] == "zipf":
        vl = _zipf_choice(rng, k, vlabels[1], vlabels[2])
    else:
        vl = rng.integers(0, vlabels[1], size=k)
    if eval_const is not None:
        el = [eval_const] * len(arcs)
    elif elabels[0] == "uniform":
        el = rng.integers(0, elabels[1], size=len(arcs)).tolist()
    else:
        raise ValueError(elabels)
    vpred = [[(EQ, int(x))] for x in vl]
    epred = [[(eop, int(x))] for x in el]
    return make_pattern(k, arcs, 1, 1, vpred, epred, name or f"rand{k}")


def is_weakly_connected(k, arcs) -> bool:
    adj = {v: set() for v in range(k)}
    for a, b in arcs:
        adj[a].add(b)
        adj[b].add(a)
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == k
