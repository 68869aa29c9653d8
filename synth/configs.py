"""The five seeded workloads (graphs + patterns) and scaled-down variants.

c1  directed Erdos-Renyi G(n=1000, m=5000), vertex labels U{0..3}, arc labels
    U{0,1}; labelled directed 3-cycle, induced isomorphism.  Companions: c1u
    (same graph, unlabelled pattern) and c1d (m=50,000).
c2  R-MAT scale 20 (a,b,c,d = .57,.19,.19,.05), 2^24 distinct arcs, vertex
    labels Zipf(1.2) over 16 values, arc labels U{0..3}; four 4-vertex motifs
    with labels drawn from the same laws; induced isomorphism and monomorphism.
c3  directed Chung-Lu, n=2e7, about 1.5e8 arcs, power-law weights (gamma 2.1,
    max 5e4), 30% reciprocal arcs, vertex labels U{0..7}, arc weight
    1+floor(exp(1+Z)); three 5-vertex motifs with arc-weight thresholds,
    monomorphism (see C3_SHAPES).
c4  256 random patterns (3..8 vertices) on the c2 graph, mixed modes.
c5  random patterns on the c3 graph arriving as a Poisson stream.

`scale` shrinks the big graphs for tests (R-MAT scale, Chung-Lu n and m).
"""
from __future__ import annotations

import numpy as np

from .graphs import connectome, erdos_renyi, rmat
from .patterns import EQ, GE, ISO, MONO, motif, random_pattern

GRAPH_SEEDS = {"c1": 101, "c1d": 102, "c2": 102, "c3": 103}
PATTERN_SEEDS = {"c2": 201, "c3": 202, "c4": 203, "c5": 204}

C2_MOTIFS = ("cycle4", "ffl_tail", "star3_back", "clique4_minus1")
C3_MOTIFS = ("bifan_plus1", "ff_chain", "recip_triad_plus")
C3_THRESHOLD = 10


def c1_graph():
    return erdos_renyi(1000, 5000, GRAPH_SEEDS["c1"])


def c1d_graph():
    return erdos_renyi(1000, 50_000, GRAPH_SEEDS["c1d"])


def c1_pattern():
    return motif("cycle3", vlabels=[0, 1, 2], elabels=[0, 0, 0], name_suffix="_c1")


def c1u_pattern():
    return motif("cycle3", name_suffix="_c1u")


def c2_graph(scale: int = 20, edge_factor: int = 16):
    return rmat(scale, edge_factor << scale, GRAPH_SEEDS["c2"])


def c2_patterns():
    """Four motifs; vertex labels Zipf(1.2, 16), arc labels U{0..3} (EQ)."""
    rng = np.random.default_rng(PATTERN_SEEDS["c2"])
    w = np.arange(1, 17, dtype=np.float64) ** -1.2
    out = []
    for name in C2_MOTIFS:
        from .patterns import MOTIFS
        k, arcs = MOTIFS[name]
        vl = rng.choice(16, size=k, p=w / w.sum()).tolist()
        el = rng.integers(0, 4, size=len(arcs)).tolist()
        out.append(motif(name, vlabels=vl, elabels=el, name_suffix="_c2"))
    return out


def c2_runs():
    """(pattern, mode) pairs making one c2 step: every motif in both modes."""
    return [(p, m) for p in c2_patterns() for m in (ISO, MONO)]


def c3_graph(n: int = 20_000_000, m: int = 150_000_000):
    return connectome(n, m, GRAPH_SEEDS["c3"])


# Per-motif query shape on the connectome graph: which vertices carry a label
# (drawn U{0..7} from the pattern seed) and the arc-weight threshold.  Chosen
# so every query has a non-trivial result on the 1.5e8-arc graph: the chain and
# reciprocal triad need triangles, which a Chung-Lu graph has few of, so they
# are unlabelled with lower thresholds.
C3_SHAPES = {
    "bifan_plus1": ((3, 4), 10),
    "ff_chain": ((), 4),
    "recip_triad_plus": ((), 6),
}


def c3_patterns():
    """Three 5-vertex motifs, monomorphism; vertex labels EQ, arc weight GE."""
    rng = np.random.default_rng(PATTERN_SEEDS["c3"])
    out = []
    for name in C3_MOTIFS:
        from .patterns import MOTIFS
        k, arcs = MOTIFS[name]
        labelled, thr = C3_SHAPES[name]
        draws = rng.integers(0, 8, size=k).tolist()
        vl = [draws[v] if v in labelled else None for v in range(k)]
        out.append(motif(name, vlabels=vl, elabels=[thr] * len(arcs), eop=GE,
                         name_suffix="_c3"))
    return out


def c4_patterns(count: int = 256):
    rng = np.random.default_rng(PATTERN_SEEDS["c4"])
    out = []
    for i in range(count):
        p = random_pattern(rng, name=f"c4_{i}")
        mode = ISO if rng.random() < 0.5 else MONO
        out.append((p, mode))
    return out
