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


def c4_draws(count: int):
    """The first `count` random pattern draws of the batched workload (pattern
    seed): sizes U{3..8}, spanning tree plus pairs up to density U[tree, 0.6],
    Zipf vertex labels, U{0..3} arc labels, mode iso or mono with p = 1/2."""
    rng = np.random.default_rng(PATTERN_SEEDS["c4"])
    out = []
    for i in range(count):
        p = random_pattern(rng, name=f"c4_{i}")
        mode = ISO if rng.random() < 0.5 else MONO
        out.append((p, mode))
    return out


def _c4_screened():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                        "golden", "batch_patterns_screened.json")
    with open(path) as f:
        return json.load(f)["accepted"]


def c4_patterns(count: int = 256):
    """The batched workload: the draws accepted by the oracle screening stored
    in tests/golden/batch_patterns_screened.json (the search on the full graph
    stays within a fixed bound of partial mappings), in draw order."""
    acc = [a["draw"] for a in _c4_screened()][:count]
    draws = c4_draws(max(acc) + 1)
    return [draws[i] for i in acc]


def c4_expected_counts(count: int = 256):
    """The oracle's embedding counts of c4_patterns(count) on the full graph."""
    return [a["count"] for a in _c4_screened()][:count]


def c5_draws(count: int):
    """Random query draws of the served workload (pattern seed): shapes as the
    batched workload's, vertex labels U{0..7} on every vertex, every arc
    weight >= the connectome threshold, iso or mono with p = 1/2."""
    rng = np.random.default_rng(PATTERN_SEEDS["c5"])
    out = []
    for i in range(count):
        p = random_pattern(rng, vlabels=("uniform", 8), eop=GE, eval_const=C3_THRESHOLD,
                           name=f"c5_{i}")
        mode = ISO if rng.random() < 0.5 else MONO
        out.append((p, mode))
    return out


def _c5_screened():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                        "golden", "serve_patterns_screened.json")
    with open(path) as f:
        return json.load(f)["accepted"]


def c5_pool():
    """The served workload's query pool: draws accepted by the oracle screening
    in tests/golden/serve_patterns_screened.json, with their oracle counts and
    fingerprints on the full connectome graph: [(pattern, mode, count, fp)]."""
    acc = _c5_screened()
    draws = c5_draws(max(a["draw"] for a in acc) + 1)
    return [(draws[a["draw"]][0], draws[a["draw"]][1], a["count"], tuple(a["fingerprint"]))
            for a in acc]


ARRIVAL_SEED = 305


def c5_trace(qps: float, n: int, pool_size: int, seed: int = ARRIVAL_SEED):
    """Poisson arrivals: (arrival time in s from the first, pool index) for n
    queries at rate qps, seeded per rate."""
    rng = np.random.default_rng([seed, int(round(qps * 1000))])
    gaps = rng.exponential(1.0 / qps, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps), rng.integers(0, pool_size, size=n)
