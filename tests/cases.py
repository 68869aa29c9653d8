"""Seeded test inputs shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import json
import os

import numpy as np

from synth.graphs import from_dense, graph_from_arcs
from synth.patterns import ANY, EQ, GE, Pattern, make_pattern

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def random_small_graph(rng, n, p, nv=1, ne=1, nlab=2, nelab=2):
    A = (rng.random((n, n)) < p).astype(np.int64)
    np.fill_diagonal(A, 0)
    vcols = [rng.integers(0, nlab, size=n) for _ in range(nv)]
    ecols = [rng.integers(0, nelab, size=(n, n)) for _ in range(ne)]
    return from_dense(A, vcols, ecols)


def random_small_pattern(rng, k, nv=1, ne=1, nlab=2, nelab=2, connected=True, p_arc=0.45,
                         p_pred=0.5):
    """Random pattern with random arcs (weakly connected unless connected=False)
    and random {ANY, EQ, GE} predicates."""
    while True:
        arcs = [(a, b) for a in range(k) for b in range(k) if a != b and rng.random() < p_arc]
        if not arcs and k > 1:
            continue
        if connected and k > 1:
            from synth.patterns import is_weakly_connected
            if not is_weakly_connected(k, arcs):
                continue
        break

    def pred(nvals):
        if rng.random() >= p_pred:
            return None
        op = int(rng.choice([EQ, GE]))
        return (op, int(rng.integers(0, nvals)))

    vpred = [[pred(nlab) for _ in range(nv)] for _ in range(k)]
    epred = [[pred(nelab) for _ in range(ne)] for _ in arcs]
    return make_pattern(k, arcs, nv, ne, vpred, epred, f"r{k}")


def load_hand_example():
    with open(os.path.join(GOLDEN, "hand_example.json")) as f:
        doc = json.load(f)
    gd = doc["graph"]
    arcs = np.array(gd["arcs"])
    order = np.lexsort((arcs[:, 1], arcs[:, 0]))
    g = graph_from_arcs(gd["n"], arcs[:, 0], arcs[:, 1], [np.array(gd["vertex_label"])])
    g.ecols = [np.ascontiguousarray(np.array(gd["arc_label"])[order], dtype=np.int32)]
    cases = []
    for c in doc["cases"]:
        vpred = None if c["vpred"] is None else [[tuple(x)] for x in c["vpred"]]
        epred = None if c["epred"] is None else [[tuple(x)] for x in c["epred"]]
        p = make_pattern(c["k"], [tuple(a) for a in c["arcs"]], 1, 1, vpred, epred, c["name"])
        mode = 0 if c["mode"] == "iso" else 1
        cases.append((c["name"], p, mode, np.array(c["rows"], dtype=np.int32).reshape(-1, c["k"])))
    return g, cases


def complete_digraph(n, label=0):
    A = np.ones((n, n), dtype=np.int64)
    np.fill_diagonal(A, 0)
    return from_dense(A, [np.full(n, label)], [np.zeros((n, n), dtype=np.int64)])


def random_tournament(rng, n, regular=False):
    A = np.zeros((n, n), dtype=np.int64)
    if regular:
        # rotational tournament on odd n: i -> i+1..i+(n-1)/2 (mod n)
        for i in range(n):
            for s in range(1, (n - 1) // 2 + 1):
                A[i, (i + s) % n] = 1
    else:
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < 0.5:
                    A[i, j] = 1
                else:
                    A[j, i] = 1
    return from_dense(A, [np.zeros(n, dtype=np.int64)], [np.zeros((n, n), dtype=np.int64)])
