"""The CPU oracle pinned to things other than itself (CPU only).

Pins: a hand-worked example (tests/golden), brute force over all injective
maps, the trace formula for labelled 3-cycles, Moon's formula for tournaments,
falling factorials on complete digraphs, out-star and 2-path closed forms,
mono = sum of iso over supergraphs, automorphism divisibility, and relabelling
invariances.
"""
import math

import numpy as np
import pytest

import oracle
from synth.graphs import erdos_renyi, permute_vertices, rmat
from synth.patterns import EQ, GE, ISO, MONO, make_pattern, motif, relabel_pattern
from tests import pins
from tests.cases import (complete_digraph, load_hand_example, random_small_graph,
                         random_small_pattern, random_tournament)


def test_hand_example():
    g, cases = load_hand_example()
    for name, p, mode, rows in cases:
        r = oracle.match(g, p, mode)
        assert r.count == rows.shape[0], name
        np.testing.assert_array_equal(r.rows, rows, err_msg=name)
        np.testing.assert_array_equal(pins.brute(g, p, mode), rows, err_msg=name)


@pytest.mark.parametrize("seed", range(240))
def test_oracle_equals_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 8))
    nv = int(rng.integers(1, 3))
    ne = int(rng.integers(1, 3))
    g = random_small_graph(rng, n, float(rng.uniform(0.2, 0.8)), nv, ne)
    k = int(rng.integers(1, min(n, 4) + 1))
    p = random_small_pattern(rng, k, nv, ne, connected=(seed % 5 != 0))
    for mode in (ISO, MONO):
        want = pins.brute(g, p, mode)
        got = oracle.match(g, p, mode, threads=1 + seed % 3)
        assert got.count == want.shape[0]
        np.testing.assert_array_equal(got.rows, want)
        assert got.fingerprint == oracle.fingerprint(want)


def _c1_like(m, seed):
    return erdos_renyi(1000, m, seed)


@pytest.mark.parametrize("m,seed", [(5000, 101), (50000, 102), (20000, 7)])
def test_trace_formula_labelled_cycle3(m, seed):
    g = _c1_like(m, seed)
    for vlab in [(0, 1, 2), (1, 1, 1), (3, 0, 2)]:
        for elab in (0, 1):
            p = motif("cycle3", vlabels=vlab, elabels=[elab] * 3)
            for mode in (ISO, MONO):
                want = pins.trace_cycle3(g, vlab, elab, mode)
                got = oracle.match(g, p, mode, threads=4, rows=False)
                assert got.count == want, (vlab, elab, mode)


def test_trace_formula_unlabelled_companion():
    g = _c1_like(5000, 101)
    g.vcols = [np.zeros(g.n, np.int32)]
    g.ecols = [np.zeros(g.m, np.int32)]
    p = motif("cycle3", vlabels=[0, 0, 0], elabels=[0, 0, 0])
    for mode in (ISO, MONO):
        assert oracle.match(g, p, mode, rows=False).count == pins.trace_cycle3(g, (0, 0, 0), 0, mode)


@pytest.mark.parametrize("seed", range(6))
def test_moon_formula_tournaments(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    t = random_tournament(rng, n)
    p = motif("cycle3")
    got = oracle.match(t, p, ISO, rows=False).count
    assert got == pins.moon_cycle3(np.diff(t.out_off))
    # in a tournament every triple carries arcs both ways round, so mono = iso for the cycle
    assert oracle.match(t, p, MONO, rows=False).count == got


@pytest.mark.parametrize("n", [5, 7, 9, 11])
def test_regular_tournament(n):
    t = random_tournament(None, n, regular=True)
    assert oracle.match(t, motif("cycle3"), ISO, rows=False).count == n * (n * n - 1) // 8


@pytest.mark.parametrize("seed", range(12))
def test_complete_digraph_falling_factorial(seed):
    rng = np.random.default_rng(50 + seed)
    n = 7
    g = complete_digraph(n)
    k = int(rng.integers(2, 5))
    p = random_small_pattern(rng, k, 1, 1, p_pred=0.0)
    complete = p.n_arcs == k * (k - 1)
    assert oracle.match(g, p, MONO, rows=False).count == pins.falling(n, k)
    assert oracle.match(g, p, ISO, rows=False).count == (pins.falling(n, k) if complete else 0)


def _star(k_leaves, centre_lab, leaf_lab, arc_op, arc_val):
    arcs = [(0, i) for i in range(1, k_leaves + 1)]
    vpred = [[(EQ, centre_lab)]] + [[(EQ, leaf_lab)]] * k_leaves
    epred = [[(arc_op, arc_val)]] * k_leaves
    return make_pattern(k_leaves + 1, arcs, 1, 1, vpred, epred, "star")


@pytest.mark.parametrize("leaves", [2, 3])
def test_out_star_closed_form(leaves):
    g = rmat(12, 1 << 15, seed=5)
    for (cl, ll, op, val) in [(0, 0, EQ, 1), (1, 0, GE, 2), (0, 2, GE, 0)]:
        p = _star(leaves, cl, ll, op, val)
        want = pins.out_star_mono(g, leaves, lambda lab: lab == cl, lambda lab: lab == ll,
                                  (lambda e: e == val) if op == EQ else (lambda e: e >= val))
        assert oracle.match(g, p, MONO, threads=4, rows=False).count == want


def test_two_path_closed_form():
    for g in (rmat(11, 1 << 14, seed=9), erdos_renyi(500, 4000, seed=3)):
        p = make_pattern(3, [(0, 1), (1, 2)], 1, 1)
        assert oracle.match(g, p, MONO, threads=4, rows=False).count == pins.two_path_mono(g)


def test_single_arc_counts():
    g = erdos_renyi(300, 3000, seed=11)
    A = pins.dense_adj(g)
    E = pins.dense_ecol(g)
    lab = np.asarray(g.vcols[0])
    for (l0, l1, el) in [(0, 1, 0), (2, 2, 1), (3, 0, 1)]:
        p = make_pattern(2, [(0, 1)], 1, 1, [[(EQ, l0)], [(EQ, l1)]], [[(EQ, el)]])
        base = A * (E == el) * np.outer(lab == l0, lab == l1)
        assert oracle.match(g, p, MONO, rows=False).count == int(base.sum())
        assert oracle.match(g, p, ISO, rows=False).count == int((base * (1 - A.T)).sum())
        pr = make_pattern(2, [(0, 1), (1, 0)], 1, 1, [[(EQ, l0)], [(EQ, l1)]],
                          [[(EQ, el)], [(GE, 1)]])
        want = A * (E == el) * (A.T * (E.T >= 1)) * np.outer(lab == l0, lab == l1)
        for mode in (ISO, MONO):
            assert oracle.match(g, pr, mode, rows=False).count == int(want.sum())


@pytest.mark.parametrize("seed", range(4))
def test_mono_is_sum_of_iso_over_supergraphs(seed):
    rng = np.random.default_rng(300 + seed)
    g = random_small_graph(rng, 24, 0.25, 1, 1, nlab=2, nelab=2)
    k = 3 if seed < 2 else 4
    p = random_small_pattern(rng, k, 1, 1, p_arc=0.4)
    mono = oracle.match(g, p, MONO, rows=False).count
    total = 0
    pa = p.arcs()
    for arcs in pins.all_supergraphs(k, pa):
        epred = [[(int(p.eop[pa.index(a), 0]), int(p.eval[pa.index(a), 0]))] if a in pa
                 else [None] for a in arcs]
        vpred = [[(int(p.vop[v, 0]), int(p.vval[v, 0]))] for v in range(k)]
        q = make_pattern(k, arcs, 1, 1, vpred, epred)
        total += oracle.match(g, q, ISO, rows=False).count
    assert mono == total


def test_automorphism_divisibility():
    g = rmat(11, 1 << 14, seed=13)
    g.vcols = [np.zeros(g.n, np.int32)]
    g.ecols = [np.zeros(g.m, np.int32)]
    for name, aut in [("cycle3", 3), ("cycle4", 4)]:
        p = motif(name)
        for mode in (ISO, MONO):
            c = oracle.match(g, p, mode, threads=4, rows=False).count
            assert c > 0 and c % aut == 0


def test_relabelling_invariance():
    rng = np.random.default_rng(77)
    g = random_small_graph(rng, 60, 0.08, 1, 1, nlab=3, nelab=2)
    p = random_small_pattern(rng, 4, 1, 1, nlab=3, p_arc=0.35, p_pred=0.4)
    perm = rng.permutation(g.n)
    gp = permute_vertices(g, perm)
    qperm = rng.permutation(p.k)
    pq = relabel_pattern(p, qperm)
    for mode in (ISO, MONO):
        base = oracle.match(g, p, mode)
        moved = oracle.match(gp, p, mode)
        np.testing.assert_array_equal(oracle.sort_rows(perm[base.rows]), moved.rows)
        # permuting pattern ids permutes the columns of every row
        pr = oracle.match(g, pq, mode)
        cols = np.empty_like(base.rows)
        cols[:, qperm] = base.rows
        np.testing.assert_array_equal(oracle.sort_rows(cols), pr.rows)


def test_root_slices_partition_the_result():
    g = rmat(10, 1 << 13, seed=21)
    p = motif("ffl_tail", vlabels=[0, 0, 1, 0], elabels=[0, 1, 2, 0])
    for mode in (ISO, MONO):
        full = oracle.match(g, p, mode, threads=3)
        rng = np.random.default_rng(4)
        part = rng.integers(0, 3, size=g.n)
        got = []
        for s in range(3):
            r = oracle.match(g, p, mode, root_mask=(part == s), threads=2)
            assert np.all(part[r.rows[:, 0]] == s)
            got.append(r.rows)
        np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(got)), full.rows)


def test_fingerprint_is_order_independent():
    rng = np.random.default_rng(5)
    rows = rng.integers(0, 1000, size=(500, 4)).astype(np.int32)
    fp = oracle.fingerprint(rows)
    assert fp == oracle.fingerprint(rows[rng.permutation(500)])
    rows2 = rows.copy()
    rows2[17, 2] += 1
    assert fp != oracle.fingerprint(rows2)
    rows3 = rows[:, [1, 0, 2, 3]]
    assert fp != oracle.fingerprint(rows3)


@pytest.mark.parametrize("n,k,threads", [(7, 4, 1), (9, 3, 3), (6, 5, 2)])
def test_search_bound_on_complete_digraph(n, k, threads):
    """In a complete digraph every vertex has n-1 out- and in-neighbours and
    every injective partial map of a connected pattern is feasible under
    monomorphism, so the search tests n roots plus n-1 candidates under each of
    the n!/(n-d)! maps at depths 1..k-1; a bound one below that total stops
    it, the exact total does not."""
    g = complete_digraph(n)
    p = make_pattern(k, [(i, i + 1) for i in range(k - 1)])
    want = n + (n - 1) * sum(pins.falling(n, d) for d in range(1, k))
    full = oracle.match(g, p, MONO, threads=threads, rows=False)
    assert full.tested == want and full.count == pins.falling(n, k)
    at = oracle.match(g, p, MONO, threads=threads, rows=False, max_tested=want)
    assert not at.capped and at.count == full.count and at.tested == want
    below = oracle.match(g, p, MONO, threads=threads, rows=False, max_tested=want - 1)
    assert below.capped and below.count is None


@pytest.mark.parametrize("seed", range(60))
def test_row_check_equals_brute_force_membership(seed):
    # every injective map (and some maps that repeat a vertex) is flagged
    # exactly when brute-force enumeration lists it
    import itertools
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(2, 7))
    nv, ne = int(rng.integers(1, 3)), int(rng.integers(1, 3))
    g = random_small_graph(rng, n, float(rng.uniform(0.2, 0.8)), nv, ne)
    k = int(rng.integers(1, min(n, 4) + 1))
    p = random_small_pattern(rng, k, nv, ne, connected=(seed % 4 != 0))
    maps = np.array(list(itertools.permutations(range(n), k)), dtype=np.int32).reshape(-1, k)
    if k >= 2:
        rep = maps[: min(len(maps), 8)].copy()
        rep[:, 1] = rep[:, 0]                 # not injective: never an embedding
        maps = np.concatenate([maps, rep])
    for mode in (ISO, MONO):
        want = {tuple(r) for r in pins.brute(g, p, mode)}
        flags = oracle.check_rows(g, p, mode, maps, threads=1 + seed % 3)
        assert [tuple(r) in want for r in maps] == flags.astype(bool).tolist()


def _bipartite_pattern(s, labels, thr):
    from synth.patterns import make_pattern
    k = s + 2
    arcs = [(a, b) for a in range(s) for b in (s, s + 1)]
    vpred = [[None] for _ in range(s)] + [[None if t is None else (EQ, t)] for t in labels]
    return make_pattern(k, arcs, 1, 1, vpred, [[(GE, thr)]] * len(arcs), f"k{s}2")


@pytest.mark.parametrize("seed", range(8))
def test_bipartite_closed_form_on_small_graphs(seed):
    # the sparse-product count of complete bipartite patterns (s sources, two
    # labelled targets) equals brute force on tiny graphs
    rng = np.random.default_rng(77 + seed)
    g = random_small_graph(rng, int(rng.integers(5, 8)), 0.6, 1, 1, nlab=2, nelab=3)
    for s in (1, 2):
        for labels in ((0, 1), (1, 1), (None, 0)):
            p = _bipartite_pattern(s, labels, 1)
            assert pins.bipartite_k2_mono(g, s, labels, 1) == pins.brute(g, p, MONO).shape[0]


def test_bipartite_closed_form_equals_the_oracle_on_a_connectome_graph():
    # the closed form that pins the full connectome bi-fan count, against the
    # oracle on a scaled-down graph of the same generator
    from synth import configs
    g = configs.c3_graph(n=4_000, m=30_000)
    for s, labels, thr in ((3, (3, 2), 2), (3, (None, 5), 6), (2, (1, 1), 3)):
        p = _bipartite_pattern(s, labels, thr)
        want = pins.bipartite_k2_mono(g, s, labels, thr)
        got = oracle.match(g, p, MONO, threads=4, rows=False).count
        assert got == want and want > 0, (s, labels, thr)
