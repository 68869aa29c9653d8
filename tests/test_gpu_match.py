"""Parity of the HIP matcher with the CPU oracle (GPU; calls through the C ABI).

Counts and sorted mapping sets must be bit-exact.  Inputs are seeded: random
small graphs, the hand-worked example, the ER workload and its companions,
scaled-down R-MAT graphs with the benchmark motifs (several tiles plus a
ragged tail), and invariances (matching order, chunked frontiers, relabelling).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_2507_04130_amd as hpm
from paper_2507_04130_amd import hpm as hb
from synth import configs
from synth.graphs import erdos_renyi, from_dense, graph_from_arcs, permute_vertices, rmat
from synth.patterns import ANY, EQ, GE, ISO, MONO, MOTIFS, make_pattern, motif, random_pattern
from tests import pins
from tests.cases import (load_hand_example, random_small_graph, random_small_pattern)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lexsorted(rows):
    rows = np.asarray(rows)
    if rows.shape[0] == 0:
        return rows.reshape(0, rows.shape[1] if rows.ndim == 2 else 0)
    return rows[np.lexsort(rows.T[::-1])]


def gpu_rows(dg, p, mode, **kw):
    cnt, t = hpm.match(dg, p, mode, mappings=True, **kw)
    rows = t.cpu().numpy() if t is not None else np.zeros((0, p.k), np.int32)
    assert rows.shape == (cnt, p.k)
    return cnt, lexsorted(rows)


def assert_parity(g, dg, p, mode, label="", **kw):
    want = oracle.match(g, p, mode, threads=8)
    cnt, rows = gpu_rows(dg, p, mode, **kw)
    assert cnt == want.count, f"{label}: count {cnt} != oracle {want.count}"
    np.testing.assert_array_equal(rows, want.rows, err_msg=label)
    c2, _ = hpm.match(dg, p, mode, **kw)
    assert c2 == want.count
    return want.count


def test_hand_example():
    g, cases = load_hand_example()
    say("hand example")
    dg = hpm.Graph.from_host(g)
    for name, p, mode, rows in cases:
        cnt, got = gpu_rows(dg, p, mode)
        assert cnt == rows.shape[0], name
        np.testing.assert_array_equal(got, rows, err_msg=name)


@pytest.mark.parametrize("seed", range(60))
def test_random_small_graphs(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(2, 40))
    nv = int(rng.integers(0, 3))
    ne = int(rng.integers(0, 3))
    g = random_small_graph(rng, n, float(rng.uniform(0.05, 0.6)), max(nv, 1), max(ne, 1))
    g.vcols = g.vcols[:nv]
    g.ecols = g.ecols[:ne]
    k = int(rng.integers(2, min(n, 6) + 1)) if n >= 2 else 2
    p = random_small_pattern(rng, k, max(nv, 1), max(ne, 1))
    p.vop, p.vval = p.vop[:, :nv].copy(), p.vval[:, :nv].copy()
    p.eop, p.eval = p.eop[:, :ne].copy(), p.eval[:, :ne].copy()
    say(f"random seed={seed} n={n} m={g.m} k={k} arcs={p.n_arcs} nv={nv} ne={ne}")
    dg = hpm.Graph.from_host(g)
    for mode in (ISO, MONO):
        assert_parity(g, dg, p, mode, f"seed {seed} mode {mode}")


def test_c1_and_companions():
    g = configs.c1_graph()
    dg = hpm.Graph.from_host(g)
    p = configs.c1_pattern()
    say("c1")
    c = assert_parity(g, dg, p, ISO, "c1")
    assert c == pins.trace_cycle3(g, (0, 1, 2), 0, ISO)
    pu = configs.c1u_pattern()
    for mode in (ISO, MONO):
        c = assert_parity(g, dg, pu, mode, "c1u")
        gu = erdos_renyi(1000, 5000, configs.GRAPH_SEEDS["c1"])
        gu.vcols = [np.zeros(g.n, np.int32)]
        gu.ecols = [np.zeros(g.m, np.int32)]
        assert c == pins.trace_cycle3(gu, (0, 0, 0), 0, mode)
    gd = configs.c1d_graph()
    dgd = hpm.Graph.from_host(gd)
    for mode in (ISO, MONO):
        c = assert_parity(gd, dgd, p, mode, "c1d")
        assert c == pins.trace_cycle3(gd, (0, 1, 2), 0, mode)


@pytest.mark.parametrize("scale", [10, 13])
def test_rmat_motifs(scale):
    g = configs.c2_graph(scale=scale)
    dg = hpm.Graph.from_host(g)
    for p, mode in configs.c2_runs():
        say(f"rmat scale={scale} {p.name} mode={mode}")
        assert_parity(g, dg, p, mode, f"{p.name}/{mode}")


def test_unlabelled_rmat_4_vertex_motifs():
    g = rmat(10, 1 << 13, seed=31)
    dg = hpm.Graph.from_host(g)
    for name in ("cycle4", "ffl_tail", "star3_back", "clique4_minus1", "cycle3"):
        p = motif(name)
        for mode in (ISO, MONO):
            say(f"unlabelled {name} {mode}")
            assert_parity(g, dg, p, mode, name)


def test_five_vertex_motifs_connectome_shape():
    from synth.graphs import connectome
    g = connectome(30_000, 240_000, seed=8)
    dg = hpm.Graph.from_host(g)
    rng = np.random.default_rng(0)
    for name in configs.C3_MOTIFS:
        k, arcs = MOTIFS[name]
        vl = rng.integers(0, 8, size=k).tolist()
        cases = [motif(name, vlabels=vl, elabels=[3] * len(arcs), eop=GE),
                 motif(name, elabels=[10] * len(arcs), eop=GE)]
        for p in cases:
            for mode in (ISO, MONO):
                say(f"connectome {name} labels={p.vval.ravel().tolist()} mode={mode}")
                assert_parity(g, dg, p, mode, name)


def test_two_vertex_patterns():
    g = erdos_renyi(300, 4000, seed=17)
    dg = hpm.Graph.from_host(g)
    pats = [
        make_pattern(2, [(0, 1)], 1, 1, [[(EQ, 1)], [(EQ, 2)]], [[(EQ, 0)]]),
        make_pattern(2, [(1, 0)], 1, 1, [[(EQ, 1)], [(GE, 2)]], None),
        make_pattern(2, [(0, 1), (1, 0)], 1, 1, None, [[(EQ, 1)], [(GE, 1)]]),
        make_pattern(2, [(0, 1)], 1, 1),
    ]
    for p in pats:
        for mode in (ISO, MONO):
            assert_parity(g, dg, p, mode, f"k2 {p.arcs()}")


def test_random_patterns_up_to_eight_vertices():
    g = configs.c2_graph(scale=11)
    dg = hpm.Graph.from_host(g)
    rng = np.random.default_rng(42)
    for i in range(24):
        p = random_pattern(rng, kmin=3, kmax=8)
        mode = ISO if i % 2 else MONO
        say(f"random pattern {i} k={p.k} arcs={p.n_arcs} mode={mode}")
        assert_parity(g, dg, p, mode, f"rp{i}")


def test_largest_pattern_sixteen_vertices():
    # directed 48-cycle plus sparse random chords; 16-vertex patterns
    rng = np.random.default_rng(3)
    n = 48
    A = np.zeros((n, n), dtype=np.int64)
    A[np.arange(n), (np.arange(n) + 1) % n] = 1
    R = (rng.random((n, n)) < 0.04).astype(np.int64)
    np.fill_diagonal(R, 0)
    A = np.maximum(A, R)
    g = from_dense(A, [rng.integers(0, 2, size=n)], [np.zeros((n, n))])
    dg = hpm.Graph.from_host(g)
    path = make_pattern(16, [(i, i + 1) for i in range(15)], 1, 1)
    assert assert_parity(g, dg, path, ISO, "path16 iso") > 0
    closed = make_pattern(16, [(i, i + 1) for i in range(15)] + [(15, 0), (3, 9)], 1, 1)
    assert assert_parity(g, dg, closed, MONO, "path16+2 mono") > 0


def test_reorder_and_budget_invariance():
    g12 = configs.c2_graph(scale=12)
    g11 = rmat(11, 1 << 14, seed=31)
    cases = [(g12, p, mode) for p, mode in configs.c2_runs()]
    cases += [(g11, motif(name), ISO) for name in ("cycle4", "ffl_tail", "clique4_minus1")]
    devs = {}
    for g, p, mode in cases:
        dg = devs.setdefault(id(g), hpm.Graph.from_host(g))
        base_cnt, base = gpu_rows(dg, p, mode)
        c1, r1 = gpu_rows(dg, p, mode, flags=hpm.F_NO_REORDER)
        assert c1 == base_cnt
        np.testing.assert_array_equal(r1, base)
        # a small scratch budget forces several arc chunks and frontier chunks
        c2, r2 = gpu_rows(dg, p, mode, budget=600_000)
        st = hpm.last_stats()
        assert c2 == base_cnt
        np.testing.assert_array_equal(r2, base)
        say(f"budget {p.name}/{mode}: chunks={st['chunks']} count={c2}")


def test_whole_depth_piece_and_its_chunked_retry():
    # A depth with millions of candidates and rows of over 512 is expanded
    # whole, into room for one frontier chunk of new rows; under tight budgets
    # more rows pass than fit, and the depth is redone in chunks of
    # candidates.  Counts and rows equal the oracle's whatever the budget.
    g = rmat(12, 1 << 17, seed=31)
    dg = hpm.Graph.from_host(g)
    for name in ("cycle4", "clique4_minus1"):
        p = motif(name)
        want = oracle.match(g, p, ISO, threads=8)
        for budget in (None, 16 << 20, 4 << 20):
            cnt, rows = gpu_rows(dg, p, ISO, budget=budget)
            st = hpm.last_stats()
            say(f"whole depth {name} budget={budget}: count={cnt} rows={st['rows'][:4]} "
                f"work={st['work'][:4]} chunks={st['chunks']}")
            assert cnt == want.count, (name, budget)
            np.testing.assert_array_equal(rows, want.rows, err_msg=f"{name} {budget}")
            c2, _ = hpm.match(dg, p, ISO, budget=budget)
            assert c2 == want.count, (name, budget)


def test_relabelled_target():
    g = configs.c2_graph(scale=11)
    perm = np.random.default_rng(9).permutation(g.n)
    gp = permute_vertices(g, perm)
    dg, dgp = hpm.Graph.from_host(g), hpm.Graph.from_host(gp)
    for p, mode in configs.c2_runs()[:4]:
        c, r = gpu_rows(dg, p, mode)
        cp, rp = gpu_rows(dgp, p, mode)
        assert c == cp
        np.testing.assert_array_equal(lexsorted(perm[r]), rp)


def test_empty_and_tiny_graphs():
    p = motif("cycle3")
    for n in (0, 1, 2, 3):
        A = np.zeros((n, n), dtype=np.int64)
        if n == 3:
            A[0, 1] = A[1, 2] = A[2, 0] = 1
        g = from_dense(A, [np.zeros(n)], [np.zeros((n, n))])
        dg = hpm.Graph.from_host(g)
        for mode in (ISO, MONO):
            cnt, rows = gpu_rows(dg, p, mode)
            assert cnt == (3 if n == 3 else 0)


def test_truncated_and_nomem():
    g = configs.c1d_graph()
    dg = hpm.Graph.from_host(g)
    p = configs.c1u_pattern()
    total, _ = hpm.match(dg, p, MONO)
    assert total > 10
    with pytest.raises(hpm.HpmError) as ei:
        hpm.match(dg, p, MONO, mappings=True, cap=10)
    assert ei.value.status == hb.E_TRUNCATED
    with pytest.raises(hpm.HpmError) as ei:
        hpm.match(dg, p, MONO, budget=1000)
    assert ei.value.status == hb.E_NOMEM
    # the graph is still usable after errors
    assert hpm.match(dg, p, MONO)[0] == total


def _create_status(n, arcs, in_arcs=None):
    lib = hpm.load()
    arcs = np.array(arcs, dtype=np.int64).reshape(-1, 2)
    in_arcs = arcs if in_arcs is None else np.array(in_arcs, dtype=np.int64).reshape(-1, 2)
    m = arcs.shape[0]
    out_off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(arcs[:, 0], minlength=n), out=out_off[1:])
    in_off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(in_arcs[:, 1], minlength=n), out=in_off[1:])
    out_nbrs = arcs[:, 1].astype(np.int32)         # rows keep the given order
    order = np.lexsort((in_arcs[:, 0], in_arcs[:, 1]))
    in_nbrs = in_arcs[order, 0].astype(np.int32)
    h = ctypes.c_void_p()
    st = lib.hpm_graph_create(ctypes.byref(h), n, m, out_off.ctypes.data, out_nbrs.ctypes.data,
                              in_off.ctypes.data, in_nbrs.ctypes.data, 0, None, 0, None, None)
    if st == 0:
        lib.hpm_graph_destroy(h)
    return st


def test_graph_create_errors():
    assert _create_status(3, [(0, 1), (1, 2), (2, 0)]) == hb.OK
    assert _create_status(3, [(0, 2), (0, 1), (1, 2)]) == hb.E_GRAPH            # unsorted row
    assert _create_status(3, [(0, 1), (0, 1), (1, 2)]) == hb.E_GRAPH            # repeat
    assert _create_status(3, [(0, 1), (1, 1), (1, 2)]) == hb.E_GRAPH            # self-loop
    assert _create_status(3, [(0, 1), (1, 2), (2, 0)],
                          [(0, 1), (1, 2), (2, 1)]) == hb.E_GRAPH               # not transpose
    lib = hpm.load()
    h = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int64)
    bad = np.array([1, 7], np.int32)                                            # id out of range
    assert lib.hpm_graph_create(ctypes.byref(h), 2, 2, off.ctypes.data, bad.ctypes.data,
                                off.ctypes.data, bad.ctypes.data, 0, None, 0, None,
                                None) == hb.E_GRAPH


def test_pattern_errors_and_column_mismatch():
    g = configs.c1_graph()
    dg = hpm.Graph.from_host(g)
    p = make_pattern(4, [(0, 1), (2, 3)], 1, 1)
    with pytest.raises(hpm.HpmError) as ei:
        hpm.match(dg, p, ISO)
    assert ei.value.status == hb.E_PATTERN
    p2 = make_pattern(3, [(0, 1), (1, 2)], 2, 1)   # two vertex columns, graph has one
    with pytest.raises(hpm.HpmError):
        hpm.match(dg, p2, ISO)


def test_repeated_calls_are_deterministic():
    g = configs.c2_graph(scale=12)
    dg = hpm.Graph.from_host(g)
    p, mode = configs.c2_runs()[4]
    first = gpu_rows(dg, p, mode)
    for _ in range(3):
        again = gpu_rows(dg, p, mode)
        assert again[0] == first[0]
        np.testing.assert_array_equal(again[1], first[1])


def test_prefiltered_lists_change_nothing():
    # Large-work depths pre-filter long shared candidate lists; the result must
    # equal the unfiltered path and the oracle.
    g = rmat(10, 1 << 13, seed=31)
    dg = hpm.Graph.from_host(g)
    used = 0
    for name, mode in (("star3_back", ISO), ("cycle4", MONO), ("ffl_tail", MONO)):
        p = motif(name)
        c0, r0 = gpu_rows(dg, p, mode, flags=hpm.F_NO_FILTER)
        assert hpm.last_stats()["filtered_lists"] == 0
        c1, r1 = gpu_rows(dg, p, mode)
        used += hpm.last_stats()["filtered_lists"]
        assert c0 == c1
        np.testing.assert_array_equal(r0, r1)
        want = oracle.match(g, p, mode, threads=8, rows=False)
        assert c1 == want.count
        assert oracle.fingerprint(r1) == want.fingerprint
        say(f"filter {name}/{mode}: count={c1} lists={hpm.last_stats()['filtered_lists']}")
        # count only: the last level may count filtered rows from their lists
        assert hpm.match(dg, p, mode)[0] == want.count
    assert used > 0


def hub_graph(seed=41, n=6000, m=24000, hubs=2, deg=2500):
    """Sparse uniform arcs plus `hubs` vertices with `deg` out-neighbours and
    `deg` other in-neighbours each: candidate lists longer than one filter
    piece that many partial mappings share."""
    rng = np.random.default_rng(seed)
    src, dst = [rng.integers(0, n, m)], [rng.integers(0, n, m)]
    for h in range(hubs):
        t = rng.choice(np.arange(hubs, n), 2 * deg, replace=False)
        src += [np.full(deg, h), t[deg:]]
        dst += [t[:deg], np.full(deg, h)]
    src, dst = np.concatenate(src), np.concatenate(dst)
    keep = src != dst
    keys = np.unique(src[keep] * n + dst[keep])
    return graph_from_arcs(n, keys // n, keys % n, [rng.integers(0, 4, n)],
                           lambda mm: [rng.integers(0, 2, mm)])


def test_prefilter_split_over_pieces_changes_nothing():
    # Hub lists of 2500 entries are filtered by several blocks each (pieces of
    # 1024 entries, then merged in order); rows must equal the unfiltered path
    # and the oracle's count and fingerprint.
    g = hub_graph()
    dg = hpm.Graph.from_host(g)
    lists = pieces = 0
    for name, mode in (("ffl_tail", MONO), ("ffl_tail", ISO), ("cycle4", ISO)):
        p = motif(name)
        c0, r0 = gpu_rows(dg, p, mode, flags=hpm.F_NO_FILTER)
        c1, r1 = gpu_rows(dg, p, mode)
        st = hpm.last_stats()
        lists += st["filtered_lists"]
        pieces += st["filter_pieces"]
        assert c0 == c1
        np.testing.assert_array_equal(r0, r1)
        want = oracle.match(g, p, mode, threads=8, rows=False)
        assert c1 == want.count
        assert oracle.fingerprint(r1) == want.fingerprint
        say(f"hub filter {name}/{mode}: count={c1} lists={st['filtered_lists']} "
            f"pieces={st['filter_pieces']}")
        # tight scratch budgets: chunked frontiers, and filters that run
        # without the split staging area or not at all
        for budget in (24 << 20, 6 << 20):
            c2, r2 = gpu_rows(dg, p, mode, budget=budget)
            st2 = hpm.last_stats()
            say(f"  budget {budget >> 20} MiB: chunks={st2['chunks']} "
                f"lists={st2['filtered_lists']} pieces={st2['filter_pieces']}")
            assert c2 == c1
            np.testing.assert_array_equal(r2, r1)
    assert pieces > lists > 0


def test_counts_from_filtered_lists_equal_the_oracle():
    # Count-only last levels whose filtered lists enforce every arc-related
    # position: monomorphism subtracts the rows' own images, induced
    # isomorphism also the neighbours of the images it must not touch (a
    # wavefront per row, or the tiled extension for hub neighbourhoods).
    g = hub_graph()
    dg = hpm.Graph.from_host(g)
    counted = {ISO: 0, MONO: 0}
    for name, mode in (("star3_back", ISO), ("star3_back", MONO), ("ffl_tail", ISO),
                       ("cycle4", ISO)):
        p = motif(name)
        c1, _ = hpm.match(dg, p, mode)
        st = hpm.last_stats()
        counted[mode] += st["counted_rows"]
        c0, _ = hpm.match(dg, p, mode, flags=hpm.F_NO_FILTER)
        want = oracle.match(g, p, mode, threads=8, rows=False)
        say(f"hub count {name}/{mode}: {c1} counted_rows={st['counted_rows']} "
            f"counted_work={st['counted_work']} work={st['work'][:p.k]}")
        assert c1 == c0 == want.count
    assert counted[ISO] > 0 and counted[MONO] > 0


def test_batch_equals_single_and_oracle():
    g = configs.c2_graph(scale=12)
    dg = hpm.Graph.from_host(g)
    rng = np.random.default_rng(77)
    pats, modes = [], []
    for i in range(48):
        p = random_pattern(rng, kmin=3, kmax=8)
        pats.append(p)
        modes.append(ISO if i % 2 else MONO)
    for workers in (1, 4, 7):
        counts, status = hpm.match_batch(dg, pats, modes, workers=workers)
        assert status == [0] * len(pats)
        for p, m, c in zip(pats, modes, counts):
            assert c == hpm.match(dg, p, m)[0]
    for p, m, c in zip(pats[:16], modes[:16], counts[:16]):
        assert c == oracle.match(g, p, m, threads=8, rows=False).count
    # the worker-count tuner runs every width on the same batch (checking the
    # counts agree) and returns one of them
    w, ms = hpm.batch_tune(dg, pats, modes)
    assert w in (1, 2, 4, 8, 16, 32) and ms > 0
    # a failing pattern reports its own status and the others still run
    bad = make_pattern(4, [(0, 1), (2, 3)], 1, 1)
    with pytest.raises(hpm.HpmError):
        hpm.match_batch(dg, pats[:3] + [bad], modes[:3] + [ISO], workers=2)


def test_first_k_stops_early_with_valid_rows():
    # max_matches: the count is min(total, limit) and every returned row is an
    # embedding from the oracle's set; a small limit stops the arc scan early.
    g = rmat(12, 1 << 15, seed=41)
    dg = hpm.Graph.from_host(g)
    p = motif("star3_back", vlabels=[0, 0, 0, 0])
    for mode in (ISO, MONO):
        want = oracle.match(g, p, mode, threads=8)
        total = want.count
        assert total > 1000
        full = {tuple(r) for r in want.rows.tolist()}
        for limit in (1, 7, 1000, total - 1, total, total + 5):
            c, _ = hpm.match(dg, p, mode, max_matches=limit)
            assert c == min(limit, total)
            c2, t = hpm.match(dg, p, mode, mappings=True, cap=min(limit, total),
                              max_matches=limit)
            assert c2 == min(limit, total)
            rows = t.cpu().numpy()
            assert rows.shape == (c2, p.k)
            got = {tuple(r) for r in rows.tolist()}
            assert len(got) == c2 and got <= full
    say(f"first-k on scale 12: total {total}")
    big = rmat(17, 1 << 21, seed=42)
    dbig = hpm.Graph.from_host(big)
    c, _ = hpm.match(dbig, motif("cycle3"), MONO, max_matches=1)
    st = hpm.last_stats()
    assert c == 1 and st["arcs_scanned"] < big.m
    call, _ = hpm.match(dbig, motif("cycle3"), MONO)
    assert hpm.last_stats()["arcs_scanned"] == big.m and call > 1
    counts, _ = hpm.match_batch(dbig, [motif("cycle3")] * 3, [MONO, ISO, MONO], workers=2,
                                max_matches=5)
    assert counts == [min(5, hpm.match(dbig, motif("cycle3"), m)[0]) for m in (MONO, ISO, MONO)]


def test_overlap_test_changes_nothing():
    # HPM_F_OVERLAP drops depth-2 rows whose endpoints share fewer neighbours
    # than the pattern's first two positions; results must not change, and rows
    # must be dropped where those positions have common neighbours.
    g = rmat(10, 1 << 13, seed=51)
    dg = hpm.Graph.from_host(g)
    removed = 0
    for name in ("clique4_minus1", "ffl_tail", "cycle4", "star3_back", "cycle3"):
        for mode in (ISO, MONO):
            p = motif(name)
            c0, _ = hpm.match(dg, p, mode)
            c1, _ = hpm.match(dg, p, mode, flags=hpm.F_OVERLAP)
            removed += hpm.last_stats()["overlap_removed"]
            assert c0 == c1, (name, mode)
            if c1 <= 1_000_000:
                _, r0 = gpu_rows(dg, p, mode)
                _, r1 = gpu_rows(dg, p, mode, flags=hpm.F_OVERLAP)
                np.testing.assert_array_equal(r0, r1)
            assert c1 == oracle.match(g, p, mode, threads=8, rows=False).count
    say(f"overlap test removed {removed} depth-2 rows")
    assert removed > 0


def test_lookahead_changes_nothing():
    # HPM_F_LOOKAHEAD drops rows with a frontier position that has no
    # candidate; counts and rows must equal the oracle's (both modes, labels
    # and predicates, alone and with the overlap test, and with a budget that
    # forces several chunks), and rows must be dropped somewhere
    g = rmat(10, 1 << 13, seed=51)
    dg = hpm.Graph.from_host(g)
    removed = 0
    cases = [(motif(n), m) for n in ("clique4_minus1", "ffl_tail", "cycle4", "star3_back")
             for m in (ISO, MONO)]
    rng = np.random.default_rng(808)
    for i in range(12):
        cases.append((random_pattern(rng, kmin=4, kmax=7), ISO if i % 2 else MONO))
    for p, mode in cases:
        want = oracle.match(g, p, mode, threads=8)
        for flags, budget in ((hpm.F_LOOKAHEAD, None), (hpm.F_LOOKAHEAD | hpm.F_OVERLAP, None),
                              (hpm.F_LOOKAHEAD, 600_000)):
            c1, _ = hpm.match(dg, p, mode, flags=flags, budget=budget)
            removed += hpm.last_stats()["lookahead_removed"]
            assert c1 == want.count, (p.name, mode, flags)
        if want.count <= 1_000_000:
            _, r1 = gpu_rows(dg, p, mode, flags=hpm.F_LOOKAHEAD)
            np.testing.assert_array_equal(r1, want.rows)
    say(f"look-ahead removed {removed} rows")
    assert removed > 0
    dg.close()
    # five-vertex motifs on a connectome-shaped graph (weights, reciprocity)
    gc = configs.c3_graph(n=20_000, m=150_000)
    dc = hpm.Graph.from_host(gc)
    for p in configs.c3_patterns():
        want = oracle.match(gc, p, MONO, threads=8, rows=False)
        c1, _ = hpm.match(dc, p, MONO, flags=hpm.F_LOOKAHEAD)
        assert c1 == want.count, p.name
    dc.close()


def _pred_ok(op, val, x):
    x = np.asarray(x)
    if op == 0:
        return np.ones(x.shape, dtype=bool)
    return (x == val) if op == 1 else (x >= val)


def _validator_survivors(g, p, mode, o0, o1):
    """Depth-2 rows the validators must keep, from their definitions (Alg. 2,
    Alg. 3 with the reverse-arc rule of Eq. (1)), with numpy over every arc."""
    n, m = g.n, g.m
    indeg, outdeg = np.diff(g.in_off), np.diff(g.out_off)
    arcs = list(p.arcs())
    pin = [sum(1 for a, b in arcs if b == v) for v in range(p.k)]
    pout = [sum(1 for a, b in arcs if a == v) for v in range(p.k)]

    def vv(a):
        ok = (indeg >= pin[a]) & (outdeg >= pout[a])
        for c in range(len(g.vcols)):
            ok &= _pred_ok(int(p.vop[a, c]), int(p.vval[a, c]), g.vcols[c])
        return ok

    def arc_pred(i, eids):
        ok = np.ones(eids.shape, dtype=bool)
        for c in range(len(g.ecols)):
            ok &= _pred_ok(int(p.eop[i, c]), int(p.eval[i, c]), g.ecols[c][eids])
        return ok

    src = np.repeat(np.arange(n, dtype=np.int64), outdeg)
    dst = g.out_nbrs.astype(np.int64)
    eid = np.arange(m)
    keys = src * n + dst
    rev_key = dst * n + src
    pos = np.searchsorted(keys, rev_key)
    pos[pos >= m] = 0
    rev = np.where(keys[pos] == rev_key, pos, -1)          # out-CSR id of the reverse arc
    idx = {a: i for i, a in enumerate(arcs)}
    if (o0, o1) in idx:        # target arc x -> y is the image of o0 -> o1
        f0, f1, fwd_i, back = src, dst, idx[(o0, o1)], idx.get((o1, o0))
    else:                      # only o1 -> o0: target arc x -> y is its image
        f0, f1, fwd_i, back = dst, src, idx[(o1, o0)], None
    ok = vv(o0)[f0] & vv(o1)[f1] & arc_pred(fwd_i, eid)
    if back is not None:
        ok &= rev >= 0
        ok[ok] &= arc_pred(back, rev[ok])
    elif mode == ISO:
        ok &= rev < 0
    return np.stack([f0[ok], f1[ok]], axis=1).astype(np.int32)


def test_scan_survivors_equal_the_validator_definitions():
    # the vertex and edge validators (Sec. III-B, Alg. 2-3) as a stage: the
    # depth-2 rows equal, as a set, a numpy filter written from their
    # definitions, and every oracle embedding's images of positions 0 and 1
    # are among them (the validators only remove what cannot extend)
    graphs = [("rmat10", rmat(10, 1 << 13, seed=61)),
              ("connectome", configs.c3_graph(n=20_000, m=150_000))]
    rng = np.random.default_rng(4242)
    for gname, g in graphs:
        dg = hpm.Graph.from_host(g)
        if gname == "rmat10":
            cases = [(p, m) for p in configs.c2_patterns() for m in (ISO, MONO)]
            for i in range(8):
                cases.append((random_pattern(rng, kmin=2, kmax=6), ISO if i % 2 else MONO))
        else:
            cases = [(p, MONO) for p in configs.c3_patterns()]
            cases += [(p, ISO) for p in configs.c3_patterns()]
        for p, mode in cases:
            order = hpm.plan_order(p, len(g.vcols), len(g.ecols))
            want = _validator_survivors(g, p, mode, order[0], order[1])
            got = hpm.scan_survivors(dg, p, mode).cpu().numpy()
            np.testing.assert_array_equal(lexsorted(got), lexsorted(want),
                                          err_msg=f"{gname} {p.name} {mode}")
            res = oracle.match(g, p, mode, threads=8, rows=True) if p.k <= 5 else None
            if res is not None and res.count:
                pairs = {(int(a), int(b)) for a, b in want}
                need = {(int(r[order[0]]), int(r[order[1]])) for r in res.rows}
                assert need <= pairs, f"{gname} {p.name}: a validator dropped an embedding"
            say(f"{gname} {p.name}/{mode}: {len(got)} survivors")
        dg.close()


def test_count_wrap_is_reported():
    # a running count that starts at 2^64 - 1 (test-only flag) wraps on the
    # first embedding: the call fails with HPM_E_OVERFLOW
    g = rmat(10, 1 << 13, seed=61)
    dg = hpm.Graph.from_host(g)
    for p, mode in ((motif("cycle3"), MONO), (motif("ffl_tail"), ISO), (motif("cycle4"), MONO)):
        c, _ = hpm.match(dg, p, mode)
        assert c > 0
        with pytest.raises(hpm.HpmError) as e:
            hpm.match(dg, p, mode, flags=hpm.F_COUNT_FROM_MAX)
        assert e.value.status == hb.E_OVERFLOW, p.name
    dg.close()


def _loosest_predicate_arcs(g, p):
    """Arcs of g whose columns pass, for every column that all pattern arcs
    constrain, the hull of the pattern arcs' ranges on it."""
    keep = np.ones(g.m, dtype=bool)
    for c in range(len(g.ecols)):
        ops, vals = p.eop[:, c], p.eval[:, c]
        if (ops == ANY).any():
            continue
        lo = int(vals.min())
        hi = np.iinfo(np.int32).max if (ops == GE).any() else int(vals.max())
        col = np.asarray(g.ecols[c])
        keep &= (col >= lo) & (col <= hi)
    return int(keep.sum())


def test_arc_index_changes_nothing():
    # monomorphism queries whose arcs all carry a predicate read adjacency
    # restricted to the arcs that pass the loosest of them: counts and rows
    # equal the oracle's and the unrestricted run's, with several chunks too,
    # and the index is built where the predicate is selective
    g = configs.c3_graph(n=20_000, m=150_000)
    dg = hpm.Graph.from_host(g)
    rng = np.random.default_rng(5150)
    cases = list(configs.c3_patterns())
    for i in range(10):
        cases.append(random_pattern(rng, kmin=3, kmax=6, vlabels=("uniform", 8), eop=GE,
                                    eval_const=int(rng.integers(3, 12))))
    built = 0
    for p in cases:
        want = oracle.match(g, p, MONO, threads=8)
        for flags, budget in ((0, None), (hpm.F_NO_ARC_INDEX, None), (0, 4 << 20),
                              (hpm.F_LOOKAHEAD, None)):
            cnt, _ = hpm.match(dg, p, MONO, flags=flags, budget=budget)
            st = hpm.last_stats()
            if flags == 0 and budget is None and st["index_arcs"] > 0:
                # the index holds exactly the arcs that pass the loosest predicate
                built += 1
                assert st["index_arcs"] == _loosest_predicate_arcs(g, p), p.name
            assert cnt == want.count, (p.name, flags, budget)
        if want.count <= 2_000_000:
            _, rows = gpu_rows(dg, p, MONO)
            np.testing.assert_array_equal(rows, want.rows, err_msg=p.name)
        say(f"arc index {p.name}: {want.count} embeddings, index arcs {st['index_arcs']}")
    assert built >= 3
    # induced isomorphism never uses it (non-arcs need the whole graph)
    p = configs.c3_patterns()[0]
    cnt, _ = hpm.match(dg, p, ISO)
    assert hpm.last_stats()["index_arcs"] == 0
    assert cnt == oracle.match(g, p, ISO, threads=8, rows=False).count
    dg.close()
