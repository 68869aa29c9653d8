"""The batched form as one persistent launch (GPU; calls through the C ABI).

Every count of hpm_match_batch_persistent is compared with the CPU oracle (or
with hpm_match, itself pinned to the oracle): random small graphs with random
patterns of 2-6 vertices in both modes under every extension setting, random
3-8 vertex patterns on an R-MAT graph, two-vertex and sixteen-vertex patterns,
an arena too small for some patterns (they are finished by the single-query
path), blocks that leave after a 1 us idle wait (the host launches again while
tasks are left), the autotuner, and the error paths.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2507_04130_amd as hpm
from synth import configs
from synth.graphs import from_dense, rmat
from synth.patterns import ISO, MONO, make_pattern, motif, random_pattern
from tests.cases import random_small_graph, random_small_pattern

pytestmark = [
    pytest.mark.gpu,
    # the persistent launch did not return on the device (twice, first case of
    # this file); the entry points are switched off until a cause is shown
    pytest.mark.skip(reason="persistent batched launch switched off: it stalled on the device "
                            "and no cause has been shown"),
]

SETTINGS = [
    {"items_per_lane": 1, "chunk_rows": 16, "task_work": 256, "strategy": hpm.X_MAPPED},
    {"items_per_lane": 2, "chunk_rows": 256, "task_work": 4096, "strategy": hpm.X_SHORTER},
    {"items_per_lane": 4, "chunk_rows": 1024, "task_work": 65536, "strategy": hpm.X_MAPPED},
    {"items_per_lane": 4, "chunk_rows": 64, "task_work": 1024, "strategy": hpm.X_SHORTER},
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seed", range(12))
def test_random_small_graphs(seed):
    rng = np.random.default_rng(9100 + seed)
    n = int(rng.integers(8, 40))
    nv, ne = int(rng.integers(0, 3)), int(rng.integers(0, 3))
    g = random_small_graph(rng, n, float(rng.uniform(0.1, 0.5)), nv, ne, nlab=3, nelab=3)
    say(f"persistent seed {seed}: n={g.n} m={g.m} cols={nv},{ne}")
    dg = hpm.Graph.from_host(g)
    pats, modes = [], []
    for i in range(16):
        k = int(rng.integers(2, 7))
        pats.append(random_small_pattern(rng, k, nv, ne, nlab=3, nelab=3))
        modes.append(ISO if i % 2 else MONO)
    want = [oracle.match(g, p, m, threads=4, rows=False).count for p, m in zip(pats, modes)]
    for cfg in SETTINGS:
        counts, status = hpm.match_batch_persistent(dg, pats, modes, config=cfg)
        assert status == [0] * len(pats)
        assert counts == want, cfg
        st = hpm.last_batch_stats()
        say(f"  {cfg}: {st['kernel_ms']:.3f} ms, {st['launches']} launch(es), error bits "
            f"{st['error_bits']}")
        assert st["fallback_patterns"] == 0 and (st["error_bits"] & ~2) == 0, st
    dg.close()


@pytest.fixture(scope="module")
def rmat12():
    g = configs.c2_graph(scale=12)
    dg = hpm.Graph.from_host(g)
    rng = np.random.default_rng(77)
    pats, modes = [], []
    for i in range(48):
        pats.append(random_pattern(rng, kmin=3, kmax=8))
        modes.append(ISO if i % 2 else MONO)
    want = [hpm.match(dg, p, m)[0] for p, m in zip(pats, modes)]
    yield g, dg, pats, modes, want
    dg.close()


def test_rmat_random_patterns(rmat12):
    g, dg, pats, modes, want = rmat12
    for p, m, c in list(zip(pats, modes, want))[:16]:
        assert c == oracle.match(g, p, m, threads=8, rows=False).count
    for cfg in [None] + SETTINGS:
        counts, status = hpm.match_batch_persistent(dg, pats, modes, config=cfg)
        st = hpm.last_batch_stats()
        say(f"rmat12 {cfg}: {st['kernel_ms']:.3f} ms, {st['launches']} launch(es), tasks "
            f"{st['tasks_scan']}/{st['tasks_expand']}, arena {st['arena_bytes']}, "
            f"error bits {st['error_bits']}")
        assert status == [0] * len(pats) and counts == want
        assert st["fallback_patterns"] == 0 and (st["error_bits"] & ~2) == 0
        assert st["tasks_scan"] > 0 and st["tasks_expand"] > 0
        assert st["grid"] >= 256


def test_repeated_launches_are_deterministic(rmat12):
    _, dg, pats, modes, want = rmat12
    for _ in range(3):
        counts, _ = hpm.match_batch_persistent(dg, pats, modes)
        assert counts == want


def test_small_arena_falls_back_to_single_queries(rmat12):
    # budgets that leave 1-8 MiB of arena: the patterns whose rows do not fit
    # are finished by hpm_match, with the same counts
    _, dg, pats, modes, want = rmat12
    hpm.match_batch_persistent(dg, pats, modes)
    st0 = hpm.last_batch_stats()
    say(f"unbounded: arena used {st0['arena_bytes']} of {st0['arena_capacity']}, "
        f"fixed {st0['fixed_bytes']}")
    fell = 0
    for extra in (1 << 20, 2 << 20, 8 << 20):
        counts, status = hpm.match_batch_persistent(dg, pats, modes,
                                                    budget=st0["fixed_bytes"] + extra)
        st = hpm.last_batch_stats()
        say(f"arena {extra >> 20} MiB: capacity {st['arena_capacity']}, fallback "
            f"{st['fallback_patterns']}, error bits {st['error_bits']}")
        assert status == [0] * len(pats) and counts == want
        assert st["arena_capacity"] <= extra
        fell += st["fallback_patterns"]
    if st0["arena_bytes"] > (1 << 20):
        assert fell > 0
    with pytest.raises(hpm.HpmError):
        hpm.match_batch_persistent(dg, pats, modes, budget=st0["fixed_bytes"])


def test_blocks_that_leave_early_are_relaunched(rmat12):
    # an idle wait of 1 us: blocks leave as soon as the queue is briefly empty;
    # the host launches again while tasks are left, and the counts are the same
    _, dg, pats, modes, want = rmat12
    counts, status = hpm.match_batch_persistent(dg, pats, modes, config={"idle_us": 1})
    st = hpm.last_batch_stats()
    say(f"idle 1 us: {st['launches']} launch(es), error bits {st['error_bits']}, fallback "
        f"{st['fallback_patterns']}")
    assert status == [0] * len(pats) and counts == want


def test_two_and_sixteen_vertex_patterns():
    # two-vertex patterns (the scan alone counts) on an R-MAT graph; 16-vertex
    # patterns (the maximum) on a 48-cycle with sparse chords
    g = rmat(10, 8 << 10, 31)
    dg = hpm.Graph.from_host(g)
    pats = [motif("cycle3"), make_pattern(2, [(0, 1)], 1, 1),
            make_pattern(2, [(0, 1), (1, 0)], 1, 1)]
    modes = [MONO, ISO, MONO]
    want = [oracle.match(g, p, m, threads=8, rows=False).count for p, m in zip(pats, modes)]
    counts, status = hpm.match_batch_persistent(dg, pats, modes)
    assert status == [0] * len(pats) and counts == want
    dg.close()
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
    closed = make_pattern(16, [(i, i + 1) for i in range(15)] + [(15, 0), (3, 9)], 1, 1)
    pats, modes = [path, closed, path], [ISO, MONO, MONO]
    want = [oracle.match(g, p, m, threads=8, rows=False).count for p, m in zip(pats, modes)]
    assert min(want) > 0
    for cfg in SETTINGS:
        counts, status = hpm.match_batch_persistent(dg, pats, modes, config=cfg)
        assert status == [0] * len(pats) and counts == want
    dg.close()


def test_autotune_picks_a_setting_with_equal_counts(rmat12):
    _, dg, pats, modes, want = rmat12
    cfg, ms = hpm.batch_autotune(dg, pats[:24], modes[:24])
    say(f"autotuned {cfg} {ms:.3f} ms")
    assert cfg["items_per_lane"] in (1, 2, 4) and cfg["chunk_rows"] in (64, 256, 1024)
    assert cfg["task_work"] in (4096, 65536) and cfg["strategy"] in (hpm.X_MAPPED, hpm.X_SHORTER)
    assert ms > 0
    counts, _ = hpm.match_batch_persistent(dg, pats[:24], modes[:24], config=cfg)
    assert counts == want[:24]


def test_errors(rmat12):
    _, dg, pats, modes, want = rmat12
    for bad in ({"items_per_lane": 3}, {"chunk_rows": 8}, {"chunk_rows": 2048},
                {"strategy": 7}, {"task_work": 100}, {"idle_us": -1}):
        with pytest.raises(hpm.HpmError):
            hpm.match_batch_persistent(dg, pats[:2], modes[:2], config=bad)
    # a failing pattern reports its own status; the others are counted
    badp = make_pattern(4, [(0, 1), (2, 3)], 1, 1)
    with pytest.raises(hpm.HpmError):
        hpm.match_batch_persistent(dg, pats[:3] + [badp], modes[:3] + [ISO])
    assert hpm.match_batch_persistent(dg, [], []) == ([], [])
    with pytest.raises(hpm.HpmError):
        hpm.batch_autotune(dg, [], [])
