"""Parity at the benchmark's full size (R-MAT scale 20, 2^24 arcs), GPU.

Every query of the benchmark step is compared with the oracle: the count
exactly; the mapping set bit-exact after sorting when it has at most 2^26
rows; above that, the order-independent 128-bit fingerprint of all rows plus a
sorted bit-exact comparison of the rows whose image of pattern vertex 0 lies
in a seeded 1% of the vertices.  Matching runs in the same launch
configuration the benchmark times (default scratch budget).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2507_04130_amd as hpm
from synth import configs

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))
FULL_ROWS_LIMIT = 1 << 26


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rmat20():
    say("generating R-MAT scale 20")
    g = configs.c2_graph()
    dg = hpm.Graph.from_host(g)
    yield g, dg
    dg.close()


def lexsorted(rows):
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] else rows


@pytest.mark.parametrize("qi", range(8))
def test_rmat20_query(rmat20, qi):
    import torch
    g, dg = rmat20
    p, mode = configs.c2_runs()[qi]
    say(f"rmat20 {p.name} mode={mode}")
    cnt, rows_dev = hpm.match(dg, p, mode, mappings=True)
    assert hpm.match(dg, p, mode)[0] == cnt
    if cnt <= FULL_ROWS_LIMIT:
        want = oracle.match(g, p, mode, threads=THREADS)
        assert cnt == want.count
        np.testing.assert_array_equal(lexsorted(rows_dev.cpu().numpy()), want.rows)
        return
    want = oracle.match(g, p, mode, threads=THREADS, rows=False)
    assert cnt == want.count
    rows = rows_dev.cpu().numpy()
    assert oracle.fingerprint(rows) == want.fingerprint
    key = np.random.default_rng(777).random(g.n) < 0.01
    sl = oracle.match(g, p, mode, threads=THREADS, root_mask=key.astype(np.uint8))
    mine = rows[key[rows[:, 0]]]
    np.testing.assert_array_equal(lexsorted(mine), sl.rows)
    del rows_dev
    torch.cuda.empty_cache()


def test_batched_workload_full_size(rmat20):
    # the 256 screened random patterns in one batched call (8 workers, as the
    # benchmark times it) give the oracle's stored counts, pattern by pattern
    g, dg = rmat20
    runs = configs.c4_patterns()
    want = configs.c4_expected_counts(len(runs))
    say(f"batched workload: {len(runs)} patterns")
    counts, status = hpm.match_batch(dg, [p for p, _ in runs], [m for _, m in runs], workers=8)
    assert status == [0] * len(runs)
    bad = [i for i, (a, b) in enumerate(zip(counts, want)) if a != b]
    assert not bad, f"patterns {bad[:8]} differ from the oracle"
    # first-k over the same patterns: min(count, 1000) each
    capped, _ = hpm.match_batch(dg, [p for p, _ in runs[:64]], [m for _, m in runs[:64]],
                                workers=8, max_matches=1000)
    assert capped == [min(c, 1000) for c in want[:64]]


@pytest.mark.skip(reason="persistent batched launch switched off: it stalled on the device and "
                         "no cause has been shown")
def test_batched_workload_persistent_full_size(rmat20):
    # the same 256 patterns in one persistent launch, with the default setting
    # and two others, give the oracle's stored counts
    g, dg = rmat20
    runs = configs.c4_patterns()
    want = configs.c4_expected_counts(len(runs))
    pats, modes = [p for p, _ in runs], [m for _, m in runs]
    for cfg in (None, {"items_per_lane": 4, "chunk_rows": 1024, "task_work": 65536,
                       "strategy": hpm.X_SHORTER},
                {"items_per_lane": 1, "chunk_rows": 64, "task_work": 4096}):
        counts, status = hpm.match_batch_persistent(dg, pats, modes, config=cfg)
        st = hpm.last_batch_stats()
        say(f"persistent {cfg}: {st['kernel_ms']:.2f} ms kernel, {st['ms_total']:.2f} ms call, "
            f"tasks {st['tasks_validate']}/{st['tasks_scan']}/{st['tasks_expand']}, arena "
            f"{st['arena_bytes'] >> 20} MiB, fallback {st['fallback_patterns']}")
        assert status == [0] * len(runs)
        bad = [i for i, (a, b) in enumerate(zip(counts, want)) if a != b]
        assert not bad, f"patterns {bad[:8]} differ from the oracle"
