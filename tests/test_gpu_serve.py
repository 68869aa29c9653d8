"""Served form (GPU): a resident graph answering queued queries through the C ABI.

Every query's result must be the same alone (hpm_match), in the mix (many
queries in flight on the server's workers, admitted against a scratch
budget) and in the oracle: counts bit-exact, mapping sets equal by sorted rows
and fingerprint.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2507_04130_amd as hpm
from paper_2507_04130_amd import hpm as hb
from synth import configs
from synth.patterns import ISO, MONO, make_pattern, random_pattern

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def graph():
    g = configs.c2_graph(scale=12)
    dg = hpm.Graph.from_host(g)
    yield g, dg
    dg.close()


def queries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        p = random_pattern(rng, kmin=3, kmax=8)
        out.append((p, ISO if rng.random() < 0.5 else MONO))
    return out


def lexsorted(rows):
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] else rows


def test_results_same_alone_in_mix_and_oracle(graph):
    g, dg = graph
    qs = queries(48, 91)
    alone = [hpm.match(dg, p, m)[0] for p, m in qs]
    srv = hpm.Server(dg, workers=4)
    tickets = [srv.submit(p, m) for p, m in qs]
    res = [srv.poll(t, wait=True) for t in tickets]
    st = srv.stats()
    srv.close()
    say(f"served 48 queries, peak running {st['peak_running']}")
    assert [r["status"] for r in res] == [0] * len(qs)
    assert [r["count"] for r in res] == alone
    assert st["admitted"] == len(qs) and st["running"] == 0 and st["queued"] == 0
    for (p, m), c in zip(qs[:20], alone[:20]):
        assert c == oracle.match(g, p, m, threads=8, rows=False).count


def test_mappings_in_the_mix_equal_the_oracle(graph):
    import torch
    g, dg = graph
    qs = queries(12, 92)
    want = [oracle.match(g, p, m, threads=8) for p, m in qs]
    srv = hpm.Server(dg, workers=3)
    tickets = []
    for (p, m), w in zip(qs, want):
        buf = torch.empty((max(w.count, 1), p.k), dtype=torch.int32, device="cuda")
        tickets.append(srv.submit(p, m, mappings=buf))
    for t, (p, m), w in zip(tickets, qs, want):
        r = srv.poll(t, wait=True)
        assert r["status"] == 0 and r["count"] == w.count
        rows = lexsorted(r["rows"].cpu().numpy())
        np.testing.assert_array_equal(rows, w.rows)
        assert oracle.fingerprint(rows) == w.fingerprint
    srv.close()


def test_admission_bounds_granted_scratch(graph):
    # pool = 640 MiB and every grant is at least 256 MiB: at most two queries
    # run at once whatever the worker count, and results do not change.
    g, dg = graph
    qs = queries(24, 93)
    alone = [hpm.match(dg, p, m)[0] for p, m in qs]
    srv = hpm.Server(dg, workers=6, budget=1280 << 20)
    tickets = [srv.submit(p, m) for p, m in qs]
    res = [srv.poll(t, wait=True) for t in tickets]
    st = srv.stats()
    srv.close()
    assert [r["count"] for r in res] == alone
    assert all(r["granted_bytes"] >= 256 << 20 for r in res)
    assert st["grant_pool_bytes"] == 640 << 20
    assert st["peak_granted_bytes"] <= st["grant_pool_bytes"]
    assert 1 <= st["peak_running"] <= 2


def test_arrivals_while_others_run(graph):
    # queries arrive from another thread while earlier ones are on the device
    g, dg = graph
    qs = queries(32, 94)
    alone = [hpm.match(dg, p, m)[0] for p, m in qs]
    srv = hpm.Server(dg, workers=4)
    tickets = [None] * len(qs)

    def feed():
        for i, (p, m) in enumerate(qs):
            tickets[i] = srv.submit(p, m)
            time.sleep(0.0005)

    th = threading.Thread(target=feed)
    th.start()
    th.join()
    got = [srv.poll(t, wait=True)["count"] for t in tickets]
    srv.close()
    assert got == alone


def test_server_errors(graph):
    g, dg = graph
    srv = hpm.Server(dg, workers=2)
    bad = make_pattern(4, [(0, 1), (2, 3)], 1, 1)      # not weakly connected
    with pytest.raises(hpm.HpmError) as e:
        srv.submit(bad, ISO)
    assert e.value.status == hb.E_PATTERN
    with pytest.raises(hpm.HpmError) as e:
        srv.poll(12345, wait=True)
    assert e.value.status == hb.E_ARG
    p, m = queries(1, 95)[0]
    t = srv.submit(p, m)
    r = srv.poll(t)
    if r is None:
        r = srv.poll(t, wait=True)
    assert r["count"] == hpm.match(dg, p, m)[0]
    with pytest.raises(hpm.HpmError):
        srv.poll(t)                                     # already collected
    # queries left unpolled are still run to completion by close()
    for p, m in queries(6, 96):
        srv.submit(p, m)
    srv.close()
