"""Full oracle results of the three connectome queries, by root slices.

Runs the oracle (count and order-independent fingerprint, no rows kept) for
every query of the connectome workload (2e7 vertices, about 1.5e8 arcs, graph
seed; three 5-vertex motifs, monomorphism) over the whole graph.  The roots
(images of pattern vertex 0) are split into SLICES classes by vertex id modulo
SLICES; each class is one oracle run, and its count and fingerprint are stored
in c3_full.json as soon as it finishes.  Counts and fingerprints are sums over
rows (mod 2^64 for the fingerprint), so the classes add up to the full result,
and a test can compare the rows of any finished classes on their own.  A
rerun skips the classes already stored.  The script calls only the oracle and
the seeded generators.

    python tests/golden/screen_c3_full.py [threads]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import configs  # noqa: E402
from synth.patterns import MONO  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_full.json")
SLICES = 16
# cheapest first, so a partial run still pins whole queries
ORDER = ("recip_triad_plus_c3", "ff_chain_c3", "bifan_plus1_c3")


def load():
    if not os.path.exists(OUT):
        return {}
    with open(OUT) as f:
        return json.load(f)["queries"]


def save(queries, m):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"about": __doc__.strip().splitlines()[0], "slices": SLICES,
                   "slice_rule": "root vertex id % slices == slice",
                   "graph": "connectome-shaped Chung-Lu, 2e7 vertices, about 1.5e8 arcs",
                   "graph_m": m, "queries": queries}, f, indent=1)
    os.replace(tmp, OUT)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    g = configs.c3_graph()
    print(f"graph n={g.n} m={g.m} in {time.time() - t0:.0f}s", flush=True)
    queries = load()
    pats = {p.name: p for p in configs.c3_patterns()}
    ids = np.arange(g.n, dtype=np.int64) % SLICES
    for name in ORDER:
        p = pats[name]
        q = queries.setdefault(name, {"k": p.k, "arcs": p.n_arcs, "mode": int(MONO),
                                      "slices": {}})
        for s in range(SLICES):
            if str(s) in q["slices"]:
                continue
            r = oracle.match(g, p, MONO, threads=threads, rows=False,
                             root_mask=(ids == s).astype(np.uint8))
            q["slices"][str(s)] = {"count": r.count, "fingerprint": list(r.fingerprint),
                                   "tested": r.tested, "seconds": round(r.seconds, 1),
                                   "threads": r.threads}
            if len(q["slices"]) == SLICES:
                sl = q["slices"].values()
                q["count"] = sum(v["count"] for v in sl)
                q["fingerprint"] = [sum(v["fingerprint"][i] for v in sl) % (1 << 64)
                                    for i in range(2)]
            save(queries, g.m)
            print(f"{name} slice {s}: count {r.count} tested {r.tested} in {r.seconds:.0f}s "
                  f"[{time.time() - t0:.0f}s]", flush=True)
        if "count" in q:
            print(f"{name}: count {q['count']} fingerprint {q['fingerprint']}", flush=True)


if __name__ == "__main__":
    main()
