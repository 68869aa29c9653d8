"""Screen the query pool of the served workload with the oracle.

Draws queries from the served workload's pattern seed in order, runs the
oracle on the full connectome-shaped graph (2e7 vertices, about 1.5e8 arcs,
graph seed) with a bound of MAX_TESTED candidate images tested, and accepts a
draw when the search finishes inside the bound.  Writes the first WANT
accepted draws with their oracle counts and fingerprints to
serve_patterns_screened.json; these are the expected results of every
served query.

    python tests/golden/screen_serve_patterns.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import configs  # noqa: E402

MAX_TESTED = 200_000_000
WANT = 128


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    g = configs.c3_graph()
    print(f"graph n={g.n} m={g.m} in {time.time() - t0:.0f}s", flush=True)
    accepted, rejected = [], []
    t0 = time.time()
    for i, (p, mode) in enumerate(configs.c5_draws(16 * WANT)):
        r = oracle.match(g, p, mode, threads=threads, rows=False, max_tested=MAX_TESTED)
        if r.capped:
            rejected.append(i)
        else:
            accepted.append({"draw": i, "k": p.k, "arcs": p.n_arcs, "mode": int(mode),
                             "count": r.count, "fingerprint": list(r.fingerprint),
                             "tested": r.tested})
        print(f"draw {i}: k={p.k} arcs={p.n_arcs} mode={mode} "
              f"{'capped' if r.capped else r.count} tested={r.tested} {r.seconds:.1f}s "
              f"[{len(accepted)} accepted, {time.time() - t0:.0f}s]", flush=True)
        if len(accepted) == WANT:
            break
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serve_patterns_screened.json")
    with open(out, "w") as f:
        json.dump({"about": __doc__.strip().splitlines()[0],
                   "graph": "connectome-shaped Chung-Lu, 2e7 vertices, about 1.5e8 arcs",
                   "max_tested": MAX_TESTED, "rejected": rejected, "accepted": accepted},
                  f, indent=0)
    print(f"{len(accepted)} accepted out of {accepted[-1]['draw'] + 1} draws")


if __name__ == "__main__":
    main()
