"""Screen the random patterns of the batched workload with the oracle.

Draws patterns from the batched workload's pattern seed in order, runs the
oracle on the full R-MAT graph (2^20 vertices, 2^24 arcs, graph seed) with a
bound of MAX_TESTED candidate images tested, and accepts a draw when the
search finishes inside the bound with at most MAX_COUNT embeddings.  The bound
stands in for a time limit (the oracle tests 1e8 candidates in 0.2-0.9 s on
eight host threads, so 2e9 is a few seconds to about twenty): it is
deterministic, unlike wall time.  Writes the first 256 accepted draw indices
with their oracle counts to batch_patterns_screened.json; these counts are the
expected per-pattern results of the batched workload.

    python tests/golden/screen_batch_patterns.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import configs  # noqa: E402

MAX_TESTED = 2_000_000_000
MAX_COUNT = 1_000_000_000
WANT = 256


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    g = configs.c2_graph()
    accepted, rejected = [], []
    t0 = time.time()
    for i, (p, mode) in enumerate(configs.c4_draws(16 * WANT)):
        r = oracle.match(g, p, mode, threads=threads, rows=False, max_tested=MAX_TESTED)
        if r.capped or r.count > MAX_COUNT:
            rejected.append(i)
        else:
            accepted.append({"draw": i, "k": p.k, "arcs": p.n_arcs, "mode": int(mode),
                             "count": r.count, "tested": r.tested})
        print(f"draw {i}: k={p.k} arcs={p.n_arcs} mode={mode} "
              f"{'capped' if r.capped else r.count} tested={r.tested} {r.seconds:.1f}s "
              f"[{len(accepted)} accepted, {time.time() - t0:.0f}s]", flush=True)
        if len(accepted) == WANT:
            break
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_patterns_screened.json")
    with open(out, "w") as f:
        json.dump({"about": __doc__.strip().splitlines()[0], "graph": "rmat scale 20, 2^24 arcs",
                   "max_tested": MAX_TESTED, "max_count": MAX_COUNT, "rejected": rejected, "accepted": accepted},
                  f, indent=0)
    print(f"{len(accepted)} accepted out of {accepted[-1]['draw'] + 1} draws")


if __name__ == "__main__":
    main()
