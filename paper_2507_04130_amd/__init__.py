"""Edge-centric subgraph matching (HiPerMotif, arXiv 2507.04130) on AMD MI355X.

The matcher is libhpm.so (HIP kernels for gfx950 behind the C ABI of
include/hpm.h); this package holds its sources (csrc/), the build script and a
thin ctypes binding.
"""
from .hpm import (ANY, EQ, GE, ISO, MONO, F_NO_FILTER, F_NO_REORDER, F_OVERLAP, F_LOOKAHEAD, F_TIMING, F_TIMING_KINDS, Graph,  # noqa: F401
                  HpmError, Server,
                  X_MAPPED, X_SHORTER, abi_version, batch_autotune, batch_tune,
                  last_batch_stats, last_stats, load, match, match_batch, match_batch_persistent,
                  match_noalloc, scan_survivors, F_COUNT_FROM_MAX, F_NO_ARC_INDEX,
                  plan_order, status_string)
