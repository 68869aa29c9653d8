"""libhpm on the CPU: symbols, the host-side planner and host-side argument checks.

No kernel runs here.  hpm_plan_order is host-only; hpm_graph_create rejects
malformed offsets before it touches the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2507_04130_amd as hpm
from paper_2507_04130_amd import hpm as hb
from synth.patterns import MOTIFS, is_weakly_connected, make_pattern, motif, random_pattern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hpm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(hpm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    lib = hpm.load()
    declared = _header_functions()
    assert set(declared) == set(hb.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    hdr = open(os.path.join(ROOT, "include", "hpm.h")).read()
    assert hpm.abi_version() == int(re.search(r"#define HPM_ABI_VERSION (\d+)", hdr).group(1))


def test_struct_mirrors_match_the_header(tmp_path):
    # the ctypes mirrors have the sizes and field offsets a C compiler gives
    # the header's structs
    mirrors = {"hpm_match_opts": hb._Opts, "hpm_server_opts": hb._ServerOpts,
               "hpm_query_result": hb._QueryResult, "hpm_server_stats": hb._ServerStats,
               "hpm_match_stats": hb._Stats, "hpm_pattern": hb._Pattern,
               "hpm_batch_config": hb._BatchConfig, "hpm_batch_stats": hb._BatchStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hpm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    # the timing-family flag bits, one family at a time
    for i, kname in enumerate(hb.KERNELS):
        lines.append(f'  printf("timing {kname} %u\\n", HPM_F_TIMING_KINDS(1u << {i}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, what, val = line.split()
        if cname == "timing":
            assert hb.F_TIMING_KINDS(what) == int(val), line
            continue
        py = mirrors[cname]
        got = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), line


def test_status_strings():
    for code in range(0, -10, -1):
        assert hpm.status_string(code) not in ("", "unknown status")
    assert hpm.status_string(-42) == "unknown status"


def _check_order(p, order):
    k = p.k
    arcs = set(p.arcs())
    assert sorted(order) == list(range(k))            # Prop. 1: a permutation
    adj = lambda a, b: (a, b) in arcs or (b, a) in arcs
    assert adj(order[0], order[1])                    # positions 0,1 form a pattern arc
    for i in range(1, k):                             # every later position touches an earlier one
        assert any(adj(order[i], order[j]) for j in range(i))


def _sigma(p):
    indeg = np.bincount(p.dst, minlength=p.k)
    outdeg = np.bincount(p.src, minlength=p.k)
    return indeg + outdeg, outdeg


def test_plan_order_follows_structural_reordering():
    rng = np.random.default_rng(0)
    for _ in range(300):
        p = random_pattern(rng, kmin=2, kmax=12)
        order = hpm.plan_order(p, 1, 1)
        _check_order(p, order)
        tot, out = _sigma(p)
        # first position: best (total degree, out-degree), ties to the smaller id
        best = max(range(p.k), key=lambda v: (tot[v], out[v], -v))
        assert order[0] == best
        # whenever the last placed vertex has unplaced out-neighbours, the next
        # position is the best-ranked of them
        arcs = set(p.arcs())
        for i in range(1, p.k):
            u = order[i - 1]
            nbrs = [w for w in range(p.k) if (u, w) in arcs and w not in order[:i]]
            if nbrs:
                assert order[i] == max(nbrs, key=lambda v: (tot[v], out[v], -v))


def test_plan_order_repairs_non_adjacent_start():
    # l1..l4 -> s, l1 -> m, m -> p, m -> q: s ranks first but is a sink; the plain
    # rule would continue with m, which is not adjacent to s.
    s, l1, l2, l3, l4, m, pp, q = range(8)
    arcs = [(l1, s), (l2, s), (l3, s), (l4, s), (l1, m), (m, pp), (m, q)]
    p = make_pattern(8, arcs, 1, 1)
    order = hpm.plan_order(p, 1, 1)
    assert order[0] == s
    assert order[1] == l1
    _check_order(p, order)


def test_plan_order_no_reorder_keeps_ids():
    rng = np.random.default_rng(1)
    for _ in range(100):
        p = random_pattern(rng, kmin=2, kmax=10)
        order = hpm.plan_order(p, 1, 1, hpm.F_NO_REORDER)
        _check_order(p, order)
        assert order[0] == 0


@pytest.mark.parametrize("bad", [
    dict(k=1, arcs=[]),
    dict(k=17, arcs=[(i, i + 1) for i in range(16)]),
    dict(k=3, arcs=[(0, 0), (0, 1), (1, 2)]),
    dict(k=3, arcs=[(0, 1), (0, 1), (1, 2)]),
    dict(k=4, arcs=[(0, 1), (2, 3)]),
    dict(k=3, arcs=[(0, 1), (1, 5)]),
])
def test_plan_order_rejects_bad_patterns(bad):
    k = bad["k"]
    arcs = bad["arcs"] or [(0, 0)]
    p = make_pattern(max(k, 1), arcs, 1, 1)
    p.k = k
    with pytest.raises(hpm.HpmError) as ei:
        hpm.plan_order(p, 1, 1)
    assert ei.value.status == hb.E_PATTERN


def test_plan_order_rejects_bad_ops():
    p = motif("cycle3", vlabels=[0, 1, 2])
    p.vop[1, 0] = 7
    with pytest.raises(hpm.HpmError) as ei:
        hpm.plan_order(p, 1, 1)
    assert ei.value.status == hb.E_PATTERN


def test_graph_create_rejects_bad_offsets_on_host():
    lib = hpm.load()
    h = ctypes.c_void_p()
    nb = np.array([1, 0], dtype=np.int32)
    for off in ([0, 1, 0], [1, 1, 2], [0, 3, 2], [0, 1, 3]):
        o = np.array(off, dtype=np.int64)
        st = lib.hpm_graph_create(ctypes.byref(h), 2, 2, o.ctypes.data, nb.ctypes.data,
                                  o.ctypes.data, nb.ctypes.data, 0, None, 0, None, None)
        assert st == hb.E_GRAPH, off
    o = np.array([0, 1, 2], dtype=np.int64)
    assert lib.hpm_graph_create(None, 2, 2, o.ctypes.data, nb.ctypes.data, o.ctypes.data,
                                nb.ctypes.data, 0, None, 0, None, None) == hb.E_ARG
    assert lib.hpm_graph_create(ctypes.byref(h), 2, 1 << 31, o.ctypes.data, nb.ctypes.data,
                                o.ctypes.data, nb.ctypes.data, 0, None, 0, None,
                                None) == hb.E_UNSUPPORTED
    assert lib.hpm_graph_create(ctypes.byref(h), 2, 2, o.ctypes.data, nb.ctypes.data,
                                o.ctypes.data, nb.ctypes.data, 5, None, 0, None,
                                None) == hb.E_ARG


def test_match_rejects_null_arguments():
    lib = hpm.load()
    cnt = ctypes.c_uint64()
    p, keep = hb._pattern_struct(motif("cycle3"))
    assert lib.hpm_match(None, ctypes.byref(p), 0, None, None, ctypes.byref(cnt), None,
                         0) == hb.E_ARG


def test_server_entry_points_reject_null_arguments():
    # host-side argument checks only: no server is created without a graph
    lib = hpm.load()
    h = ctypes.c_void_p()
    assert lib.hpm_server_create(ctypes.byref(h), None, None) == hb.E_ARG
    assert lib.hpm_server_create(None, None, None) == hb.E_ARG
    p, keep = hb._pattern_struct(motif("cycle3"))
    t = ctypes.c_uint64()
    assert lib.hpm_server_submit(None, ctypes.byref(p), 0, None, 0, ctypes.byref(t)) == hb.E_ARG
    r = hb._QueryResult()
    assert lib.hpm_server_poll(None, 1, 0, ctypes.byref(r)) == hb.E_ARG
    s = hb._ServerStats()
    assert lib.hpm_server_read_stats(None, ctypes.byref(s)) == hb.E_ARG
    assert lib.hpm_server_destroy(None) == hb.OK
    assert lib.hpm_match_batch(None, 0, None, None, None, None, 0, None, None) == hb.E_ARG
    assert lib.hpm_batch_tune(None, 1, None, None, None, None, None, None) == hb.E_ARG


def test_motif_orders_are_valid():
    for name, (k, arcs) in MOTIFS.items():
        p = make_pattern(k, arcs, 1, 1)
        assert is_weakly_connected(k, arcs)
        _check_order(p, hpm.plan_order(p, 1, 1))


def test_persistent_batch_entry_points_are_switched_off():
    # the persistent batched launch stalled on the device; its entry points
    # refuse to run before touching any argument or the device
    lib = hpm.load()
    assert lib.hpm_match_batch_persistent(None, 0, None, None, None, None, None, None,
                                          None) == hpm.hpm.E_UNSUPPORTED
    assert lib.hpm_batch_autotune(None, 0, None, None, None, None, None, None) == \
        hpm.hpm.E_UNSUPPORTED
    assert "switched off" in lib.hpm_last_error().decode()
