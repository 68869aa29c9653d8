"""hpm_match_noalloc against hpm_match (GPU; through the C ABI).

Two calls in a row on the allocation-free entry point, the second with a
smaller input, each compared with hpm_match on the same input: the count
exactly and the sorted mapping rows bit-exact.  The calls leave the device's
free memory unchanged, a caller budget below the fixed part fails with
HPM_E_NOMEM, and a short output buffer gives HPM_E_TRUNCATED with the count.
"""
import sys

import numpy as np
import pytest

import paper_2507_04130_amd as hpm
from synth import configs
from synth.patterns import ISO, MONO, motif

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lexsorted(rows):
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] else rows


def test_noalloc_equals_match_on_two_calls():
    import torch
    big = configs.c2_graph(scale=12)
    small = configs.c2_graph(scale=10)
    dbig, dsmall = hpm.Graph.from_host(big), hpm.Graph.from_host(small)
    cases = [(dbig, motif("ffl_tail"), ISO, "rmat12 ffl_tail iso"),
             (dsmall, motif("cycle3"), MONO, "rmat10 cycle3 mono")]
    want, outs = [], []
    for d, p, mode, name in cases:
        cnt, rows = hpm.match(d, p, mode, mappings=True)
        want.append((cnt, lexsorted(rows.cpu().numpy())))
        outs.append(torch.empty((max(cnt, 1) + 5, p.k), dtype=torch.int32, device="cuda"))
        say(f"{name}: hpm_match count {cnt}")
    assert want[0][0] > want[1][0] > 0
    # set-up: the first call on the device resolves its scratch array
    hpm.match_noalloc(dsmall, motif("cycle3"), MONO)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = []
    for (d, p, mode, name), out in zip(cases, outs):
        cnt, rows = hpm.match_noalloc(d, p, mode, out=out)
        c_only, _ = hpm.match_noalloc(d, p, mode)
        got.append((cnt, c_only, lexsorted(rows.cpu().numpy())))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "an allocation-free call allocated"
    for (cnt, c_only, rows), (wcnt, wrows), (_, _, _, name) in zip(got, want, cases):
        say(f"{name}: hpm_match_noalloc count {cnt}")
        assert cnt == c_only == wcnt, name
        np.testing.assert_array_equal(rows, wrows, err_msg=name)
    # a budget below the fixed part of the call's scratch
    with pytest.raises(hpm.HpmError) as e:
        hpm.match_noalloc(dbig, motif("ffl_tail"), ISO, budget=1024)
    assert e.value.status == hpm.hpm.E_NOMEM
    # a short output buffer: truncated
    short = torch.empty((1, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(hpm.HpmError) as e:
        hpm.match_noalloc(dsmall, motif("cycle3"), MONO, out=short)
    assert e.value.status == hpm.hpm.E_TRUNCATED
    # the regular entry point still works after the allocation-free ones
    assert hpm.match(dsmall, motif("cycle3"), MONO)[0] == want[1][0]
    dsmall.close()
    dbig.close()
