"""Seeded generators: determinism and structural invariants (CPU only)."""
import numpy as np
import pytest

from synth.graphs import (connectome, erdos_renyi, reciprocal_fraction, rmat, zipf_probs)
from synth.patterns import MOTIFS, is_weakly_connected, random_pattern


def _check_simple_csr(g):
    assert g.out_off[0] == 0 and g.out_off[-1] == g.m
    assert g.in_off[0] == 0 and g.in_off[-1] == g.m
    src = g.src()
    assert np.all(src != g.out_nbrs), "self-loop"
    keys = src.astype(np.int64) * g.n + g.out_nbrs
    assert np.all(np.diff(keys) > 0), "rows not strictly ascending / duplicates"
    # in-CSR is the transpose
    dst = np.repeat(np.arange(g.n), np.diff(g.in_off))
    tkeys = np.sort(g.in_nbrs.astype(np.int64) * g.n + dst)
    np.testing.assert_array_equal(tkeys, keys)
    for c in g.vcols:
        assert c.shape == (g.n,) and c.dtype == np.int32
    for c in g.ecols:
        assert c.shape == (g.m,) and c.dtype == np.int32


@pytest.mark.parametrize("fn", [
    lambda: erdos_renyi(1000, 5000, 101),
    lambda: rmat(12, 1 << 15, 7),
    lambda: connectome(50_000, 300_000, 3),
])
def test_deterministic_and_simple(fn):
    a, b = fn(), fn()
    assert a.sha256() == b.sha256()
    _check_simple_csr(a)


def test_er_shape():
    g = erdos_renyi(1000, 5000, 101)
    assert g.n == 1000 and g.m == 5000
    assert set(np.unique(g.vcols[0])) <= {0, 1, 2, 3}
    assert set(np.unique(g.ecols[0])) <= {0, 1}


def test_rmat_labels_and_skew():
    g = rmat(14, 1 << 18, 11)
    assert g.m == 1 << 18
    p = zipf_probs(1.2, 16)
    assert abs(p[0] - 0.365) < 0.002
    hist = np.bincount(g.vcols[0], minlength=16) / g.n
    assert np.abs(hist - p).max() < 0.02
    deg = np.diff(g.out_off) + np.diff(g.in_off)
    assert deg.max() > 20 * deg.mean()          # heavy-tailed


def test_connectome_reciprocity_and_weights():
    g = connectome(200_000, 1_500_000, 4)
    assert abs(g.m - 1_500_000) < 15_000
    assert abs(reciprocal_fraction(g) - 0.30) < 0.005
    w = g.ecols[0]
    assert w.min() >= 1
    assert abs((w >= 10).mean() - 0.116) < 0.01
    assert set(np.unique(g.vcols[0])) <= set(range(8))


def test_motifs_connected():
    for name, (k, arcs) in MOTIFS.items():
        assert is_weakly_connected(k, arcs), name
        assert len(set(arcs)) == len(arcs)
        assert all(a != b for a, b in arcs)


def test_random_patterns():
    rng = np.random.default_rng(201)
    for _ in range(200):
        p = random_pattern(rng)
        assert 3 <= p.k <= 8
        arcs = p.arcs()
        assert len(set(arcs)) == len(arcs)
        assert all(a != b for a, b in arcs)
        assert is_weakly_connected(p.k, arcs)


def test_connectome_independent_of_thread_count():
    a = connectome(40_000, 300_000, 9, threads=1)
    b = connectome(40_000, 300_000, 9, threads=5)
    assert a.sha256() == b.sha256()
