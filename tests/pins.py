"""Independent checks for the oracle: brute force and closed-form counts.

Nothing here shares code with oracle/ or with the library.  Each function is
derived from the problem definition (Sec. II-A, Eq. (1)-(3) and the
monomorphism relaxation) or from a classical counting identity, written in a
different style (dense matrices, whole-map enumeration) so that a slip in the
oracle's backtracking (a dropped check, a reversed arc, a wrong index) shows up
as a disagreement.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def dense_adj(g) -> np.ndarray:
    """n x n 0/1 matrix with A[u,v] = 1 iff u->v is an arc."""
    A = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    A[src, g.out_nbrs] = 1
    return A


def dense_ecol(g, col=0) -> np.ndarray:
    """n x n matrix holding the attribute of arc u->v at [u,v] (0 where no arc)."""
    E = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    E[src, g.out_nbrs] = g.ecols[col]
    return E


def _ok(op, val, x):
    return op == 0 or (op == 1 and x == val) or (op == 2 and x >= val)


def brute(g, p, mode):
    """Every injective map checked against the definition; returns sorted rows.

    Enumerates all k-permutations of the target vertices, so keep n <= 9.
    """
    A = dense_adj(g)
    Es = [dense_ecol(g, c) for c in range(len(g.ecols))]
    arcs = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(p.src, p.dst))}
    vcols = [np.asarray(c) for c in g.vcols]
    rows = []
    for f in itertools.permutations(range(g.n), p.k):
        good = True
        for a in range(p.k):
            for c, vc in enumerate(vcols):
                if not _ok(p.vop[a, c], p.vval[a, c], vc[f[a]]):
                    good = False
                    break
            if not good:
                break
        if not good:
            continue
        for a in range(p.k):
            for b in range(p.k):
                if a == b:
                    continue
                has = A[f[a], f[b]] == 1
                i = arcs.get((a, b))
                if i is not None:
                    if not has or not all(_ok(p.eop[i, c], p.eval[i, c], Es[c][f[a], f[b]])
                                          for c in range(len(Es))):
                        good = False
                elif mode == 0 and has:
                    good = False
                if not good:
                    break
            if not good:
                break
        if good:
            rows.append(f)
    return np.array(sorted(rows), dtype=np.int32).reshape(-1, p.k)


# ------------------------------------------------------------ closed forms

def trace_cycle3(g, vlab, elab, mode) -> int:
    """Embeddings of the directed 3-cycle 0->1->2->0 with vertex labels vlab
    (EQ on column 0) and every arc EQ elab on column 0.

    With D_x the diagonal indicator of vertex label x and L the adjacency
    restricted to arcs of label elab, the count is tr(D0 M D1 M D2 M) where
    M = L for monomorphism and M = L o (1 - A^T) for induced isomorphism
    (a 3-cycle's only non-arcs are the three reverse arcs).  Distinct images
    are automatic: a self-loop-free graph has no closed walk of length 3
    through a repeated vertex.
    """
    import scipy.sparse as sp
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    A = sp.csr_matrix((np.ones(g.m, dtype=np.int64), (src, g.out_nbrs)), shape=(g.n, g.n))
    keep = (np.asarray(g.ecols[0]) == elab).astype(np.int64)
    L = sp.csr_matrix((keep, (src, g.out_nbrs)), shape=(g.n, g.n))
    L.eliminate_zeros()
    M = L if mode == 1 else L - L.multiply(A.T)
    lab = np.asarray(g.vcols[0])
    D = [sp.diags((lab == x).astype(np.int64)) for x in vlab]
    B = D[0] @ M @ D[1] @ M @ D[2]
    return int(B.multiply(M.T).sum())


def moon_cycle3(outdeg: np.ndarray) -> int:
    """Embeddings of the induced directed 3-cycle in a tournament: three per
    cyclic triple, and the cyclic triples number C(n,3) - sum_i C(s_i, 2)
    (Moon 1968) with s_i the out-degrees."""
    n = len(outdeg)
    return 3 * (math.comb(n, 3) - sum(math.comb(int(s), 2) for s in outdeg))


def falling(x: int, k: int) -> int:
    out = 1
    for i in range(k):
        out *= (x - i)
    return out


def out_star_mono(g, k_leaves, centre_pred, leaf_pred, arc_pred) -> int:
    """Monomorphisms of the out-star centre->leaf_1..leaf_k (all leaves share
    one predicate): sum over admissible centres v of (c_v)_k where c_v counts
    out-neighbours w with leaf_pred(w) and arc_pred on v->w."""
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    lab = np.asarray(g.vcols[0])
    el = np.asarray(g.ecols[0])
    ok = leaf_pred(lab[g.out_nbrs]) & arc_pred(el)
    c = np.bincount(src[ok], minlength=g.n)
    total = 0
    for v in np.flatnonzero(centre_pred(lab)):
        total += falling(int(c[v]), k_leaves)
    return total


def two_path_mono(g) -> int:
    """Unlabelled monomorphisms of a->b->c: sum_b in(b)*out(b) - recip(b),
    removing the walks u->b->u that revisit u."""
    A = dense_adj(g) if g.n <= 4000 else None
    indeg = np.diff(g.in_off)
    outdeg = np.diff(g.out_off)
    if A is not None:
        recip = (A * A.T).sum(axis=1)
    else:
        src = np.repeat(np.arange(g.n, dtype=np.int64), outdeg)
        keys = src * g.n + g.out_nbrs
        rev = g.out_nbrs.astype(np.int64) * g.n + src
        pos = np.searchsorted(keys, rev)
        pos[pos >= keys.shape[0]] = 0
        recip = np.bincount(src[keys[pos] == rev], minlength=g.n)
    return int((indeg.astype(np.int64) * outdeg - recip).sum())


def all_supergraphs(k, arcs):
    """Every arc set on k vertices (no loops) that contains `arcs`."""
    base = set(arcs)
    rest = [(a, b) for a in range(k) for b in range(k) if a != b and (a, b) not in base]
    for r in range(len(rest) + 1):
        for extra in itertools.combinations(rest, r):
            yield sorted(base) + list(extra)


def bipartite_k2_mono(g, s, target_labels, arc_ge):
    """Monomorphisms of the complete bipartite pattern with s sources and two
    targets (every source -> both targets), sources unlabelled, target t
    (t = 0, 1) restricted to vertex label target_labels[t] on column 0 (None:
    any), every arc GE arc_ge on arc column 0.

    Writing c(y, z) for the number of common in-neighbours x of y and z whose
    arcs x->y and x->z both pass the arc predicate, the count is the sum over
    ordered pairs y != z of admissible targets of the falling factorial
    c(y, z) (c(y, z) - 1) ... (c(y, z) - s + 1): the s sources are distinct
    common in-neighbours, and they differ from y and z because the graph has
    no self-loops.  c is the sparse product B_y^T B_z of the filtered
    adjacency restricted to each target's admissible columns.
    """
    import scipy.sparse as sp
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.out_off))
    ok = np.asarray(g.ecols[0]) >= arc_ge
    A = sp.csc_matrix((np.ones(int(ok.sum()), dtype=np.int64), (src[ok], g.out_nbrs[ok])),
                      shape=(g.n, g.n))
    lab = np.asarray(g.vcols[0])
    cols = [np.flatnonzero(lab == t) if t is not None else np.arange(g.n) for t in target_labels]
    C = (A[:, cols[0]].T @ A[:, cols[1]]).tocoo()
    c = C.data.astype(np.int64)
    keep = cols[0][C.row] != cols[1][C.col]
    c = c[keep]
    total = np.ones_like(c)
    for i in range(s):
        total = total * (c - i)
    return int(total.sum())
