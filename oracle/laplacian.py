"""Graph Laplacian of a submesh, in FP64.  Test infrastructure only.

Paper, Section 3: a triangle mesh M = (V, F); the edge set E follows from the
faces; L = D - C (Eq. 1) with C_ij = 1/||v_i - v_j||^2 on edges (Eq. 2) and
D diagonal.  The binary-connectivity variant uses C = adjacency.

Readings (listed in the design notes):
  * Eq. 2 with D_ii = |N(i)| (a count) does not give a Laplacian when C is
    weighted (rows would not sum to zero).  The weighted mode therefore uses
    D_ii = sum_j C_ij.  For binary C the two coincide, which is the paper's
    combinatorial L = D - A.
  * A submesh is the subgraph induced by its vertices: every mesh edge with
    both ends in the block.  Face corners outside the block are marked -1 and
    the edges touching them are dropped.
  * Self-loops (a repeated corner) are dropped, duplicate edges merged, an
    isolated vertex keeps a stored zero diagonal.
"""
from __future__ import annotations

import numpy as np

COMBINATORIAL = 0
INV_SQ_DIST = 1
USER = 2
INV_DIST = 3


class IndexError_(ValueError):
    """A primitive references a vertex id outside [-1, n)."""


class DegenerateError(ValueError):
    """A zero-length edge under a distance-based weight."""


def canonical_edges(prims: np.ndarray, n: int) -> np.ndarray:
    """Edges (i, j), i < j, of the primitives (faces of 3 corners or edges of
    2), sorted lexicographically and unique.  Corner -1 = outside the block."""
    prims = np.asarray(prims, dtype=np.int64)
    if prims.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    if (prims < -1).any() or (prims >= n).any():
        raise IndexError_("primitive index out of range")
    k = prims.shape[1]
    pairs = []
    if k == 2:
        pairs.append(prims)
    else:
        for a in range(k):
            pairs.append(prims[:, [a, (a + 1) % k]])
    e = np.concatenate(pairs)
    e = e[(e[:, 0] >= 0) & (e[:, 1] >= 0) & (e[:, 0] != e[:, 1])]
    e = np.sort(e, axis=1)
    if e.shape[0] == 0:
        return np.zeros((0, 2), dtype=np.int64)
    e = np.unique(e, axis=0)  # lexicographic order
    return e


def edge_weights(edges: np.ndarray, coords, mode: int, user_w=None) -> np.ndarray:
    """Off-diagonal weights C_ij per canonical edge (Eq. 2), in FP64."""
    m = edges.shape[0]
    if mode == COMBINATORIAL:
        return np.ones(m)
    if mode == USER:
        w = np.asarray(user_w, dtype=np.float64)
        assert w.shape == (m,)
        return w.copy()
    X = np.asarray(coords, dtype=np.float64)
    d2 = ((X[edges[:, 0]] - X[edges[:, 1]]) ** 2).sum(axis=1)
    if (d2 == 0).any():
        raise DegenerateError("zero-length edge")
    if mode == INV_SQ_DIST:
        return 1.0 / d2
    if mode == INV_DIST:
        return 1.0 / np.sqrt(d2)
    raise ValueError("unknown weight mode")


def laplacian_dense(n: int, edges: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Dense L = D - C with D_ii = sum_j C_ij (Eq. 1)."""
    L = np.zeros((n, n))
    i, j = edges[:, 0], edges[:, 1]
    np.add.at(L, (i, j), -w)
    np.add.at(L, (j, i), -w)
    np.add.at(L, (i, i), w)
    np.add.at(L, (j, j), w)
    return L


def laplacian_csr(n: int, edges: np.ndarray, w: np.ndarray):
    """CSR of L with the diagonal always stored and columns ascending.
    Returns (row_ptr int64 [n+1], col int64 [nnz], val float64 [nnz])."""
    rows = [[] for _ in range(n)]
    diag = np.zeros(n)
    for (i, j), wij in zip(edges.tolist(), w.tolist()):
        rows[i].append((j, -wij))
        rows[j].append((i, -wij))
        diag[i] += wij
        diag[j] += wij
    row_ptr = [0]
    col = []
    val = []
    for i in range(n):
        ent = rows[i] + [(i, diag[i])]
        ent.sort(key=lambda t: t[0])
        for j, v in ent:
            col.append(j)
            val.append(v)
        row_ptr.append(len(col))
    return (np.asarray(row_ptr, dtype=np.int64), np.asarray(col, dtype=np.int64),
            np.asarray(val, dtype=np.float64))


def csr_to_dense(n, row_ptr, col, val):
    L = np.zeros((n, n))
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            L[i, col[k]] += val[k]
    return L


def laplacian_literal_mixed(n: int, edges: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Eq. 1-2 read literally: D_ii = |N(i)| (neighbour count) with weighted
    C.  Diagnostic only (rows do not sum to zero when C is weighted)."""
    L = np.zeros((n, n))
    i, j = edges[:, 0], edges[:, 1]
    np.add.at(L, (i, j), -w)
    np.add.at(L, (j, i), -w)
    np.add.at(L, (i, i), 1.0)
    np.add.at(L, (j, j), 1.0)
    return L


def block_laplacian(faces, coords, mode=COMBINATORIAL, user_w=None):
    """Convenience: (edges, weights, dense L) of one block."""
    n = np.asarray(coords).shape[0]
    e = canonical_edges(faces, n)
    w = edge_weights(e, coords, mode, user_w)
    return e, w, laplacian_dense(n, e, w)
