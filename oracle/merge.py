"""Merge of overlapped submeshes, in FP64.  Test infrastructure only.

Paper, Section 6.1 and its weighted-average algorithm (Alg. 3): a mesh
vertex that lies in several overlapped submeshes gets, as its final
position, the average of its reconstructions in those submeshes, each
weighted by the vertex's degree (its number of neighbours) in that
submesh.

Readings (listed in the design notes):
  * "Degree in the submesh" is the number of neighbours of the vertex in
    the submesh's graph: the subgraph induced by the submesh's vertices,
    i.e. the off-diagonal entries of its row of the submesh Laplacian.
  * The paper does not say what happens when every weight of a vertex is
    zero (the vertex is isolated in every submesh that holds it); the
    merge then takes the plain mean of its reconstructions.  A vertex in
    no submesh gets the position 0.
  * The sums run over the submeshes in ascending index, in FP64; the
    result is rounded to FP32 once, at the end.
"""
from __future__ import annotations

import numpy as np

from .laplacian import canonical_edges


def submesh_degrees(faces: np.ndarray, n: int) -> np.ndarray:
    """Number of neighbours of every vertex of a submesh (faces in local
    ids, -1 = corner outside), from the submesh's edge set (Section 3)."""
    e = canonical_edges(faces, n)
    deg = np.zeros(n, dtype=np.int64)
    for i, j in e:
        deg[i] += 1
        deg[j] += 1
    return deg


def weighted_average(n_vertices: int, global_ids: list, degrees: list, X_blocks: list) -> np.ndarray:
    """Alg. 3: for every mesh vertex, find the submeshes that contain it and
    return sum_j w_ij v_ij / sum_j w_ij over them (FP64 sums, FP32 result).

    global_ids[j][k] is the mesh vertex of row k of submesh j, degrees[j][k]
    its degree there and X_blocks[j][k] its reconstructed position."""
    occ = [[] for _ in range(n_vertices)]
    for j, gid in enumerate(global_ids):
        for k, g in enumerate(gid):
            occ[int(g)].append((j, k))
    out = np.zeros((n_vertices, 3), dtype=np.float64)
    for i in range(n_vertices):
        if not occ[i]:
            continue
        sumv = np.zeros(3, dtype=np.float64)
        sumw = 0.0
        for j, k in occ[i]:  # ascending submesh index
            w = float(degrees[j][k])
            sumv = sumv + w * np.asarray(X_blocks[j][k], dtype=np.float64)
            sumw = sumw + w
        if sumw > 0.0:
            out[i] = sumv / sumw
        else:
            s = np.zeros(3, dtype=np.float64)
            for j, k in occ[i]:
                s = s + np.asarray(X_blocks[j][k], dtype=np.float64)
            out[i] = s / float(len(occ[i]))
    return out.astype(np.float32)
