"""Reconstruction-quality metrics and the choice of c, FP64.  Test
infrastructure only.

Section 8, Eq. 16 (NMSVE) as printed, read literally:
    NMSVE = ( ||v - v~||_2 + ||GL(v) - GL(v~)||_2 ) / (2n)
over the 3n-vector of coordinates, with
    GL(v_i) = v_i - (sum_{j in N(i)} d_ij^-1 v_j) / (sum_{j in N(i)} d_ij^-1)
Reading: d_ij are the Euclidean edge lengths of the ORIGINAL mesh for both
GL(v) and GL(v~), which makes GL a fixed linear operator (GL(v~) with the
reconstruction's own distances is undefined when reconstructed vertices
coincide).  dB = 10 log10.

Section 5, Eq. 6: the DOI residual e = sum_{j in x,y,z} (v_j - U U^T v_j).

Section 8 (theta): the angle between the normal of every face of the
original mesh and the normal of the same face of the reconstruction,
averaged over all faces, in degrees (the unit of the paper's table of
theta values).  Reading: a face whose normal vanishes on either side (zero
area) has no direction and is left out of the average.

Choice of c (Section 5: smallest subspace meeting a quality constraint):
smallest c in [1, c_max] with NMSVE(c) <= target (c_max if none), then moved
up to the first cut with a relative spectral gap
(lambda_{c+1} - lambda_c) / lambda_{c+1} >= g_min, so the kept subspace is
well defined (reading; the paper is silent on near-ties).
"""
from __future__ import annotations

import math

import numpy as np

from . import laplacian as lap


def gl_matrix(n: int, edges: np.ndarray, coords0: np.ndarray) -> np.ndarray:
    """Dense GL operator: G = I - D_d^-1 A_d, A_d the 1/d_ij adjacency of the
    original mesh, D_d its row sums.  Rows of isolated vertices are identity."""
    w = lap.edge_weights(edges, coords0, lap.INV_DIST)
    A = np.zeros((n, n))
    A[edges[:, 0], edges[:, 1]] = w
    A[edges[:, 1], edges[:, 0]] = w
    d = A.sum(1)
    G = np.eye(n)
    nz = d > 0
    G[nz] -= A[nz] / d[nz, None]
    return G


def nmsve(X: np.ndarray, Xr: np.ndarray, G: np.ndarray) -> float:
    """Eq. 16 (literal reading above)."""
    n = X.shape[0]
    a = np.linalg.norm(X - Xr)
    b = np.linalg.norm(G @ X - G @ Xr)
    return float((a + b) / (2.0 * n))


def nmsve_db(x: float) -> float:
    return float(10.0 * np.log10(x))


def gl_apply(n: int, edges: np.ndarray, coords0: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """G Y for the GL operator of gl_matrix, one edge at a time (sparse, for
    whole meshes): row i gets Y_i - sum_j w_ij Y_j / sum_j w_ij, w = 1/d_ij of
    the original mesh; rows without neighbours are left unchanged."""
    w = lap.edge_weights(edges, coords0, lap.INV_DIST)
    Y = np.asarray(Y, dtype=np.float64)
    num = np.zeros_like(Y)
    den = np.zeros(n)
    i, j = edges[:, 0], edges[:, 1]
    np.add.at(num, i, w[:, None] * Y[j])
    np.add.at(num, j, w[:, None] * Y[i])
    np.add.at(den, i, w)
    np.add.at(den, j, w)
    out = Y.copy()
    nz = den > 0
    out[nz] -= num[nz] / den[nz, None]
    return out


def nmsve_mesh(n: int, edges: np.ndarray, X: np.ndarray, Xr: np.ndarray) -> float:
    """Eq. 16 over a whole mesh given by its edge list, with the GL weights
    of the original coordinates X (literal reading above)."""
    X = np.asarray(X, dtype=np.float64)
    Xr = np.asarray(Xr, dtype=np.float64)
    a = np.linalg.norm(X - Xr)
    b = np.linalg.norm(gl_apply(n, edges, X, X) - gl_apply(n, edges, X, Xr))
    return float((a + b) / (2.0 * n))


def mean_normal_angle(faces: np.ndarray, X: np.ndarray, Xr: np.ndarray):
    """theta of Section 8: the mean over faces of the angle, in degrees,
    between the face normal (v1 - v0) x (v2 - v0) of X and of Xr.  Returns
    (theta, number of faces averaged); faces with a zero normal on either
    side are skipped."""
    X = np.asarray(X, dtype=np.float64)
    Xr = np.asarray(Xr, dtype=np.float64)
    total, used = 0.0, 0
    for a, b, c in np.asarray(faces):
        no = np.cross(X[b] - X[a], X[c] - X[a])
        nr = np.cross(Xr[b] - Xr[a], Xr[c] - Xr[a])
        lo, lr = np.linalg.norm(no), np.linalg.norm(nr)
        if lo == 0.0 or lr == 0.0:
            continue
        cosang = min(1.0, max(-1.0, float(no @ nr) / (lo * lr)))
        total += math.degrees(math.acos(cosang))
        used += 1
    return (total / used if used else 0.0), used


def nmsve_curve(U: np.ndarray, X: np.ndarray, G: np.ndarray, c_max: int) -> np.ndarray:
    """NMSVE(c) for c = 1..c_max, each by an explicit reconstruction with the
    first c columns of U (brute force)."""
    out = np.empty(c_max)
    for c in range(1, c_max + 1):
        Uc = U[:, :c]
        out[c - 1] = nmsve(X, Uc @ (Uc.T @ X), G)
    return out


def nmsve_curve_sparse(U: np.ndarray, X: np.ndarray, edges: np.ndarray, coords0: np.ndarray,
                       c_max: int) -> np.ndarray:
    """NMSVE(c) for c = 1..c_max by explicit reconstructions, with the GL
    operator applied edge by edge (gl_apply) instead of as a dense matrix,
    for blocks too large for gl_matrix: GL is linear (original distances),
    so GL(U_c E_c) = GL(U_c) E_c and GL(U) is formed once."""
    n = X.shape[0]
    X = np.asarray(X, dtype=np.float64)
    GX = gl_apply(n, edges, coords0, X)
    GU = gl_apply(n, edges, coords0, U[:, :c_max])
    out = np.empty(c_max)
    for c in range(1, c_max + 1):
        E = U[:, :c].T @ X
        a = np.linalg.norm(X - U[:, :c] @ E)
        b = np.linalg.norm(GX - GU[:, :c] @ E)
        out[c - 1] = (a + b) / (2.0 * n)
    return out


def l2_residual_curve(U: np.ndarray, X: np.ndarray, c_max: int) -> np.ndarray:
    """||X - U_c U_c^T X||_F for c = 1..c_max, brute force."""
    return np.array([np.linalg.norm(X - U[:, :c] @ (U[:, :c].T @ X)) for c in range(1, c_max + 1)])


def choose_c(curve: np.ndarray, lam: np.ndarray, target: float, g_min: float) -> int:
    """Smallest c with curve[c-1] <= target (len(curve) if none), then snapped
    up to the first c whose relative gap to lambda_{c+1} is >= g_min (never
    beyond len(curve))."""
    c_max = curve.size
    ok = np.nonzero(curve <= target)[0]
    c = int(ok[0]) + 1 if ok.size else c_max
    while c < c_max and c < lam.size:
        if (lam[c] - lam[c - 1]) >= g_min * abs(lam[c]):
            break
        c += 1
    return c


def doi_residual(U: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Eq. 6: e = sum over x, y, z of (v_j - U U^T v_j); an n-vector."""
    R = X - U @ (U.T @ X)
    return R.sum(axis=1)
