"""Eigendecomposition, graph Fourier transform and subspace comparison, FP64.
Test infrastructure only.

Paper, Section 3: L = U Lambda U^T (Eq. 3); the eigenvalues are graph
frequencies; the GFT of the coordinates is v_bar = U^T v and the inverse GFT
v = U v_bar.  Section 4: the block tracks U_c, the eigenvectors of the c
lowest eigenvalues.  Section 7.1: encode E = U_c^T v, decode v~ = U_c E.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def eigh_lowest(L: np.ndarray, k: int | None = None):
    """Ascending eigenpairs of the dense symmetric L (LAPACK).  With k, only
    the k lowest (subset driver for large blocks)."""
    n = L.shape[0]
    if k is None or k >= n:
        lam, U = np.linalg.eigh(L)
        return lam, U
    lam, U = scipy.linalg.eigh(L, subset_by_index=[0, k - 1], driver="evr")
    return lam, U


def project(U: np.ndarray, X: np.ndarray) -> np.ndarray:
    """GFT coefficients E = U^T X (Section 3; feature vectors of Section 5)."""
    return U.T @ X


def reconstruct(U: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Inverse GFT X~ = U E (Section 3, Section 7.1)."""
    return U @ E


def encode_decode(U_c: np.ndarray, X: np.ndarray) -> np.ndarray:
    """v^ = U_c U_c^T v (Section 7.2)."""
    return reconstruct(U_c, project(U_c, X))


def orthonormalize(A: np.ndarray) -> np.ndarray:
    """Orthonormal basis of span(A) by Householder QR."""
    q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    return q


def principal_angles(U_ref: np.ndarray, U_test: np.ndarray) -> np.ndarray:
    """Principal angles (ascending) between span(U_ref) and span(U_test), via
    the singular values of Q_ref^T Q_test.  Small angles are taken from
    ||(I - Q_ref Q_ref^T) Q_test|| singular values for accuracy."""
    Qr = orthonormalize(U_ref)
    Qt = orthonormalize(U_test)
    R = Qt - Qr @ (Qr.T @ Qt)
    s = np.linalg.svd(R, compute_uv=False)
    s = np.clip(s, 0.0, 1.0)
    return np.sort(np.arcsin(s))


def sin_theta_max(U_ref: np.ndarray, U_test: np.ndarray) -> float:
    """sin of the largest principal angle = ||(I - Q_ref Q_ref^T) Q_test||_2."""
    Qr = orthonormalize(U_ref)
    Qt = orthonormalize(U_test)
    R = Qt - Qr @ (Qr.T @ Qt)
    return float(np.linalg.norm(R, 2)) if R.size else 0.0


def rel_error(A: np.ndarray, B_ref: np.ndarray) -> float:
    den = np.linalg.norm(B_ref)
    return float(np.linalg.norm(np.asarray(A, np.float64) - B_ref) / (den if den > 0 else 1.0))


def gap_at(lam: np.ndarray, c: int) -> float:
    """Spectral gap lambda_{c+1} - lambda_c (1-based c)."""
    return float(lam[c] - lam[c - 1]) if c < lam.size else float("inf")


def fp32_floor(lam: np.ndarray, c: int, p: int | None = None) -> float:
    """Rough FP32 accuracy floor of a tracked c-subspace (Davis-Kahan):
    u32 * lambda_p / gap_c, with u32 = 2^-24."""
    g = gap_at(lam, c)
    top = lam[min((p or c), lam.size) - 1]
    return float(2.0 ** -24 * max(top, 1e-30) / g) if g > 0 else float("inf")


def sign_fix(U: np.ndarray) -> np.ndarray:
    """Sign rule for comparing individual eigenvectors: the entry of largest
    magnitude is positive (lowest index on ties)."""
    U = np.array(U, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1
    return U * s[None, :]
