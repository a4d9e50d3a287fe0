"""Subspace iterations in FP64.  Test infrastructure only.

paper_oi        Algorithm 1 as the paper states it: U(t) = Onorm(R^z U(t-1)),
                R = (L + delta I)^-1, Onorm = Householder QR keeping the first
                c columns (Section 4, Eq. 4-5).  Used to show that the paper's
                iteration and the GPU's filtered iteration approach the same
                eigenspace, and to measure the rate |lambda_{c+1}/lambda_c|^z
                of R quoted in Section 4.
paper_doi       Algorithm 2 (dynamic OI, Section 5) with the branch reading
                of the text (grow c when the residual of Eq. 6 is above
                eps_h, shrink when below eps_l), bounded iterations.
doi_chebyshev   the same walk with the operator of the tracking path: each
                iteration applies `passes` degree-m Chebyshev filters on a
                fixed interval [a, b] in place of R^z, then Onorm.
chebyshev_span  the exact subspace span(f(L)^T V0) reached by T outer
                iterations that each apply the degree-m Chebyshev polynomial
                of the first kind on the damped interval [a, b]; the
                re-orthonormalisations and Rayleigh-Ritz rotations between
                applications do not change the span, so this is the
                iterate's reference *before* convergence.
rayleigh_ritz   eigenpairs of V^T L V for an orthonormal V, ascending.
ritz_residuals  r_j = || L v_j - theta_j v_j ||_2 of Ritz pairs, the accuracy
                measure of the iteration count question of Section 4 (how
                many iterations a block needs).
"""
from __future__ import annotations

import numpy as np

from .metrics import doi_residual


def householder_onorm(Y: np.ndarray, c: int) -> np.ndarray:
    """Eq. 4-5: QR of Y by Householder reflections (LAPACK geqrf via numpy),
    keep the first c columns of Q."""
    q, r = np.linalg.qr(Y)
    return q[:, :c]


def paper_oi(L: np.ndarray, U0: np.ndarray, z: int, delta: float, t_max: int,
             history: list | None = None) -> np.ndarray:
    """Algorithm 1 with R = (L + delta I)^-1 formed densely and applied z
    times per iteration."""
    n, c = U0.shape
    R = np.linalg.inv(L + delta * np.eye(n))
    U = U0
    for _ in range(t_max):
        Y = U
        for _ in range(z):
            Y = R @ Y
        U = householder_onorm(Y, c)
        if history is not None:
            history.append(U)
    return U


def dynamic_oi(apply_op, U0: np.ndarray, X: np.ndarray, eps_l: float, eps_h: float,
               c_max: int, t_max: int):
    """Algorithm 2 (dynamic OI) with the text's branch reading, for an
    operator apply_op (Y = op(U)): U(t) = Onorm(op(U(t-1))); e(t) of Eq. 6;
    if ||e|| is above eps_h (and c < c_max) append e/||e|| as a new column
    (Eq. 7), the next iteration's Onorm orthonormalises it; if below eps_l
    (and c > 1) keep the first c - 1 columns; otherwise stop.  After t_max
    iterations the walk stops where it is.  Returns (U, c, trajectory of
    (c, ||e||) before each decision)."""
    U = U0.copy()
    traj = []
    for _ in range(t_max):
        U = householder_onorm(apply_op(U), U.shape[1])
        e = doi_residual(U, X)
        ne = float(np.linalg.norm(e))
        traj.append((U.shape[1], ne))
        if ne > eps_h and U.shape[1] < c_max and ne > 0:
            U = np.concatenate([U, (e / ne)[:, None]], axis=1)
        elif ne < eps_l and U.shape[1] > 1:
            U = U[:, :-1]
        else:
            break
    return U, U.shape[1], traj


def paper_doi(L: np.ndarray, U0: np.ndarray, X: np.ndarray, z: int, delta: float,
              eps_l: float, eps_h: float, c_max: int, t_max: int = 200):
    """Algorithm 2 with the paper's operator R^z, R = (L + delta I)^-1.
    The basis returned is orthonormal (a column appended by the last
    decision is orthonormalised once more)."""
    n = L.shape[0]
    R = np.linalg.inv(L + delta * np.eye(n))

    def op(U):
        Y = U
        for _ in range(z):
            Y = R @ Y
        return Y

    U, c, traj = dynamic_oi(op, U0, X, eps_l, eps_h, c_max, t_max)
    return householder_onorm(U, c), c, traj


def doi_chebyshev(L: np.ndarray, U0: np.ndarray, X: np.ndarray, a: float, b: float, m: int,
                  passes: int, eps_l: float, eps_h: float, c_max: int, t_max: int):
    """Algorithm 2 with `passes` degree-m Chebyshev filters on the fixed
    damped interval [a, b] as the operator (the tracking path's filter; a
    re-orthonormalisation between passes does not change the span)."""
    def op(U):
        Y = U
        for _ in range(passes):
            Y = chebyshev_apply(L, Y, a, b, m)
        return Y

    return dynamic_oi(op, U0, X, eps_l, eps_h, c_max, t_max)


def chebyshev_apply(L: np.ndarray, V: np.ndarray, a: float, b: float, m: int) -> np.ndarray:
    """T_m(t(L)) V with t(x) = (2x - a - b) / (b - a), by the three-term
    recurrence T_0 = 1, T_1 = t, T_{k+1} = 2 t T_k - T_{k-1}."""
    tL = (2.0 * L - (a + b) * np.eye(L.shape[0])) / (b - a)
    Z0 = V
    if m == 0:
        return V.copy()
    Z1 = tL @ V
    for _ in range(1, m):
        Z0, Z1 = Z1, 2.0 * (tL @ Z1) - Z0
    return Z1


def chebyshev_span(L: np.ndarray, V0: np.ndarray, a: float, b: float, m: int, T: int) -> np.ndarray:
    """Orthonormal basis of span(T_m(t(L))^T V0).  The QR after each outer
    application only keeps the numbers representable; it does not change
    the span."""
    V = V0
    for _ in range(T):
        V, _ = np.linalg.qr(chebyshev_apply(L, V, a, b, m))
    return V


def rayleigh_ritz(L: np.ndarray, V: np.ndarray):
    """Ritz pairs of L on span(V) (V orthonormal): H = V^T L V = S Theta S^T,
    Ritz vectors V S, ascending."""
    H = V.T @ L @ V
    H = 0.5 * (H + H.T)
    th, S = np.linalg.eigh(H)
    return th, V @ S


def ritz_residuals(L: np.ndarray, V: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Section 4 (iteration count): residual norm of every Ritz pair,
    r_j = || L v_j - theta_j v_j ||_2, columns of V."""
    return np.linalg.norm(L @ V - V * theta[None, :], axis=0)
