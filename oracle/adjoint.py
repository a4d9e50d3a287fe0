"""Gradient of a block's encode/decode with respect to the vertex coordinates
and the Laplacian edge weights, through the unrolled orthogonal iteration,
in FP64.  Test infrastructure only.

The paper does not differentiate its pipeline; the map differentiated here is
the one the tracking computes for one block:

  L(w)  = sum_e w_e (e_a - e_b)(e_a - e_b)^T        Laplacian of Section 3, Eq. 1-2
                                                      (D_ii = sum of the weights at i)
  Y_0   = V0;  Y <- orth(T_m(t(L)) Y), N times       orthogonal iteration of Section 4,
                                                      Alg. 1, with the polynomial operator
  H     = Q^T L Q = S Theta S^T (ascending)          Rayleigh-Ritz on the final basis
  U_c   = Q S[:, :c]                                 the first c columns in eigenvalue order
  X~    = U_c U_c^T X                                encode / truncate / decode, Section 3
                                                      (GFT) and Section 7.1
  loss  = <Gbar, X~>                                 so d loss / d X~ = Gbar

with w = 1 (combinatorial), w = 1/|x_a - x_b|^2 (distance weights, then the
weights depend on X) or user weights.  The filter interval [a, b] is a
constant: no gradient flows into it.  tracked_grad runs the same map with the
tracking's interval schedule (Gershgorin b, adaptive a) and warm starts, the
interval and the start again held constant.  Torch autograd on the CPU in float64
differentiates the plain forward (QR is Householder, eigh is LAPACK).

eigenprojector_grad is the converged limit of the same gradient (first-order
perturbation of the spectral projector P_c = U_c U_c^T), written out from its
definition with a full eigendecomposition.
"""
from __future__ import annotations

import numpy as np
import torch

from .laplacian import COMBINATORIAL, INV_DIST, INV_SQ_DIST, USER  # noqa: F401


def weights(edges: torch.Tensor, X: torch.Tensor, mode: int, user_w=None) -> torch.Tensor:
    """Off-diagonal weights per canonical edge (Section 3, Eq. 2)."""
    if mode == COMBINATORIAL:
        return torch.ones(edges.shape[0], dtype=torch.float64)
    if mode == USER:
        return user_w
    d2 = ((X[edges[:, 0]] - X[edges[:, 1]]) ** 2).sum(dim=1)
    return 1.0 / d2 if mode == INV_SQ_DIST else 1.0 / torch.sqrt(d2)


def laplacian(n: int, edges: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """L = B^T diag(w) B with B the signed edge-vertex incidence (Eq. 1)."""
    B = torch.zeros(edges.shape[0], n, dtype=torch.float64)
    r = torch.arange(edges.shape[0])
    B[r, edges[:, 0]] = 1.0
    B[r, edges[:, 1]] = -1.0
    return B.T @ (w[:, None] * B)


def chebyshev(L: torch.Tensor, V: torch.Tensor, a: float, b: float, m: int) -> torch.Tensor:
    """T_m(t(L)) V, t(x) = (2x - a - b)/(b - a), three-term recurrence."""
    tL = (2.0 * L - (a + b) * torch.eye(L.shape[0], dtype=torch.float64)) / (b - a)
    Z0, Z1 = V, tL @ V
    for _ in range(1, m):
        Z0, Z1 = Z1, 2.0 * (tL @ Z1) - Z0
    return Z1


def encdec(n, edges, X, mode, V0, a, b, m, N, c, user_w=None) -> torch.Tensor:
    """X~ of one block after N filter passes from V0 and Rayleigh-Ritz."""
    w = weights(edges, X, mode, user_w)
    L = laplacian(n, edges, w)
    Q = V0
    for _ in range(N):
        Q, _ = torch.linalg.qr(chebyshev(L, Q, a, b, m))
    H = Q.T @ L @ Q
    H = 0.5 * (H + H.T)
    _, S = torch.linalg.eigh(H)
    U = Q @ S[:, :c]
    return U @ (U.T @ X)


def unrolled_grad(n: int, edges: np.ndarray, X: np.ndarray, mode: int, V0: np.ndarray, a: float,
                  b: float, m: int, N: int, c: int, Gbar: np.ndarray, user_w=None):
    """(d loss/d X, d loss/d w) of loss = <Gbar, X~>; d/dw is per canonical
    edge (for distance weights it is the gradient at the weights, before the
    chain rule into X, which d/dX already includes)."""
    e = torch.from_numpy(np.asarray(edges, np.int64))
    Xt = torch.tensor(np.asarray(X, np.float64), requires_grad=True)
    if mode == USER:
        w0 = torch.tensor(np.asarray(user_w, np.float64), requires_grad=True)
    else:
        w0 = weights(e, Xt, mode).detach().requires_grad_(True)
    # weights as a leaf, then chained into X by a second backward
    L = laplacian(n, e, w0)
    Q = torch.from_numpy(np.asarray(V0, np.float64))
    for _ in range(N):
        Q, _ = torch.linalg.qr(chebyshev(L, Q, a, b, m))
    H = Q.T @ L @ Q
    H = 0.5 * (H + H.T)
    _, S = torch.linalg.eigh(H)
    U = Q @ S[:, :c]
    Xr = U @ (U.T @ Xt)
    loss = (torch.from_numpy(np.asarray(Gbar, np.float64)) * Xr).sum()
    gX, gw = torch.autograd.grad(loss, (Xt, w0))
    gX = gX.clone()
    if mode in (INV_SQ_DIST, INV_DIST):
        Xc = Xt.detach().clone().requires_grad_(True)
        (gX2,) = torch.autograd.grad((weights(e, Xc, mode) * gw).sum(), (Xc,))
        gX += gX2
    return gX.numpy(), gw.numpy()


def gershgorin(L: torch.Tensor) -> float:
    """max_i sum_j |L_ij|: an upper bound of the spectrum (Gershgorin's
    circle theorem)."""
    return float(L.detach().abs().sum(dim=1).max())


def warm_start(V_pred: np.ndarray, n: int, p: int) -> np.ndarray:
    """The tracking's index-aligned warm start of an n-vertex block of width p
    from its predecessor's basis: shared rows and columns copied, missing rows
    zero, columns j past the predecessor's width the unit vector
    e_{(997 j) mod n}."""
    npd, ppd = V_pred.shape
    S0 = np.zeros((n, p))
    k, q = min(n, npd), min(p, ppd)
    S0[:k, :q] = V_pred[:k, :q]
    for j in range(ppd, p):
        S0[(997 * j) % n, j] = 1.0
    return S0


def tracked_grad(n: int, edges: np.ndarray, X: np.ndarray, mode: int, start: np.ndarray, c: int,
                 Gbar: np.ndarray, *, T: int, m: int, passes: int, a0, b=None, adapt=False,
                 orth_start=False, user_w=None, schedule=None):
    """Gradient of loss = <Gbar, X~> through one block's tracking as the
    library schedules it, with its filter interval held constant:
      b    the given bound, or gershgorin(L) when None;
      a_0  a0, or a0(b) when callable (the initial lower bound of a_mode);
      per iteration t the filter runs on [clip(a_t, 1e-3 b, 0.95 b), b];
      with adapt, a_{t+1} = max_j q_j^T L q_j over the orthonormalised basis
      after iteration t (not after the last);
      T iterations of `passes` Chebyshev passes of degree m, the basis
      orthonormalised after every pass, Rayleigh-Ritz at the end
    (Section 4, Alg. 1).  The start (orthonormalised first when orth_start)
    is a constant, and so are b and every a_t: the gradient is stopped at
    them.  `schedule` = (b, [a_0 .. a_{T-1}]) replaces the rule (for finite
    differences at a frozen interval).
    Returns (d loss/dX, d loss/dw, info) with info = {"b", "a" (the a_t used,
    before clipping), "theta" (Ritz values, ascending), "U" (n x p Ritz
    vectors)}."""
    e = torch.from_numpy(np.asarray(edges, np.int64))
    Xt = torch.tensor(np.asarray(X, np.float64), requires_grad=True)
    if mode == USER:
        w0 = torch.tensor(np.asarray(user_w, np.float64), requires_grad=True)
    else:
        w0 = weights(e, Xt, mode).detach().requires_grad_(True)
    L = laplacian(n, e, w0)
    Ld = L.detach()
    if schedule is not None:
        bb, a_list = float(schedule[0]), [float(a) for a in schedule[1]]
    else:
        bb = float(b) if b is not None else gershgorin(Ld)
        a_list = [float(a0(bb)) if callable(a0) else float(a0)]
    Q = torch.from_numpy(np.asarray(start, np.float64))
    if orth_start:
        Q, _ = torch.linalg.qr(Q)
    for t in range(T):
        a = a_list[t]
        ac = min(max(a, 1e-3 * bb), 0.95 * bb)
        for _ in range(passes):
            Q, _ = torch.linalg.qr(chebyshev(L, Q, ac, bb, m))
        if schedule is None and t < T - 1:
            Qd = Q.detach()
            a_list.append(float(torch.diagonal(Qd.T @ Ld @ Qd).max()) if adapt else a)
    H = Q.T @ L @ Q
    H = 0.5 * (H + H.T)
    theta, S = torch.linalg.eigh(H)
    U = Q @ S[:, :c]
    Xr = U @ (U.T @ Xt)
    loss = (torch.from_numpy(np.asarray(Gbar, np.float64)) * Xr).sum()
    gX, gw = torch.autograd.grad(loss, (Xt, w0))
    gX = gX.clone()
    if mode in (INV_SQ_DIST, INV_DIST):
        Xc = Xt.detach().clone().requires_grad_(True)
        (gX2,) = torch.autograd.grad((weights(e, Xc, mode) * gw).sum(), (Xc,))
        gX += gX2
    info = {"b": bb, "a": a_list, "theta": theta.detach().numpy(),
            "U": (Q @ S).detach().numpy(), "loss": float(loss.detach())}
    return gX.numpy(), gw.numpy(), info


def eigenprojector_grad(L: np.ndarray, edges: np.ndarray, X: np.ndarray, Gbar: np.ndarray, c: int):
    """Converged limit: loss = <Gbar, P_c X> = <P_c, A>, A = sym(Gbar X^T), and
    dP_c = sum_{i<c<=j} (u_i u_j^T + u_j u_i^T) (u_j^T dL u_i)/(lambda_i - lambda_j),
    u_j^T dL u_i = sum_e dw_e (u_j[a]-u_j[b])(u_i[a]-u_i[b]).
    Returns (d loss/dX at fixed L, d loss/dw)."""
    lam, U = np.linalg.eigh(L)
    Uc = U[:, :c]
    gX = Uc @ (Uc.T @ Gbar)
    A = 0.5 * (Gbar @ X.T + X @ Gbar.T)
    Du = U[edges[:, 0]] - U[edges[:, 1]]  # |E| x n
    gw = np.zeros(edges.shape[0])
    for i in range(c):
        for j in range(c, L.shape[0]):
            coef = 2.0 * (U[:, j] @ A @ U[:, i]) / (lam[i] - lam[j])
            gw += coef * Du[:, j] * Du[:, i]
    return gX, gw
