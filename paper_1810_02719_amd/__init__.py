"""Block-based spectral processing of triangle meshes on MI355X.

Thin Python binding over the HIP library ``libmispectral.so`` (C ABI in
``include/mispectral.h``).  Torch provides device memory and the current
stream; every step of the computation runs in the library's kernels.  The
functions mirror the C entry points:

    build_laplacian   graph Laplacian of every block (Section 3, Eq. 1-2)
    oi_track          eigenspace tracking by orthogonal iteration (Section 4, Alg. 1)
    ritz_residuals    || L v_j - theta_j v_j || of the tracked pairs (Section 4)
    oi_track_tol      tolerance mode of the iteration count (oi_track + ritz_residuals)
    project           GFT coefficients E = U_c^T X (Section 3, 7.1)
    reconstruct       inverse GFT X~ = U_c E (Section 3, 7.1)
    choose_c          per-block subspace size for an NMSVE target (Section 5, Eq. 16)
    encdec_adjoint    gradient of encode/decode w.r.t. coordinates and edge weights
                      through the unrolled iteration; EncodeDecode wraps the forward
                      and this adjoint as a torch.autograd.Function
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from ._lib import MI_OP_CHEB, MI_OP_RZ  # noqa: F401
from ._lib import (MI_A_ABS, MI_A_RITZ, MI_A_WEYL, MI_BF16_IN, MI_FP32, MI_FP64, MI_RANDOM,  # noqa: F401
                   MI_W_COMBINATORIAL, MI_W_INV_DIST, MI_W_INV_SQ_DIST, MI_W_USER, MI_WARM_GIVEN,
                   MI_WARM_PRED, MiError)

__all__ = ["Blocks", "Context", "Laplacian", "OiParams", "build_laplacian", "laplacian_values",
           "oi_track", "ritz_residuals", "oi_track_tol", "TolResult", "encdec_adjoint", "EncodeDecode",
           "project", "reconstruct", "choose_c", "MiError"]


def _np_ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Blocks:
    """Host block table: sizes n_b, tracked widths p_b, slab strides ld_b
    (multiples of 32), warm-start predecessors and the kept pairs c_b that
    the tolerance test covers (None: p_b)."""

    def __init__(self, n, p=None, ld=None, pred=None, c=None):
        self.n = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
        B = self.n.size
        self.p = np.ascontiguousarray(np.asarray(p if p is not None else np.ones(B), dtype=np.int32))
        if ld is None:
            ld = ((self.p.astype(np.int64) + 31) // 32) * 32
        self.ld = np.ascontiguousarray(np.asarray(ld, dtype=np.int32))
        self.pred = (np.ascontiguousarray(np.asarray(pred, dtype=np.int32))
                     if pred is not None else None)
        self.c = (np.ascontiguousarray(np.asarray(c, dtype=np.int32).reshape(-1))
                  if c is not None else None)
        if self.c is not None and self.c.size == 1 and B > 1:
            self.c = np.full(B, int(self.c[0]), np.int32)
        self.v_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64))
        self.u_off = np.ascontiguousarray(
            np.concatenate([[0], np.cumsum(self.n * self.ld.astype(np.int64))]).astype(np.int64))
        self.t_off = np.concatenate([[0], np.cumsum(self.p.astype(np.int64))]).astype(np.int64)
        self._s = L.MiBlocks(B, _np_ptr(self.v_off, C.c_int64), _np_ptr(self.p, C.c_int32),
                             _np_ptr(self.ld, C.c_int32), _np_ptr(self.u_off, C.c_int64),
                             _np_ptr(self.pred, C.c_int32), _np_ptr(self.c, C.c_int32))

    @property
    def n_blocks(self):
        return int(self.n.size)

    @property
    def ref(self):
        return C.byref(self._s)

    def slab_view(self, V, b):
        """Block b's n_b x ld_b view of a flat slab tensor."""
        return V[int(self.u_off[b]):int(self.u_off[b + 1])].view(int(self.n[b]), int(self.ld[b]))


class Context:
    """Library context on one HIP device; caches workspaces so repeated calls
    reuse the same buffers (and the library can replay its captured graph)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        L.check(L.lib().mi_ctx_create(C.byref(h), device))
        self.h = h
        self._ws = {}

    def workspace(self, tag, nbytes):
        t = self._ws.get(tag)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                            device=f"cuda:{self.device}")
            self._ws[tag] = t
        return t

    def tuning(self):
        """Launch shapes of the current tracking plan: one (gram_target, nch,
        spmm_elements_per_lane, spmm_variant) tuple per wave."""
        n = C.c_int32()
        L.check(L.lib().mi_oi_tuning(self.h, None, 0, C.byref(n)))
        buf = (C.c_int32 * (4 * max(n.value, 1)))()
        L.check(L.lib().mi_oi_tuning(self.h, buf, n.value, C.byref(n)))
        return [tuple(buf[4 * w:4 * w + 4]) for w in range(n.value)]

    def force_spmm(self, variant: int = -1):
        """Run later tracking plans' per-row SpMM as `variant` (0..12, the codes
        `tuning()` reports) in every wave that uses it; -1 restores the
        autotuner's or the default choice."""
        L.check(L.lib().mi_oi_force_spmm(self.h, int(variant)))

    def set_timing(self, on: bool):
        """Per-kernel event timing of later oi_track / project / reconstruct
        calls (eager launches); restarts the totals."""
        L.check(L.lib().mi_ctx_set_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        """{class: (total_ms, launches)} since timing was switched on."""
        ms = (C.c_double * L.MI_K_COUNT)()
        n = (C.c_int64 * L.MI_K_COUNT)()
        L.check(L.lib().mi_ctx_kernel_times(self.h, ms, n))
        return {name: (float(ms[k]), int(n[k])) for k, name in enumerate(L.KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "h", None) is not None:
            L.lib().mi_ctx_destroy(self.h)
            self.h = None
        self._ws.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Laplacian:
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    edges: torch.Tensor
    edge_w: torch.Tensor
    nnz_off: np.ndarray
    edge_off: np.ndarray
    mode: int


def build_laplacian(ctx: Context, blocks: Blocks, prim_off, prims: torch.Tensor, arity: int = 3,
                    coords: torch.Tensor | None = None, mode: int = MI_W_COMBINATORIAL,
                    user_w: torch.Tensor | None = None) -> Laplacian:
    """CSR Laplacian of every block (mi_build_laplacian_count + mi_build_laplacian)."""
    lib = L.lib()
    prim_off = np.ascontiguousarray(np.asarray(prim_off, dtype=np.int64))
    ws_n = C.c_size_t()
    L.check(lib.mi_laplacian_workspace_size(blocks.ref, _np_ptr(prim_off, C.c_int64), arity,
                                            C.byref(ws_n)))
    ws = ctx.workspace("lap", ws_n.value)
    B = blocks.n_blocks
    nnz_off = np.zeros(B + 1, np.int64)
    edge_off = np.zeros(B + 1, np.int64)
    L.check(lib.mi_build_laplacian_count(ctx.h, blocks.ref, _np_ptr(prim_off, C.c_int64),
                                         _dptr(prims), arity, _np_ptr(nnz_off, C.c_int64),
                                         _np_ptr(edge_off, C.c_int64), _dptr(ws), ws.numel(),
                                         _stream()))
    dev = prims.device
    N = int(blocks.v_off[-1])
    row_ptr = torch.empty(N + B, dtype=torch.int32, device=dev)
    col = torch.empty(max(int(nnz_off[-1]), 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(int(nnz_off[-1]), 1), dtype=torch.float32, device=dev)
    edges = torch.empty(max(int(edge_off[-1]), 1) * 2, dtype=torch.int32, device=dev)
    edge_w = torch.empty(max(int(edge_off[-1]), 1), dtype=torch.float32, device=dev)
    L.check(lib.mi_build_laplacian(ctx.h, blocks.ref, _np_ptr(prim_off, C.c_int64), _dptr(prims),
                                   arity, _np_ptr(nnz_off, C.c_int64),
                                   _np_ptr(edge_off, C.c_int64), mode, _dptr(coords),
                                   _dptr(user_w), _dptr(row_ptr), _dptr(col), _dptr(val),
                                   _dptr(edges), _dptr(edge_w), _dptr(ws), ws.numel(), _stream()))
    return Laplacian(row_ptr, col, val, edges, edge_w, nnz_off, edge_off, mode)


def laplacian_values(ctx: Context, blocks: Blocks, lap: Laplacian, coords=None, mode=None,
                     user_w=None, err_flag=None):
    """Recompute lap.val / lap.edge_w in place on the existing structure."""
    mode = lap.mode if mode is None else mode
    L.check(L.lib().mi_laplacian_values(
        ctx.h, blocks.ref, _np_ptr(lap.nnz_off, C.c_int64), _np_ptr(lap.edge_off, C.c_int64), mode,
        _dptr(coords), _dptr(user_w), _dptr(lap.row_ptr), _dptr(lap.col), _dptr(lap.edges),
        _dptr(lap.val), _dptr(lap.edge_w), _dptr(err_flag), _stream()))
    lap.mode = mode
    return lap


@dataclass
class OiParams:
    """Mirror of mi_oi_params (see include/mispectral.h)."""
    precision: int = MI_FP32
    warm: int = MI_WARM_PRED
    T: int = 3
    m: int = 10
    passes: int = 2
    T0: int = 5
    m0: int = 10
    passes0: int = 2
    adapt: int = 1
    max_sweeps: int = 12
    a_mode: int = MI_A_WEYL
    a_value: float = 1.0
    b_abs: float = 0.0
    jacobi_tol: float = 1e-14
    rr_every: int = 0
    eig: int = 0  # MI_EIG_TRIDIAG (Jacobi for ld > 192) or MI_EIG_JACOBI
    autotune: int = 0  # 1: time candidate launch shapes when the plan is made
    op: int = 0  # MI_OP_CHEB (Chebyshev filter) or MI_OP_RZ ((L + delta I)^-z by CG)
    z: int = 1
    cg_iters: int = 200
    delta: float = 1e-3
    tol: float = 0.0  # > 0: tolerance mode (T, T0 cap the iterations)
    seed: int = 0     # seed of the MI_RANDOM start
    persistent: int = 0  # 1: each filter pass as one persistent launch (block work queue)

    def struct(self):
        return L.MiOiParams(self.precision, self.warm, self.T, self.m, self.passes, self.T0,
                            self.m0, self.passes0, self.adapt, self.max_sweeps, self.a_mode, self.rr_every,
                            self.eig, self.autotune, self.a_value, self.b_abs, self.jacobi_tol,
                            self.op, self.z, self.cg_iters, self.persistent, self.delta, self.tol,
                            int(self.seed) & 0xFFFFFFFFFFFFFFFF)


def _dtype(precision):
    return torch.float64 if precision == MI_FP64 else torch.float32


def oi_track(ctx: Context, blocks: Blocks, lap: Laplacian, params: OiParams, V0=None, V=None,
             ritz=None, status=None, per_block: bool = False, resid=None, iters=None):
    """Tracked subspaces of every block (mi_oi_track / mi_oi_track_per_block).
    Returns (V, ritz, status); resid (FP64 [sum p_b]) and iters (int32 [B])
    are filled when given (resid is allocated in tolerance mode)."""
    lib = L.lib()
    prm = params.struct()
    dev = f"cuda:{ctx.device}"
    dt = _dtype(params.precision)
    if V is None:
        V = torch.empty(int(blocks.u_off[-1]), dtype=dt, device=dev)
    if ritz is None:
        ritz = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    if status is None:
        status = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    if resid is None and params.tol > 0:
        resid = torch.empty(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    ws_n = C.c_size_t()
    L.check(lib.mi_oi_workspace_size(ctx.h, blocks.ref, C.byref(prm), C.byref(ws_n)))
    ws = ctx.workspace("oi", ws_n.value)
    fn = lib.mi_oi_track_per_block if per_block else lib.mi_oi_track
    L.check(fn(ctx.h, blocks.ref, C.byref(prm), _dptr(lap.row_ptr), _dptr(lap.col), _dptr(lap.val),
               _np_ptr(lap.nnz_off, C.c_int64), _dptr(V0), _dptr(V), _dptr(ritz), _dptr(resid),
               _dptr(iters), _dptr(status), _dptr(ws), ws.numel(), _stream()))
    return V, ritz, status


class DoiResult:
    """Output of doi_track: final bases V, sizes c, trajectory traj [B, t_max,
    2] of (c, ||e||) before each decision ((-1, -1) after a block stopped),
    iterations run and status flags (device tensors)."""

    def __init__(self, V, c, traj, iters, status):
        self.V, self.c, self.traj, self.iters, self.status = V, c, traj, iters, status


def doi_track(ctx: Context, blocks: Blocks, lap: Laplacian, params: OiParams, X: torch.Tensor,
              c0: torch.Tensor, eps_l: float, eps_h: float, c_max: int, t_max: int,
              V0: torch.Tensor | None = None) -> DoiResult:
    """Dynamic OI, Alg. 2 (mi_doi_track): X the block coordinates (FP32 [v_off[B]
    * 3]); c0 int32 [B] start sizes of blocks without predecessor."""
    lib = L.lib()
    prm = params.struct()
    dp = L.MiDoiParams(float(eps_l), float(eps_h), int(c_max), int(t_max))
    dev = f"cuda:{ctx.device}"
    V = torch.empty(int(blocks.u_off[-1]), dtype=_dtype(params.precision), device=dev)
    c = c0.to(torch.int32).clone()
    traj = torch.empty(max(blocks.n_blocks * int(t_max) * 2, 1), dtype=torch.float64, device=dev)
    iters = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    status = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    ws_n = C.c_size_t()
    L.check(lib.mi_doi_workspace_size(ctx.h, blocks.ref, C.byref(prm), C.byref(dp), C.byref(ws_n)))
    ws = ctx.workspace("doi", ws_n.value)
    L.check(lib.mi_doi_track(ctx.h, blocks.ref, C.byref(prm), C.byref(dp), _dptr(lap.row_ptr),
                             _dptr(lap.col), _dptr(lap.val), _np_ptr(lap.nnz_off, C.c_int64),
                             _dptr(X), _dptr(V0), _dptr(V), _dptr(c), _dptr(traj), _dptr(iters),
                             _dptr(status), _dptr(ws), ws.numel(), _stream()))
    return DoiResult(V, c, traj[:blocks.n_blocks * int(t_max) * 2].view(blocks.n_blocks, int(t_max), 2),
                     iters, status)


def ritz_residuals(ctx: Context, blocks: Blocks, lap: Laplacian, V: torch.Tensor,
                   ritz: torch.Tensor, precision: int = MI_FP32,
                   resid: torch.Tensor | None = None) -> torch.Tensor:
    """resid[t_off_b + j] = || L_b v_j - theta_j v_j || for every tracked column
    (mi_ritz_residuals); device float64 [sum p_b]."""
    if resid is None:
        resid = torch.empty(int(blocks.t_off[-1]), dtype=torch.float64, device=V.device)
    lib = L.lib()
    ws_n = C.c_size_t()
    L.check(lib.mi_residual_workspace_size(ctx.h, blocks.ref, C.byref(ws_n)))
    ws = ctx.workspace("resid", ws_n.value)
    L.check(lib.mi_ritz_residuals(ctx.h, blocks.ref, precision, _dptr(lap.row_ptr), _dptr(lap.col),
                                  _dptr(lap.val), _np_ptr(lap.nnz_off, C.c_int64), _dptr(V),
                                  _dptr(ritz), _dptr(resid), _dptr(ws), ws.numel(), _stream()))
    return resid


@dataclass
class TolResult:
    V: torch.Tensor
    ritz: torch.Tensor
    status: torch.Tensor
    resid: torch.Tensor        # residual norms of the returned pairs (device FP64)
    iters: torch.Tensor        # per block: iteration whose result is returned (device int32)
    converged: torch.Tensor    # per block: met tol within the cap (device bool)


def oi_track_tol(ctx: Context, blocks: Blocks, lap: Laplacian, params: OiParams, tol: float,
                 V0=None) -> TolResult:
    """Tolerance mode of the iteration control (mi_oi_track with params.tol
    = tol): every block stops at the first iteration whose kept pairs j <
    c_b (blocks.c) satisfy ||L v_j - theta_j v_j|| <= tol |theta_{p_b - 1}|;
    params.T / T0 cap the iterations.  The test runs on the device, inside
    the library's launch sequence."""
    prm = OiParams(**{**params.__dict__, "tol": float(tol)})
    dev = f"cuda:{ctx.device}"
    resid = torch.empty(int(blocks.t_off[-1]), dtype=torch.float64, device=dev)
    iters = torch.zeros(blocks.n_blocks, dtype=torch.int32, device=dev)
    V, ritz, status = oi_track(ctx, blocks, lap, prm, V0=V0, resid=resid, iters=iters)
    conv = (status & L.MI_BLOCK_UNCONVERGED) == 0
    return TolResult(V, ritz, status, resid, iters, conv)


def project(ctx: Context, blocks: Blocks, c: torch.Tensor, U: torch.Tensor, X: torch.Tensor,
            precision: int = MI_FP32, E: torch.Tensor | None = None) -> torch.Tensor:
    """E = U_c^T X per block (rows k >= c_b zero)."""
    if E is None:
        E = torch.empty(int(blocks.t_off[-1]) * 3, dtype=_dtype(precision), device=U.device)
    lib = L.lib()
    ws_n = C.c_size_t()
    L.check(lib.mi_encdec_workspace_size(ctx.h, blocks.ref, precision, C.byref(ws_n)))
    ws = ctx.workspace("encdec", ws_n.value)
    L.check(lib.mi_project(ctx.h, blocks.ref, precision, _dptr(c), _dptr(U), _dptr(X), _dptr(E),
                           _dptr(ws), ws.numel(), _stream()))
    return E


def project_noalloc(ctx: Context, blocks: Blocks, c: torch.Tensor, U: torch.Tensor,
                    X: torch.Tensor, E: torch.Tensor, precision: int = MI_FP32) -> torch.Tensor:
    """E = U_c^T X per block without any device allocation
    (mi_project_noalloc): E must be given (device, [sum p_b * 3])."""
    L.check(L.lib().mi_project_noalloc(ctx.h, blocks.ref, precision, _dptr(c), _dptr(U), _dptr(X),
                                       _dptr(E), _stream()))
    return E


def reconstruct(ctx: Context, blocks: Blocks, c: torch.Tensor, U: torch.Tensor, E: torch.Tensor,
                precision: int = MI_FP32, Xr: torch.Tensor | None = None) -> torch.Tensor:
    """X~ = U_c E per block."""
    if Xr is None:
        Xr = torch.empty(int(blocks.v_off[-1]) * 3, dtype=_dtype(precision), device=U.device)
    L.check(L.lib().mi_reconstruct(ctx.h, blocks.ref, precision, _dptr(c), _dptr(U), _dptr(E),
                                   _dptr(Xr), _stream()))
    return Xr


def merge_overlapped(ctx: Context, blocks: Blocks, gid, n_vertices: int, lap: Laplacian,
                     Xr: torch.Tensor, Xout: torch.Tensor | None = None) -> torch.Tensor:
    """Degree-weighted merge of the reconstructions of overlapped submeshes
    (mi_merge_overlapped).  gid: host int32 [v_off[B]], the mesh vertex of
    every block row; Xr: FP32 [v_off[B] * 3]; returns FP32 [n_vertices * 3]."""
    gid = np.ascontiguousarray(np.asarray(gid, dtype=np.int32))
    if Xout is None:
        Xout = torch.empty(int(n_vertices) * 3, dtype=torch.float32, device=Xr.device)
    L.check(L.lib().mi_merge_overlapped(ctx.h, blocks.ref, _np_ptr(gid, C.c_int32), int(n_vertices),
                                        _dptr(lap.row_ptr), _dptr(Xr), _dptr(Xout), _stream()))
    return Xout


def quantize(ctx: Context, blocks: Blocks, c: torch.Tensor, E: torch.Tensor, qbits: int = 12,
             dequantize: bool = True):
    """Uniform qbits-bit quantisation of the feature vectors (mi_quantize).
    Returns (codes uint16 [sum p_b * 3] as int16 storage, params FP32 [B * 6],
    dequantised E or None)."""
    n = int(blocks.t_off[-1]) * 3
    codes = torch.empty(n, dtype=torch.int16, device=E.device)
    params = torch.empty(blocks.n_blocks * 6, dtype=torch.float32, device=E.device)
    Eq = torch.empty(n, dtype=torch.float32, device=E.device) if dequantize else None
    L.check(L.lib().mi_quantize(ctx.h, blocks.ref, _dptr(c), int(qbits), _dptr(E), _dptr(codes),
                                _dptr(params), _dptr(Eq) if Eq is not None else None, _stream()))
    return codes, params, Eq


def mesh_laplacian(ctx: Context, n_vertices: int, faces: torch.Tensor,
                   coords: torch.Tensor | None = None, mode: int = MI_W_COMBINATORIAL) -> Laplacian:
    """Laplacian of a whole mesh (one block holding every vertex): its
    row_ptr / col are the neighbour lists mesh_quality takes."""
    nf = int(faces.numel() // 3)
    blocks = Blocks(np.array([int(n_vertices)]), p=np.array([1]), pred=np.array([-1]))
    return build_laplacian(ctx, blocks, np.array([0, nf]), faces, 3, coords, mode)


QUALITY_FIELDS = ("nmsve", "nmsve_db", "l2", "gl", "theta_deg", "faces_used", "zero_edges",
                  "bad_indices")


def mesh_quality(ctx: Context, n_vertices: int, row_ptr: torch.Tensor, col: torch.Tensor,
                 faces: torch.Tensor, X: torch.Tensor, Xr: torch.Tensor,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """NMSVE (Eq. 16) and mean face-normal angle of a whole mesh
    (mi_mesh_quality).  row_ptr / col: neighbour CSR of the mesh (a
    Laplacian's diagonal is skipped); faces int32 [F * 3]; X, Xr FP32
    [n * 3].  Returns the FP64 [8] device tensor named by QUALITY_FIELDS."""
    if out is None:
        out = torch.empty(8, dtype=torch.float64, device=X.device)
    L.check(L.lib().mi_mesh_quality(ctx.h, int(n_vertices), _dptr(row_ptr), _dptr(col),
                                    int(col.numel()), int(faces.numel() // 3), _dptr(faces),
                                    _dptr(X), _dptr(Xr), _dptr(out), _stream()))
    return out


def choose_c(ctx: Context, blocks: Blocks, c_max: torch.Tensor, target: float, g_min: float,
             U: torch.Tensor, ritz: torch.Tensor, X: torch.Tensor, gl: Laplacian,
             c_out: torch.Tensor | None = None, metric: torch.Tensor | None = None):
    """Per-block c for an NMSVE target (gl: the MI_W_INV_DIST Laplacian of the
    original mesh).  Returns (c, metric curve)."""
    lib = L.lib()
    ws_n = C.c_size_t()
    L.check(lib.mi_choose_c_workspace_size(ctx.h, blocks.ref, C.byref(ws_n)))
    ws = ctx.workspace("cc", ws_n.value)
    if c_out is None:
        c_out = torch.empty(blocks.n_blocks, dtype=torch.int32, device=U.device)
    if metric is None:
        metric = torch.zeros(int(blocks.t_off[-1]), dtype=torch.float64, device=U.device)
    L.check(lib.mi_choose_c(ctx.h, blocks.ref, _dptr(c_max), float(target), float(g_min), _dptr(U),
                            _dptr(ritz), _dptr(X), _dptr(gl.row_ptr), _dptr(gl.col), _dptr(gl.val),
                            _np_ptr(gl.nnz_off, C.c_int64), _dptr(c_out), _dptr(metric), _dptr(ws),
                            ws.numel(), _stream()))
    return c_out, metric


def encdec_adjoint(ctx: Context, blocks: Blocks, lap: Laplacian, params: OiParams, V0: torch.Tensor,
                   X: torch.Tensor, c: torch.Tensor, Gbar: torch.Tensor, mode: int | None = None):
    """(d loss/d X, d loss/d w) of loss = <Gbar, X~> through the unrolled
    tracking (mi_encdec_adjoint).  X, Gbar: flat [3 n] in the params'
    element type; returns float64 tensors [3 n] and [sum |E_b|]."""
    lib = L.lib()
    prm = params.struct()
    mode = lap.mode if mode is None else mode
    ws_n = C.c_size_t()
    L.check(lib.mi_adjoint_workspace_size(ctx.h, blocks.ref, C.byref(prm),
                                          _np_ptr(lap.nnz_off, C.c_int64), C.byref(ws_n)))
    ws = ctx.workspace("adjoint", ws_n.value)
    Xbar = torch.empty(int(blocks.v_off[-1]) * 3, dtype=torch.float64, device=X.device)
    wbar = torch.zeros(max(int(lap.edge_off[-1]), 1), dtype=torch.float64, device=X.device)
    L.check(lib.mi_encdec_adjoint(ctx.h, blocks.ref, C.byref(prm), mode, _dptr(lap.row_ptr),
                                  _dptr(lap.col), _dptr(lap.val), _np_ptr(lap.nnz_off, C.c_int64),
                                  _dptr(lap.edges), _np_ptr(lap.edge_off, C.c_int64), _dptr(V0),
                                  _dptr(X), _dptr(c), _dptr(Gbar), _dptr(Xbar), _dptr(wbar),
                                  _dptr(ws), ws.numel(), _stream()))
    return Xbar, wbar[:int(lap.edge_off[-1])]


class EncodeDecode(torch.autograd.Function):
    """X~ = U_c U_c^T X per block with U_c from the tracking of V0 under the
    Laplacian of (X, w); differentiable in X and w (user weights).

        Xr = EncodeDecode.apply(X, w, ctx, blocks, lap, params, V0, c)

    X: flat [3 n] coordinates (float32; the projection runs in the params'
    precision); w: per-edge user weights (float32) when lap.mode is
    MI_W_USER, else None.  The forward recomputes the Laplacian values,
    tracks, projects and reconstructs; the backward restores the Laplacian
    values of its own forward (lap is shared: another forward may have
    rewritten lap.val since, e.g. the next frame of a sequence) and calls
    encdec_adjoint.  After a backward, lap holds that forward's values."""

    @staticmethod
    def forward(fctx, X, w, ctx, blocks, lap, params, V0, c):
        dt = _dtype(params.precision)
        X32 = X.detach().to(torch.float32).contiguous()
        uw = w.detach().to(torch.float32).contiguous() if w is not None else None
        laplacian_values(ctx, blocks, lap, X32, lap.mode, uw)
        V, _, _ = oi_track(ctx, blocks, lap, params, V0=V0)
        Xp = X.detach().to(dt).contiguous()
        E = project(ctx, blocks, c, V, Xp, params.precision)
        Xr = reconstruct(ctx, blocks, c, V, E, params.precision)
        # the inputs that set the Laplacian values of this forward
        fctx.save_for_backward(Xp, V0, c, X32, uw)
        fctx.meta = (ctx, blocks, lap, params, X.dtype, None if w is None else w.dtype)
        return Xr.to(X.dtype)

    @staticmethod
    def backward(fctx, g):
        Xp, V0, c, X32, uw = fctx.saved_tensors
        ctx, blocks, lap, params, xdt, wdt = fctx.meta
        laplacian_values(ctx, blocks, lap, X32, lap.mode, uw)
        G = g.detach().to(Xp.dtype).contiguous()
        Xbar, wbar = encdec_adjoint(ctx, blocks, lap, params, V0, Xp, c, G)
        gw = wbar.to(wdt) if wdt is not None else None
        return Xbar.to(xdt), gw, None, None, None, None, None, None
