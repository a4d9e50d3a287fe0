"""ctypes declarations of the C ABI in include/mispectral.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmispectral.so")

MI_OK = 0
MI_ERR_ARG = -1
MI_ERR_INDEX = -2
MI_ERR_DEGENERATE = -3
MI_ERR_NOT_PD = -4
MI_ERR_NOCONV = -5
MI_ERR_HIP = -6
MI_ERR_WORKSPACE = -7
MI_ERR_CAPACITY = -8

MI_W_COMBINATORIAL = 0
MI_W_INV_SQ_DIST = 1
MI_W_USER = 2
MI_W_INV_DIST = 3

MI_FP32 = 0
MI_FP64 = 1
MI_BF16_IN = 2

MI_WARM_GIVEN = 0
MI_WARM_PRED = 1
MI_RANDOM = 2

MI_A_WEYL = 0
MI_A_ABS = 1
MI_A_RITZ = 2

MI_EIG_TRIDIAG = 0
MI_EIG_JACOBI = 1

MI_OP_CHEB = 0
MI_OP_RZ = 1

KERNEL_CLASSES = ["spmm", "gram", "gram_small", "gram_reduce", "chol", "rowmul", "rowmul_small",
                  "rq_max", "jacobi_init", "jacobi_sweep", "apply_rot", "rr_finish", "perm_cast",
                  "setup", "project", "reconstruct", "eig_reduce", "eig_values", "eig_vectors",
                  "eig_back", "merge", "quantize", "quality", "doi", "cg", "cheb_pass"]
MI_K_COUNT = len(KERNEL_CLASSES)

MI_BLOCK_OK = 0
MI_BLOCK_SHIFTED = 1
MI_BLOCK_NOT_PD = 2
MI_BLOCK_NOCONV = 4
MI_BLOCK_NONFINITE = 8
MI_BLOCK_UNCONVERGED = 16

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_szp = C.POINTER(C.c_size_t)
_vp = C.c_void_p


class MiBlocks(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("v_off", _i64p), ("p", _i32p), ("ld", _i32p),
                ("u_off", _i64p), ("pred", _i32p), ("c", _i32p)]


class MiOiParams(C.Structure):
    _fields_ = [("precision", C.c_int32), ("warm", C.c_int32), ("T", C.c_int32), ("m", C.c_int32),
                ("passes", C.c_int32), ("T0", C.c_int32), ("m0", C.c_int32),
                ("passes0", C.c_int32), ("adapt", C.c_int32), ("max_sweeps", C.c_int32),
                ("a_mode", C.c_int32), ("rr_every", C.c_int32), ("eig", C.c_int32),
                ("autotune", C.c_int32), ("a_value", C.c_double),
                ("b_abs", C.c_double), ("jacobi_tol", C.c_double), ("op", C.c_int32),
                ("z", C.c_int32), ("cg_iters", C.c_int32), ("persistent", C.c_int32),
                ("delta", C.c_double), ("tol", C.c_double), ("seed", C.c_uint64)]


class MiDoiParams(C.Structure):
    _fields_ = [("eps_l", C.c_double), ("eps_h", C.c_double), ("c_max", C.c_int32),
                ("t_max", C.c_int32)]


_SIGS = {
    "mi_ctx_create": [C.POINTER(_vp), C.c_int32],
    "mi_ctx_destroy": [_vp],
    "mi_ctx_set_timing": [_vp, C.c_int32],
    "mi_oi_force_spmm": [_vp, C.c_int32],
    "mi_ctx_kernel_times": [_vp, C.POINTER(C.c_double), _i64p],
    "mi_laplacian_workspace_size": [C.POINTER(MiBlocks), _i64p, C.c_int32, _szp],
    "mi_build_laplacian_count": [_vp, C.POINTER(MiBlocks), _i64p, _vp, C.c_int32, _i64p, _i64p,
                                 _vp, C.c_size_t, _vp],
    "mi_build_laplacian": [_vp, C.POINTER(MiBlocks), _i64p, _vp, C.c_int32, _i64p, _i64p,
                           C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
    "mi_laplacian_values": [_vp, C.POINTER(MiBlocks), _i64p, _i64p, C.c_int32, _vp, _vp, _vp, _vp,
                            _vp, _vp, _vp, _vp, _vp],
    "mi_oi_workspace_size": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), _szp],
    "mi_oi_tuning": [_vp, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)],
    "mi_oi_track": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), _vp, _vp, _vp, _i64p, _vp,
                    _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
    "mi_doi_workspace_size": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams),
                              C.POINTER(MiDoiParams), _szp],
    "mi_doi_track": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), C.POINTER(MiDoiParams), _vp,
                     _vp, _vp, _i64p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
    "mi_oi_track_per_block": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), _vp, _vp, _vp,
                              _i64p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
    "mi_residual_workspace_size": [_vp, C.POINTER(MiBlocks), _szp],
    "mi_ritz_residuals": [_vp, C.POINTER(MiBlocks), C.c_int32, _vp, _vp, _vp, _i64p, _vp, _vp, _vp,
                          _vp, C.c_size_t, _vp],
    "mi_adjoint_workspace_size": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), _i64p, _szp],
    "mi_encdec_adjoint": [_vp, C.POINTER(MiBlocks), C.POINTER(MiOiParams), C.c_int32, _vp, _vp,
                          _vp, _i64p, _vp, _i64p, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t,
                          _vp],
    "mi_encdec_workspace_size": [_vp, C.POINTER(MiBlocks), C.c_int32, _szp],
    "mi_project": [_vp, C.POINTER(MiBlocks), C.c_int32, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp],
    "mi_project_noalloc": [_vp, C.POINTER(MiBlocks), C.c_int32, _vp, _vp, _vp, _vp, _vp],
    "mi_reconstruct": [_vp, C.POINTER(MiBlocks), C.c_int32, _vp, _vp, _vp, _vp, _vp],
    "mi_merge_overlapped": [_vp, C.POINTER(MiBlocks), _vp, C.c_int64, _vp, _vp, _vp, _vp],
    "mi_quantize": [_vp, C.POINTER(MiBlocks), _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp],
    "mi_mesh_quality": [_vp, C.c_int64, _vp, _vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp],
    "mi_choose_c_workspace_size": [_vp, C.POINTER(MiBlocks), _szp],
    "mi_choose_c": [_vp, C.POINTER(MiBlocks), _vp, C.c_double, C.c_double, _vp, _vp, _vp, _vp,
                    _vp, _vp, _i64p, _vp, _vp, _vp, C.c_size_t, _vp],
}

_lib = None


def lib():
    """The loaded library (raises if it is missing: there is no CPU path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1810_02719_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.mi_last_error.restype = C.c_char_p
        L.mi_last_error.argtypes = []
        L.mi_version.restype = C.c_char_p
        L.mi_version.argtypes = []
        L.mi_kernel_class_name.restype = C.c_char_p
        L.mi_kernel_class_name.argtypes = [C.c_int32]
        names = [L.mi_kernel_class_name(k).decode() for k in range(MI_K_COUNT)]
        if names != KERNEL_CLASSES or L.mi_kernel_class_name(MI_K_COUNT) is not None:
            raise ImportError(f"kernel class table of {LIB_PATH} does not match the binding")
        _lib = L
    return _lib


def declared_symbols():
    """Function names declared in include/mispectral.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "mispectral.h")
    txt = open(hdr).read()
    pat = r"^\s*(?:mi_status|const\s+char\s*\*)\s*(mi_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(pat, txt, flags=re.M)))


class MiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(code):
    if code != MI_OK:
        raise MiError(code, lib().mi_last_error().decode())
