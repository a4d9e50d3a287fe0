"""CPU tests of the C ABI boundary: the library loads, exports every symbol
the header declares, and rejects bad block tables and parameters on the host
(no GPU needed: the workspace-size queries are host arithmetic)."""
import ctypes as C

import numpy as np
import pytest

import paper_1810_02719_amd as mis
from paper_1810_02719_amd import _lib as L


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = L.declared_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.mi_version().decode().startswith("mispectral")


def _oi_ws(blocks, prm):
    n = C.c_size_t()
    code = L.lib().mi_oi_workspace_size(None, blocks.ref, C.byref(prm.struct()), C.byref(n))
    return code, n.value


def test_oi_workspace_query_valid_table():
    b = mis.Blocks([100, 200, 150], p=[20, 40, 30], pred=[-1, 0, 1])
    code, n = _oi_ws(b, mis.OiParams())
    assert code == 0 and n > 0
    # the slabs alone are 4 * sum(n * ld) floats
    assert n >= 4 * int(b.u_off[-1]) * 4


@pytest.mark.parametrize("kw,code", [
    (dict(n=[100], p=[101]), L.MI_ERR_CAPACITY),         # p > n
    (dict(n=[100], p=[10], ld=[48]), L.MI_ERR_CAPACITY),  # ld not a multiple of 32
    (dict(n=[100], p=[40], ld=[32]), L.MI_ERR_CAPACITY),  # ld < p
])
def test_bad_block_tables(kw, code):
    b = mis.Blocks(**kw)
    c, _ = _oi_ws(b, mis.OiParams())
    assert c == code
    assert L.lib().mi_last_error().decode() != ""


def test_predecessor_cycle_rejected():
    b = mis.Blocks([50, 50], p=[8, 8], pred=[1, 0])
    c, _ = _oi_ws(b, mis.OiParams())
    assert c == L.MI_ERR_ARG
    assert "cycle" in L.lib().mi_last_error().decode()


@pytest.mark.parametrize("field,value", [("m", 0), ("passes", 0), ("T", -1), ("precision", 7),
                                         ("a_mode", 9), ("max_sweeps", 0), ("jacobi_tol", 0.0),
                                         ("autotune", 2), ("eig", 5), ("rr_every", 3)])
def test_bad_params(field, value):
    b = mis.Blocks([100], p=[10])
    prm = mis.OiParams()
    setattr(prm, field, value)
    c, _ = _oi_ws(b, prm)
    assert c == L.MI_ERR_ARG


def test_slab_offsets_must_match():
    b = mis.Blocks([100, 60], p=[10, 10])
    b.u_off[1] += 32  # corrupt the table the struct points at
    c, _ = _oi_ws(b, mis.OiParams())
    assert c == L.MI_ERR_ARG


def test_laplacian_workspace_query_arity():
    b = mis.Blocks([10])
    n = C.c_size_t()
    off = np.array([0, 4], np.int64)
    ptr = off.ctypes.data_as(C.POINTER(C.c_int64))
    assert L.lib().mi_laplacian_workspace_size(b.ref, ptr, 4, C.byref(n)) == L.MI_ERR_ARG
    assert L.lib().mi_laplacian_workspace_size(b.ref, ptr, 3, C.byref(n)) == 0
    assert n.value > 0


def test_choose_and_encdec_workspace_queries():
    b = mis.Blocks([300, 500], p=[40, 64])
    n = C.c_size_t()
    assert L.lib().mi_choose_c_workspace_size(None, b.ref, C.byref(n)) == 0 and n.value > 0
    assert L.lib().mi_encdec_workspace_size(None, b.ref, L.MI_FP32, C.byref(n)) == 0 and n.value > 0
    assert L.lib().mi_encdec_workspace_size(None, b.ref, 5, C.byref(n)) == L.MI_ERR_ARG


def test_kernel_class_table_and_timer_arguments():
    import ctypes as C
    lib = L.lib()
    names = [lib.mi_kernel_class_name(k).decode() for k in range(L.MI_K_COUNT)]
    assert names == L.KERNEL_CLASSES
    assert lib.mi_kernel_class_name(-1) is None and lib.mi_kernel_class_name(L.MI_K_COUNT) is None
    ms = (C.c_double * L.MI_K_COUNT)()
    n = (C.c_int64 * L.MI_K_COUNT)()
    assert lib.mi_ctx_kernel_times(None, ms, n) == L.MI_ERR_ARG
    assert lib.mi_ctx_set_timing(None, 1) == L.MI_ERR_ARG


def test_residual_and_adjoint_workspace_queries():
    b = mis.Blocks([300, 500], p=[40, 64])
    n = C.c_size_t()
    assert L.lib().mi_residual_workspace_size(None, b.ref, C.byref(n)) == 0
    # one FP64 partial of ld per 16-row tile
    assert n.value == 8 * (19 * 64 + 32 * 64)
    nnz = np.array([0, 2000, 5500], np.int64)
    nnz_p = nnz.ctypes.data_as(C.POINTER(C.c_int64))
    ok = mis.OiParams(warm=mis.MI_WARM_GIVEN, adapt=0, T0=2, passes0=2, m0=4, a_mode=mis.MI_A_ABS,
                      a_value=1.0, b_abs=10.0)

    def q(prm, blocks=b):
        return L.lib().mi_adjoint_workspace_size(None, blocks.ref, C.byref(prm.struct()), nnz_p,
                                                 C.byref(n))

    assert q(ok) == 0 and n.value > 0
    # the interval schedule and the start are held constant by the reverse
    # sweep, whatever rule sets them
    for field, value in (("warm", mis.MI_WARM_PRED), ("adapt", 1), ("b_abs", 0.0),
                         ("a_mode", mis.MI_A_WEYL), ("warm", mis.MI_RANDOM)):
        assert q(mis.OiParams(**{**ok.__dict__, field: value})) == 0, field
    for field, value in (("rr_every", 1), ("eig", L.MI_EIG_JACOBI), ("T0", 0), ("tol", 1e-6),
                         ("precision", mis.MI_BF16_IN), ("op", mis.MI_OP_RZ)):
        bad = mis.OiParams(**{**ok.__dict__, field: value})
        assert q(bad) == L.MI_ERR_ARG, field
    # warm-started blocks with more passes than the roots need more checkpoints
    q(ok)
    n_root = n.value
    chain = mis.Blocks([300, 500], p=[40, 64], pred=[-1, 0])
    warm = mis.OiParams(**{**ok.__dict__, "warm": mis.MI_WARM_PRED, "T": 4, "passes": 2})
    assert q(warm, chain) == 0 and n.value > n_root
    assert q(mis.OiParams(**{**warm.__dict__, "T": 0}), chain) == L.MI_ERR_ARG
    wide = mis.Blocks([300, 500], p=[40, 200])
    assert q(ok, wide) == L.MI_ERR_ARG


def test_params_struct_layout_matches_header():
    # 14 int32 fields, 3 doubles, 4 int32 (operator fields), delta, tol, seed
    assert C.sizeof(L.MiOiParams) == 56 + 3 * 8 + 16 + 8 + 8 + 8
    assert L.MiOiParams.a_value.offset == 56 and L.MiOiParams.autotune.offset == 52
    assert L.MiOiParams.op.offset == 80 and L.MiOiParams.delta.offset == 96
    assert L.MiOiParams.tol.offset == 104 and L.MiOiParams.seed.offset == 112
    # the block table: n_blocks, then six pointers
    assert C.sizeof(L.MiBlocks) == 8 + 6 * 8 and L.MiBlocks.c.offset == 48


def test_tolerance_and_seeded_start_params():
    b = mis.Blocks([100, 80], p=[10, 12])
    assert _oi_ws(b, mis.OiParams(warm=mis.MI_RANDOM))[0] == 0
    assert _oi_ws(b, mis.OiParams(tol=1e-6, T=4, T0=4))[0] == 0
    for kw in (dict(warm=3), dict(tol=-1.0), dict(tol=1.5), dict(tol=1e-6, T0=0),
               dict(tol=1e-6, T=0)):
        assert _oi_ws(b, mis.OiParams(**kw))[0] == L.MI_ERR_ARG, kw
    # kept pairs outside [1, p_b]
    for c in ([0, 5], [11, 5], [10, 13]):
        bad = mis.Blocks([100, 80], p=[10, 12], c=c)
        assert _oi_ws(bad, mis.OiParams(tol=1e-6))[0] == L.MI_ERR_CAPACITY, c
    assert _oi_ws(mis.Blocks([100, 80], p=[10, 12], c=[10, 1]), mis.OiParams(tol=1e-6))[0] == 0
    # the dynamic walk has its own stopping rule and takes no seeded start
    dp = L.MiDoiParams(0.01, 0.02, 8, 5)
    n = C.c_size_t()
    for kw in (dict(warm=mis.MI_RANDOM), dict(tol=1e-6)):
        prm = mis.OiParams(**kw)
        assert L.lib().mi_doi_workspace_size(None, b.ref, C.byref(prm.struct()), C.byref(dp),
                                             C.byref(n)) == L.MI_ERR_ARG, kw


def test_quality_report_argument_checks():
    lib = L.lib()
    out = (C.c_double * 8)()
    assert lib.mi_mesh_quality(None, 10, None, None, 0, 0, None, None, None, out, None) == L.MI_ERR_ARG
    assert b"NULL" in lib.mi_last_error()
    assert mis.QUALITY_FIELDS[:2] == ("nmsve", "nmsve_db") and len(mis.QUALITY_FIELDS) == 8


def test_rz_operator_params():
    b = mis.Blocks([100], p=[10])
    assert _oi_ws(b, mis.OiParams(op=mis.MI_OP_RZ))[0] == 0
    for kw in (dict(op=2), dict(op=mis.MI_OP_RZ, z=0), dict(op=mis.MI_OP_RZ, z=17),
               dict(op=mis.MI_OP_RZ, cg_iters=0), dict(op=mis.MI_OP_RZ, delta=0.0)):
        assert _oi_ws(b, mis.OiParams(**kw))[0] == L.MI_ERR_ARG, kw
