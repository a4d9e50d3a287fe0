"""The allocation-free projection (mi_project_noalloc) against mi_project
through the C ABI: the same kernels on the same inputs, so the coefficients
agree bit for bit; two calls in a row, the second with a smaller block
table (the fixed scratch keeps the first call's contents), in FP32 and
FP64, and a block table too large for the fixed scratch is refused before
anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1810_02719_amd as mis
from paper_1810_02719_amd import _lib as L
from synth import workloads as W

from gpu_common import Uploaded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = mis.Context(0)
    yield c
    c.close()


def _case(level, nb, p, key, precision):
    bs = W.icosphere_blocks(level=level, n_blocks=nb, c=p // 2, p=p, key=key)
    up = Uploaded(bs)
    dt = torch.float64 if precision == mis.MI_FP64 else torch.float32
    U = up.starts(dt, key=(71, level))
    X = up.coords.to(dt)
    rng = np.random.default_rng(level)
    c = torch.from_numpy(rng.integers(1, p + 1, nb).astype(np.int32)).cuda()
    return up, U, X, c, dt


@pytest.mark.parametrize("precision", [mis.MI_FP32, mis.MI_FP64], ids=["fp32", "fp64"])
def test_noalloc_projection_matches_workspace_projection(ctx, precision):
    # first a larger table, then a smaller one (ld 256 -> 64, 60 -> 5 blocks)
    for level, nb, p in ((6, 60, 256), (4, 5, 64)):
        up, U, X, c, dt = _case(level, nb, p, (40 + level,), precision)
        n = int(up.blocks.t_off[-1]) * 3
        E_ref = mis.project(ctx, up.blocks, c, U, X, precision=precision)
        E = torch.full((n,), float("nan"), dtype=dt, device="cuda:0")
        mis.project_noalloc(ctx, up.blocks, c, U, X, E, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(E, E_ref), (level, (E - E_ref).abs().max().item())


def test_noalloc_projection_refuses_tables_beyond_the_scratch(ctx):
    # 200 blocks at ld = 256 need about 19.7 MB of partials (> 16 MiB)
    n = np.full(200, 300, np.int64)
    blocks = mis.Blocks(n, p=np.full(200, 256))
    U = torch.zeros(int(blocks.u_off[-1]), dtype=torch.float32, device="cuda:0")
    X = torch.zeros(int(blocks.v_off[-1]) * 3, dtype=torch.float32, device="cuda:0")
    E = torch.zeros(int(blocks.t_off[-1]) * 3, dtype=torch.float32, device="cuda:0")
    c = torch.ones(200, dtype=torch.int32, device="cuda:0")
    st = L.lib().mi_project_noalloc(ctx.h, blocks.ref, mis.MI_FP32, C.c_void_p(c.data_ptr()),
                                    C.c_void_p(U.data_ptr()), C.c_void_p(X.data_ptr()),
                                    C.c_void_p(E.data_ptr()), C.c_void_p(0))
    assert st == L.MI_ERR_WORKSPACE
    assert b"scratch" in L.lib().mi_last_error()
    torch.cuda.synchronize()
    assert int(E.abs().sum()) == 0
