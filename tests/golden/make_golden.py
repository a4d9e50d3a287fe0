"""Writes the stored expected values under tests/golden/ by calling only the
CPU oracle on the seeded inputs.  Run from the repo root:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import laplacian as lap, metrics as met, spectral as S  # noqa: E402
from synth import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def grid32():
    bs = W.grid_single()
    X = bs.coords[0]
    n = X.shape[0]
    e = lap.canonical_edges(bs.faces[0], n)
    L = lap.laplacian_dense(n, e, np.ones(len(e)))
    lam, U = S.eigh_lowest(L)
    G = met.gl_matrix(n, e, X)
    c = int(bs.c[0])
    Xr = S.encode_decode(U[:, :c], X)
    with open(os.path.join(HERE, "grid32_combinatorial.txt"), "w") as f:
        f.write("# 32x32 grid workload (Section 3 combinatorial L = D - A), seeded coords;\n")
        f.write("# written by tests/golden/make_golden.py from the FP64 oracle (eigh).\n")
        f.write(f"n {n}\nedges {e.shape[0]}\nnnz {n + 2 * e.shape[0]}\n")
        f.write("lambda_1_to_76 " + " ".join(f"{x:.17g}" for x in lam[:76]) + "\n")
        f.write(f"nmsve_c50 {met.nmsve(X, Xr, G):.17g}\n")
        f.write(f"l2_residual_c50 {np.linalg.norm(X - Xr):.17g}\n")


def c3_target():
    """Calibrated NMSVE target of the batched-uneven workload (1,024 disks):
    the literal target 1e-4 is met by no block with c <= 256, so the choice
    of c is also run at the median over a seeded sample of 64 blocks (plus
    the smallest and the largest) of NMSVE(c = 128) (Eq. 16, original edge
    lengths in GL), from the oracle's eigenvectors."""
    bs = W.disk_blocks()
    sample = W.sample_blocks(bs.n)
    vals = []
    for b in sample:
        X = bs.coords[b].astype(np.float32).astype(np.float64)
        n = X.shape[0]
        e = lap.canonical_edges(bs.faces[b], n)
        _, U = S.eigh_lowest(lap.laplacian_dense(n, e, np.ones(len(e))), 128)
        vals.append(met.nmsve_curve_sparse(U, X, e, X, 128)[-1])
    with open(os.path.join(HERE, "c3_calibrated_target.txt"), "w") as f:
        f.write("# Batched-uneven workload (1,024 Delaunay disks, combinatorial L): median over\n")
        f.write("# the seeded 64-block sample (plus smallest and largest) of NMSVE(c = 128),\n")
        f.write("# Section 8 Eq. 16 with GL on the original edge lengths, coordinates rounded\n")
        f.write("# to FP32 as the GPU sees them; written by tests/golden/make_golden.py from\n")
        f.write("# the FP64 oracle (eigh).\n")
        f.write(f"blocks {len(sample)}\n")
        f.write(f"target {float(np.median(vals)):.17g}\n")
        f.write(f"min {float(np.min(vals)):.17g}\nmax {float(np.max(vals)):.17g}\n")


if __name__ == "__main__":
    which = sys.argv[1:] or ["grid32", "c3_target"]
    if "grid32" in which:
        grid32()
    if "c3_target" in which:
        c3_target()
