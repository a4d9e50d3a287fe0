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


if __name__ == "__main__":
    grid32()
