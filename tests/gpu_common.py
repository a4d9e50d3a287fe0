"""Shared helpers of the GPU parity tests: upload a seeded workload through
the binding, and the oracle's per-block reference (eigh) with caching."""
from __future__ import annotations

import functools

import numpy as np
import torch

import paper_1810_02719_amd as mis
from oracle import laplacian as lap
from oracle import spectral as S
from synth import workloads as W


class Uploaded:
    def __init__(self, bs: W.BlockSet, ld=None, device="cuda:0"):
        fl = W.flatten(bs, ld)
        self.bs = bs
        self.fl = fl
        self.blocks = mis.Blocks(bs.n, p=fl["p"], ld=fl["ld"], pred=bs.pred)
        self.prim_off = fl["prim_off"]
        self.prims = torch.from_numpy(np.ascontiguousarray(fl["prims"].reshape(-1))).to(device)
        self.coords = torch.from_numpy(np.ascontiguousarray(fl["coords"].reshape(-1))).to(device)
        self.device = device

    def laplacian(self, ctx, mode=mis.MI_W_COMBINATORIAL):
        return mis.build_laplacian(ctx, self.blocks, self.prim_off, self.prims, 3, self.coords, mode)

    def X32(self, b):
        return self.fl["coords"][self.blocks.v_off[b]:self.blocks.v_off[b + 1]].astype(np.float64)

    def slab(self, V, b):
        n, ld = int(self.blocks.n[b]), int(self.blocks.ld[b])
        return V[int(self.blocks.u_off[b]):int(self.blocks.u_off[b + 1])].view(n, ld).double().cpu().numpy()

    def starts(self, dtype=torch.float32, key=(9,)):
        """Seeded orthonormal start for every block, laid out as a slab."""
        V0 = np.zeros(int(self.blocks.u_off[-1]))
        for b, Q in enumerate(W.random_starts(self.bs, key)):
            n, ld = int(self.blocks.n[b]), int(self.blocks.ld[b])
            s = V0[int(self.blocks.u_off[b]):int(self.blocks.u_off[b + 1])].reshape(n, ld)
            s[:, :Q.shape[1]] = Q
        return torch.from_numpy(V0).to(dtype).to(self.device)


@functools.lru_cache(maxsize=None)
def _oracle(key, faces_bytes, fshape, coords_bytes, n, mode, k):
    faces = np.frombuffer(faces_bytes, dtype=np.int64).reshape(fshape)
    X = np.frombuffer(coords_bytes, dtype=np.float64).reshape(n, 3)
    e = lap.canonical_edges(faces, n)
    w = lap.edge_weights(e, X, mode)
    L = lap.laplacian_dense(n, e, w)
    lam, U = S.eigh_lowest(L, k)
    return L, lam, U


def oracle_block(up: Uploaded, b, mode=lap.COMBINATORIAL, k=None):
    """(dense L, ascending eigenvalues, eigenvectors) of block b in FP64 from the
    same FP32 coordinates the GPU sees."""
    f = np.ascontiguousarray(up.bs.faces[b].astype(np.int64))
    X = np.ascontiguousarray(up.X32(b))
    return _oracle((up.bs.name, b), f.tobytes(), f.shape, X.tobytes(), X.shape[0], mode, k)
