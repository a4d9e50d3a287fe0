"""Seeded block workloads: each is a list of submeshes (block-local vertex
coordinates and faces) with a processing order, warm-start predecessors and
the subspace sizes to track.  Input generation only (see ``meshes``).

Faces are block-local; a corner outside the block is -1 (the face still
contributes its in-block edge).  Vertices of a block are in BFS order from the
block's seed vertex.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes as M


@dataclass
class BlockSet:
    name: str
    coords: list            # per block (n_b, 3) float64, block-local order
    faces: list             # per block (F_b, 3) int64, local ids, -1 = outside
    pred: np.ndarray        # warm-start predecessor per block (-1 none)
    level: np.ndarray       # BFS depth in the block order
    order: np.ndarray       # processing order
    c: np.ndarray           # kept subspace size per block
    p: np.ndarray           # tracked width per block (>= c)
    global_ids: list = field(default_factory=list)  # per block: global vertex ids
    n_global: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return np.array([x.shape[0] for x in self.coords], dtype=np.int64)

    @property
    def n_blocks(self):
        return len(self.coords)


def ld_for(p):
    return ((np.asarray(p) + 31) // 32) * 32


def flatten(bs: BlockSet, ld=None):
    """Concatenated arrays in the layout the C ABI takes: v_off, prim_off,
    prims (int32), coords (float32, n x 3), u_off for a row-major n_b x ld_b
    slab per block."""
    n = bs.n
    p = np.asarray(bs.p, dtype=np.int64)
    ld = ld_for(p) if ld is None else np.asarray(ld, dtype=np.int64)
    v_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    nf = np.array([f.shape[0] for f in bs.faces], dtype=np.int64)
    prim_off = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)
    prims = np.concatenate(bs.faces).astype(np.int32) if nf.sum() else np.zeros((0, 3), np.int32)
    coords = np.concatenate(bs.coords).astype(np.float32)
    u_off = np.concatenate([[0], np.cumsum(n * ld)]).astype(np.int64)
    return dict(v_off=v_off, prim_off=prim_off, prims=prims, coords=coords,
                p=p.astype(np.int32), ld=ld.astype(np.int32), u_off=u_off,
                pred=np.asarray(bs.pred, dtype=np.int32),
                c=np.asarray(bs.c, dtype=np.int32))


def _partitioned(name, verts, faces, n_blocks, key, c, p, n_roots=1):
    n = verts.shape[0]
    indptr, indices = M.vertex_adjacency(n, faces)
    label, seeds = M.region_grow(indptr, indices, n_blocks, M.rng_for(*key, 1), pts=verts)
    blocks = M.split_blocks(n, faces, label, seeds)
    order, pred, level = M.block_graph_order(n, faces, label, n_blocks, M.rng_for(*key, 2),
                                             n_roots)
    coords = [verts[g] for g, _ in blocks]
    fl = [f for _, f in blocks]
    nb = len(blocks)
    return BlockSet(name=name, coords=coords, faces=fl, pred=pred, level=level, order=order,
                    c=np.full(nb, c), p=np.full(nb, p), global_ids=[g for g, _ in blocks],
                    n_global=n, extra=dict(label=label, seeds=seeds, faces_global=faces))


def overlapped(name, verts, faces, n_blocks, key, c, p, overlap=0.15, n_roots=1):
    """Region-grown parts extended to equal-size overlapped submeshes of
    n_d = ceil((1 + overlap) * max part size) vertices (Section 6.1; the paper
    finds 15 % sufficient).  The block order and the warm-start predecessors
    follow the parts' adjacency, as for non-overlapping blocks."""
    n = verts.shape[0]
    indptr, indices = M.vertex_adjacency(n, faces)
    label, seeds = M.region_grow(indptr, indices, n_blocks, M.rng_for(*key, 1), pts=verts)
    sizes = np.bincount(label, minlength=n_blocks)
    n_d = int(np.ceil((1.0 + overlap) * sizes.max()))
    members = M.overlap_extend(indptr, indices, label, n_blocks, n_d)
    blocks = M.split_members(n, faces, members, seeds)
    order, pred, level = M.block_graph_order(n, faces, label, n_blocks, M.rng_for(*key, 2),
                                             n_roots)
    nb = len(blocks)
    return BlockSet(name=name, coords=[verts[g] for g, _ in blocks], faces=[f for _, f in blocks],
                    pred=pred, level=level, order=order, c=np.full(nb, c), p=np.full(nb, p),
                    global_ids=[g for g, _ in blocks], n_global=n,
                    extra=dict(label=label, seeds=seeds, faces_global=faces, n_d=n_d,
                               verts_global=verts))


def icosphere_overlapped(level=7, n_blocks=100, c=100, p=192, amp=0.05, overlap=0.15, key=(2,),
                         n_roots=1):
    """The static icosphere workload with overlapped equal-size submeshes
    (same mesh, same parts as icosphere_blocks with the same key)."""
    v, f = M.icosphere(level)
    v = M.displaced_sphere(v, M.rng_for(*key, 0), amp)
    name = f"icosphere{level}_b{n_blocks}_ov{int(round(100 * overlap))}"
    return overlapped(name, v, f, n_blocks, key, c, p, overlap, n_roots)


def grid_single(nx=32, ny=32, c=50, p=75, sigma=1e-3, key=(1,)):
    """Single submesh: nx-by-ny grid on [0, 2pi]^2, z = 0.1 sin x cos y + N(0, sigma)."""
    v, f = M.grid_mesh(nx, ny)
    rng = M.rng_for(*key)
    v[:, 2] = 0.1 * np.sin(v[:, 0]) * np.cos(v[:, 1]) + rng.normal(scale=sigma, size=v.shape[0])
    return BlockSet(name=f"grid{nx}x{ny}", coords=[v], faces=[f], pred=np.array([-1]),
                    level=np.array([0]), order=np.array([0]), c=np.array([c]), p=np.array([p]),
                    global_ids=[np.arange(v.shape[0])], n_global=v.shape[0])


def icosphere_blocks(level=7, n_blocks=100, c=100, p=150, amp=0.05, key=(2,), n_roots=1):
    """Static block sequence: displaced icosphere split by region growing;
    n_roots first blocks (cold starts), every other block warm-started from
    its BFS parent."""
    v, f = M.icosphere(level)
    v = M.displaced_sphere(v, M.rng_for(*key, 0), amp)
    name = f"icosphere{level}_b{n_blocks}" + (f"_r{n_roots}" if n_roots > 1 else "")
    return _partitioned(name, v, f, n_blocks, key, c, p, n_roots)


def disk_blocks(n_blocks=1024, n_min=500, n_max=5000, c_max=256, p_max=320, key=(3,)):
    """Batched uneven: independent Delaunay disks of U{n_min..n_max} vertices."""
    rng = M.rng_for(*key, 0)
    sizes = rng.integers(n_min, n_max + 1, size=n_blocks)
    coords, faces, gids = [], [], []
    for b, nb in enumerate(sizes):
        v, fc = M.delaunay_disk(int(nb), M.rng_for(*key, 1, b))
        # canonical order: BFS from the vertex nearest the centre
        indptr, indices = M.vertex_adjacency(v.shape[0], fc)
        start = int(np.argmin((v[:, :2] ** 2).sum(1)))
        order = M.bfs_order(indptr, indices, np.arange(v.shape[0]), start)
        g2l = np.empty_like(order)
        g2l[order] = np.arange(order.size)
        coords.append(v[order])
        faces.append(g2l[fc])
        gids.append(order)
    p = np.minimum(p_max, sizes)
    c = np.minimum(c_max, p)
    return BlockSet(name=f"disks{n_blocks}", coords=coords, faces=faces,
                    pred=-np.ones(n_blocks, dtype=np.int64), level=np.zeros(n_blocks, np.int64),
                    order=np.arange(n_blocks), c=c, p=p, global_ids=gids, n_global=int(sizes.sum()))


def sample_blocks(n, k=64, key=(97,)):
    """Seeded sample of k block indices of a set with block sizes n (without
    replacement), always including the smallest and the largest block;
    ascending."""
    n = np.asarray(n)
    rng = M.rng_for(*key)
    pick = rng.choice(n.size, size=min(k, n.size), replace=False)
    return np.array(sorted({int(np.argmin(n)), int(np.argmax(n)), *map(int, pick)}))


def geodesic_blocks(nu=316, n_blocks=100, c=200, p=256, amp=0.05, key=(4,)):
    """Precision workload: displaced geodesic sphere (10 nu^2 + 2 vertices)."""
    v, f = M.geodesic_sphere(nu)
    v = M.displaced_sphere(v, M.rng_for(*key, 0), amp)
    return _partitioned(f"geodesic{nu}_b{n_blocks}", v, f, n_blocks, key, c, p)


def dynamic_frames(nu=100, n_blocks=64, n_frames=60, c=150, p=192, key=(5,)):
    """Dynamic workload: fixed connectivity, frames deformed by 3 waves.
    Returns the BlockSet of frame 0 and a list of per-frame block coords."""
    v, f = M.geodesic_sphere(nu)
    bs = _partitioned(f"dyn{nu}_b{n_blocks}", v, f, n_blocks, key, c, p)
    frames = M.wave_frames(v, n_frames, M.rng_for(*key, 3))
    per_frame = [[fr[g] for g in bs.global_ids] for fr in frames]
    bs.coords = per_frame[0]
    # frames are independent of the block order: every block warm-starts from
    # itself in the previous frame
    bs.extra["frames"] = per_frame
    return bs


def random_starts(bs: BlockSet, key=(9,)):
    """Seeded orthonormal n_b x p_b start per block (float64)."""
    return [M.random_orthonormal(int(x.shape[0]), int(pb), M.rng_for(*key, b))
            for b, (x, pb) in enumerate(zip(bs.coords, bs.p))]
