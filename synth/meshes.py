"""Seeded synthetic meshes and block partitions.

This module only *generates inputs*: vertex coordinates, triangle faces,
vertex partitions into submeshes ("blocks"), block orders and random start
subspaces.  It contains none of the spectral method's arithmetic (no edge
extraction for the Laplacian, no Laplacian, no eigen-solves, no projection);
both the CPU oracle and the GPU library consume what it produces.

The paper evaluates on scanned and CAD meshes (Bunny, Armadillo, Hand, ...)
that are not available here; the generators below stand in for them with
meshes of the same kind (closed or open triangulated surfaces, ~6-regular
connectivity, smooth geometry plus noise) and the sizes the workloads name.
All randomness flows from ``numpy.random.SeedSequence`` so every input is
reproducible from one integer.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 181002719


def rng_for(*key: int) -> np.random.Generator:
    """A generator keyed by the master seed and a tuple of small integers."""
    return np.random.default_rng(np.random.SeedSequence([MASTER_SEED, *key]))


# ---------------------------------------------------------------------------
# Base meshes
# ---------------------------------------------------------------------------

def grid_mesh(nx: int = 32, ny: int = 32, span: float = 2 * np.pi):
    """Regular nx-by-ny vertex grid on [0, span]^2, each square split into two
    triangles along the (i,j)-(i+1,j+1) diagonal.  Vertex id = i*ny + j."""
    xs = np.linspace(0.0, span, nx)
    ys = np.linspace(0.0, span, ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), np.zeros(nx * ny)], axis=1)
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00 = i * ny + j
    v10 = (i + 1) * ny + j
    v01 = i * ny + j + 1
    v11 = (i + 1) * ny + j + 1
    f1 = np.stack([v00, v10, v11], axis=1)
    f2 = np.stack([v00, v11, v01], axis=1)
    faces = np.concatenate([f1, f2]).astype(np.int64)
    return verts, faces


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def icosahedron():
    return _icosahedron()


def tetrahedron():
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int64)
    return v, f


def octahedron():
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int64)
    return v, f


def icosphere(level: int):
    """Icosahedron refined `level` times by 4:1 midpoint subdivision, projected
    to the unit sphere.  V = 10*4^level + 2, F = 20*4^level."""
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        key = e[:, 0] * (nv + 1) + e[:, 1]
        ukey, inv = np.unique(key, return_inverse=True)
        a = ukey // (nv + 1)
        b = ukey % (nv + 1)
        mid = 0.5 * (v[a] + v[b])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        m01 = nv + inv[:nf]
        m12 = nv + inv[nf:2 * nf]
        m20 = nv + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)])
    return v, f


def geodesic_sphere(nu: int):
    """Class-I geodesic sphere of frequency nu: every icosahedron face is cut
    into nu^2 triangles on its barycentric grid, then projected to the unit
    sphere.  V = 10*nu^2 + 2, F = 20*nu^2."""
    iv, ifc = _icosahedron()
    # barycentric lattice (i, j, k), i + j + k = nu, local index in a face
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    keep = ii + jj <= nu
    ii = ii[keep]
    jj = jj[keep]
    kk = nu - ii - jj
    loc = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    loc[ii, jj] = np.arange(ii.size)
    npf = ii.size
    # a global key per lattice point: corner ids with non-zero weight, sorted
    corners = ifc  # (20, 3)
    W = np.stack([ii, jj, kk], 1)  # weight of corner 0, 1, 2
    ids = np.broadcast_to(corners[:, None, :], (20, npf, 3)).copy()
    w = np.broadcast_to(W[None], (20, npf, 3)).copy()
    ids[w == 0] = 12
    order = np.argsort(ids, axis=2, kind="stable")
    ids_s = np.take_along_axis(ids, order, 2)
    w_s = np.take_along_axis(w, order, 2)
    base = nu + 1
    key = (((ids_s[..., 0] * 13 + ids_s[..., 1]) * 13 + ids_s[..., 2]) * base * base * base
           + (w_s[..., 0] * base + w_s[..., 1]) * base + w_s[..., 2])
    ukey, first, inv = np.unique(key.ravel(), return_index=True, return_inverse=True)
    inv = inv.reshape(20, npf)
    # positions from the first occurrence
    fidx = first // npf
    pidx = first % npf
    P = (W[pidx, 0:1] * iv[corners[fidx, 0]] + W[pidx, 1:2] * iv[corners[fidx, 1]]
         + W[pidx, 2:3] * iv[corners[fidx, 2]]) / nu
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    # small triangles in each face
    ui, uj = np.meshgrid(np.arange(nu), np.arange(nu), indexing="ij")
    m = ui + uj <= nu - 1
    ui, uj = ui[m], uj[m]
    up = np.stack([loc[ui, uj], loc[ui + 1, uj], loc[ui, uj + 1]], 1)
    di, dj = np.meshgrid(np.arange(nu), np.arange(nu), indexing="ij")
    m = di + dj <= nu - 2
    di, dj = di[m], dj[m]
    dn = np.stack([loc[di + 1, dj], loc[di + 1, dj + 1], loc[di, dj + 1]], 1)
    tri = np.concatenate([up, dn])  # local lattice ids
    faces = inv[:, tri].reshape(-1, 3)
    return P, faces.astype(np.int64)


def torus_faces(a: int, b: int):
    """Triangulated a-by-b torus (periodic grid, diagonal (i,j)-(i+1,j+1)).
    Returns faces only; vertex id = i*b + j."""
    i, j = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00 = i * b + j
    v10 = ((i + 1) % a) * b + j
    v01 = i * b + (j + 1) % b
    v11 = ((i + 1) % a) * b + (j + 1) % b
    return np.concatenate([np.stack([v00, v10, v11], 1),
                           np.stack([v00, v11, v01], 1)]).astype(np.int64)


# ---------------------------------------------------------------------------
# Geometry: noise and deformation
# ---------------------------------------------------------------------------

def _wave_field(dirs, phases, pts, freq):
    return np.cos(freq * (pts @ dirs.T) + phases).sum(axis=1) / np.sqrt(dirs.shape[0])


def octave_noise(pts: np.ndarray, rng: np.random.Generator, octaves: int = 3, waves: int = 16):
    """Smooth seeded noise on R^3: sum over octaves o of 2^-o * s(2^o x), where
    s is a normalised sum of `waves` cosine plane waves in random directions."""
    out = np.zeros(pts.shape[0])
    for o in range(octaves):
        d = rng.normal(size=(waves, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        ph = rng.uniform(0, 2 * np.pi, size=waves)
        out += 2.0 ** (-o) * _wave_field(d, ph, pts, 2.0 ** o * 2.0)
    return out


def displaced_sphere(verts: np.ndarray, rng: np.random.Generator, amp: float = 0.05):
    """Radius 1 + amp * N3(v) with N3 the 3-octave noise above."""
    r = 1.0 + amp * octave_noise(verts, rng)
    return verts * r[:, None]


def delaunay_disk(n: int, rng: np.random.Generator, sigma: float = 0.01):
    """n points uniform in the unit disk, Delaunay-triangulated, with height
    z = 0.1 sin(pi x) cos(pi y) + N(0, sigma)."""
    from scipy.spatial import Delaunay
    r = np.sqrt(rng.uniform(size=n))
    th = 2 * np.pi * rng.uniform(size=n)
    x = r * np.cos(th)
    y = r * np.sin(th)
    faces = Delaunay(np.stack([x, y], 1)).simplices.astype(np.int64)
    z = 0.1 * np.sin(np.pi * x) * np.cos(np.pi * y) + rng.normal(scale=sigma, size=n)
    return np.stack([x, y, z], 1), faces


def vertex_normals_sphere(verts: np.ndarray):
    return verts / np.linalg.norm(verts, axis=1, keepdims=True)


def wave_frames(x0: np.ndarray, n_frames: int, rng: np.random.Generator,
                amp: float = 0.1, modes: int = 3):
    """Frames x_t = x0 + sum_j amp*sin(k_j.x0 - w_j t + phi_j) * n(x0) with
    seeded directions k_j (|k_j| = 2*pi*j), w_j = 2*pi*j/n_frames."""
    nrm = vertex_normals_sphere(x0)
    ks = []
    for j in range(1, modes + 1):
        d = rng.normal(size=3)
        ks.append(2 * np.pi * j * d / np.linalg.norm(d))
    phis = rng.uniform(0, 2 * np.pi, size=modes)
    frames = []
    for t in range(n_frames):
        disp = np.zeros(x0.shape[0])
        for j in range(modes):
            disp += amp * np.sin(x0 @ ks[j] - 2 * np.pi * (j + 1) * t / n_frames + phis[j])
        frames.append(x0 + disp[:, None] * nrm)
    return frames


# ---------------------------------------------------------------------------
# Partition into blocks
# ---------------------------------------------------------------------------

def vertex_adjacency(n: int, faces: np.ndarray):
    """CSR vertex adjacency used by the *partitioner* (region growing, BFS
    orders); not the Laplacian.  Returns (indptr, indices), sorted rows."""
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    e = e[(e[:, 0] >= 0) & (e[:, 1] >= 0) & (e[:, 0] != e[:, 1])]
    e = np.concatenate([e, e[:, ::-1]])
    key = np.unique(e[:, 0] * n + e[:, 1])
    src = key // n
    dst = key % n
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, src + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, dst.astype(np.int64)


def farthest_point_seeds(pts: np.ndarray, k: int, rng: np.random.Generator):
    """k seed vertices by Euclidean farthest-point sampling from a seeded
    random first vertex (spreads the regions evenly)."""
    first = int(rng.integers(pts.shape[0]))
    seeds = [first]
    d = ((pts - pts[first]) ** 2).sum(1)
    for _ in range(k - 1):
        s = int(np.argmax(d))
        seeds.append(s)
        d = np.minimum(d, ((pts - pts[s]) ** 2).sum(1))
    return np.asarray(seeds, dtype=np.int64)


def region_grow(indptr, indices, n_blocks: int, rng: np.random.Generator, pts=None):
    """Synchronous multi-source BFS from `n_blocks` seed vertices (farthest-point
    samples of `pts` when given, else uniform without replacement); each
    round every region claims the unassigned neighbours of its frontier, a
    vertex reached by several regions in the same round goes to the lowest
    region id.  Returns (label per vertex, seed vertex per region)."""
    n = indptr.size - 1
    if pts is not None:
        seeds = farthest_point_seeds(pts, n_blocks, rng)
    else:
        seeds = rng.choice(n, size=n_blocks, replace=False)
    label = -np.ones(n, dtype=np.int64)
    label[seeds] = np.arange(n_blocks)
    frontier = seeds.copy()
    deg = np.diff(indptr)
    while frontier.size:
        counts = deg[frontier]
        src = np.repeat(frontier, counts)
        starts = indptr[frontier]
        offs = np.arange(counts.sum()) - np.repeat(np.cumsum(counts) - counts, counts)
        nb = indices[np.repeat(starts, counts) + offs]
        cand_lab = label[src]
        m = label[nb] < 0
        nb = nb[m]
        cand_lab = cand_lab[m]
        if nb.size == 0:
            break
        best = np.full(n, np.iinfo(np.int64).max)
        np.minimum.at(best, nb, cand_lab)
        newv = np.unique(nb)
        label[newv] = best[newv]
        frontier = newv
    if (label < 0).any():  # disconnected leftovers join region 0
        label[label < 0] = 0
    return label, seeds


def bfs_order(indptr, indices, members: np.ndarray, start: int):
    """BFS order of the subgraph induced by `members`, from `start`, neighbours
    visited in ascending id; vertices unreachable from `start` follow in
    ascending id, each starting a new BFS."""
    inset = np.zeros(indptr.size - 1, dtype=bool)
    inset[members] = True
    seen = np.zeros_like(inset)
    out = []
    pending = [start] + sorted(int(x) for x in members)
    from collections import deque
    for s in pending:
        if seen[s] or not inset[s]:
            continue
        seen[s] = True
        q = deque([s])
        while q:
            u = q.popleft()
            out.append(u)
            for v in indices[indptr[u]:indptr[u + 1]]:
                if inset[v] and not seen[v]:
                    seen[v] = True
                    q.append(v)
    return np.asarray(out, dtype=np.int64)


def split_blocks(n: int, faces: np.ndarray, label: np.ndarray, seeds: np.ndarray):
    """Per block: global vertex ids in canonical (BFS-from-seed) order, and the
    faces that have at least two vertices in the block, rewritten to
    block-local ids with -1 marking a corner outside the block."""
    indptr, indices = vertex_adjacency(n, faces)
    nb = seeds.size
    blocks = []
    flab = label[faces]  # (F, 3)
    for b in range(nb):
        members = np.nonzero(label == b)[0]
        order = bfs_order(indptr, indices, members, int(seeds[b]))
        g2l = -np.ones(n, dtype=np.int64)
        g2l[order] = np.arange(order.size)
        inb = (flab == b)
        fsel = faces[inb.sum(1) >= 2]
        lf = g2l[fsel]
        blocks.append((order, lf))
    return blocks


def overlap_extend(indptr, indices, label: np.ndarray, n_parts: int, n_d: int):
    """Equal-size overlapped submeshes (Section 6.1): every part is extended
    with the neighbours of its boundary vertices in adjacent parts, ring
    after ring, until it holds n_d vertices; from the ring that would
    overshoot, the lowest global ids are taken.  A part whose connected
    surroundings hold fewer than n_d vertices keeps all of them.  Returns the
    sorted global vertex ids of every extended part."""
    n = indptr.size - 1
    out = []
    for b in range(n_parts):
        inset = label == b
        members = list(np.nonzero(inset)[0])
        frontier = np.asarray(members, dtype=np.int64)
        while len(members) < n_d and frontier.size:
            counts = indptr[frontier + 1] - indptr[frontier]
            starts = np.repeat(indptr[frontier], counts)
            offs = np.arange(counts.sum()) - np.repeat(np.cumsum(counts) - counts, counts)
            ring = np.unique(indices[starts + offs])
            ring = ring[~inset[ring]]
            take = ring[: n_d - len(members)]
            inset[take] = True
            members.extend(int(v) for v in take)
            frontier = take
        out.append(np.sort(np.asarray(members, dtype=np.int64)))
    return out


def split_members(n: int, faces: np.ndarray, members: list, seeds: np.ndarray):
    """As split_blocks, for explicit (possibly overlapping) vertex sets: per
    block the global ids in BFS-from-seed order and the faces with at least
    two vertices in the block, in block-local ids (-1 = corner outside)."""
    indptr, indices = vertex_adjacency(n, faces)
    blocks = []
    for b, mem in enumerate(members):
        order = bfs_order(indptr, indices, mem, int(seeds[b]))
        g2l = -np.ones(n, dtype=np.int64)
        g2l[order] = np.arange(order.size)
        lf_all = g2l[faces]
        fsel = (lf_all >= 0).sum(1) >= 2
        blocks.append((order, lf_all[fsel]))
    return blocks


def block_graph_order(n: int, faces: np.ndarray, label: np.ndarray, n_blocks: int,
                      rng: np.random.Generator, n_roots: int = 1):
    """Block processing order: a seeded first block (and, for n_roots > 1,
    further first blocks chosen farthest-first on the block graph: each the
    block at the largest BFS distance from those already chosen, ties by
    block id), then multi-source BFS over the block adjacency graph (blocks
    adjacent when a mesh edge joins them), ties by block id.  Returns
    (order, pred, level) with pred = BFS parent (-1 for first blocks) and
    level = BFS depth."""
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    la = label[e[:, 0]]
    lb = label[e[:, 1]]
    m = la != lb
    pairs = np.unique(np.stack([la[m], lb[m]], 1), axis=0)
    adj = [[] for _ in range(n_blocks)]
    for a, b in pairs:
        adj[a].append(int(b))
    for a in range(n_blocks):
        adj[a] = sorted(set(adj[a]))
    from collections import deque

    def depth(srcs):
        d = -np.ones(n_blocks, dtype=np.int64)
        dq = deque(srcs)
        for r in srcs:
            d[r] = 0
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if d[v] < 0:
                    d[v] = d[u] + 1
                    dq.append(v)
        return d

    roots = [int(rng.integers(n_blocks))]
    while len(roots) < min(n_roots, n_blocks):
        roots.append(int(np.argmax(depth(roots))))
    pred = -np.ones(n_blocks, dtype=np.int64)
    level = -np.ones(n_blocks, dtype=np.int64)
    order = list(roots)
    level[roots] = 0
    q = deque(roots)
    while q:
        u = q.popleft()
        for v in adj[u]:
            if level[v] < 0:
                level[v] = level[u] + 1
                pred[v] = u
                order.append(v)
                q.append(v)
    for b in range(n_blocks):  # disconnected block graph: new roots
        if level[b] < 0:
            level[b] = 0
            order.append(b)
    return np.asarray(order), pred, level


def random_orthonormal(n: int, p: int, rng: np.random.Generator):
    """Seeded random start subspace: Gaussian n-by-p, orthonormalised by
    Householder QR (this is an *input* of the tracking, not a step of it)."""
    g = rng.normal(size=(n, p))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]
