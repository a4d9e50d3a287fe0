"""Pins of the CPU oracle against mathematics that shares no code with it:
closed-form spectra, exact integer arithmetic, brute force and identities.

Each test names the part of the paper it fixes.  None of them recomputes an
oracle formula with the same library call it makes.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from oracle import iterations as it
from oracle import codec as cd
from oracle import laplacian as lap
from oracle import merge as mg
from oracle import metrics as met
from oracle import spectral as S
from synth import meshes as M
from synth import workloads as W


def path_edges(n):
    return np.stack([np.arange(n - 1), np.arange(1, n)], 1)


def cycle_edges(n):
    return np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)


def grid_edges(a, b):
    idx = np.arange(a * b).reshape(a, b)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)
    return np.concatenate([h, v])


def comb_L(prims, n):
    e = lap.canonical_edges(prims, n)
    return e, lap.laplacian_dense(n, e, np.ones(len(e)))


# ---------------------------------------------------------------- Section 3, Eq. 1-2

class TestLaplacianInvariants:
    @pytest.fixture(scope="class")
    def block(self):
        bs = W.icosphere_blocks(level=4, n_blocks=6, c=20, p=30)
        return bs

    def test_csr_matches_dense_and_invariants(self, block):
        for b in range(block.n_blocks):
            X = block.coords[b]
            n = X.shape[0]
            for mode in (lap.COMBINATORIAL, lap.INV_SQ_DIST):
                e = lap.canonical_edges(block.faces[b], n)
                w = lap.edge_weights(e, X, mode)
                L = lap.laplacian_dense(n, e, w)
                rp, col, val = lap.laplacian_csr(n, e, w)
                # CSR structure: diagonal present, columns ascending, degree = nnz - 1
                for i in range(n):
                    cols = col[rp[i]:rp[i + 1]]
                    assert i in cols
                    assert np.all(np.diff(cols) > 0)
                deg = np.zeros(n, dtype=int)
                np.add.at(deg, e[:, 0], 1)
                np.add.at(deg, e[:, 1], 1)
                assert np.array_equal(np.diff(rp) - 1, deg)
                tol = 0.0 if mode == lap.COMBINATORIAL else 1e-14 * np.abs(L).max()
                assert np.abs(lap.csr_to_dense(n, rp, col, val) - L).max() <= tol
                # symmetric, zero row sums, PSD, trace = 2 sum w
                assert np.array_equal(L, L.T)
                assert np.abs(L.sum(1)).max() <= 1e-12 * max(1.0, np.abs(L).max())
                lam = np.linalg.eigvalsh(L)
                assert lam.min() >= -1e-10 * lam.max()
                assert math.isclose(np.trace(L), 2 * w.sum(), rel_tol=1e-12)

    def test_null_space_dimension_is_component_count(self):
        # two disjoint triangles + an isolated vertex: 3 components
        f = np.array([[0, 1, 2], [3, 4, 5]])
        e, L = comb_L(f, 7)
        lam = np.linalg.eigvalsh(L)
        assert int((np.abs(lam) < 1e-12).sum()) == 3
        # the constant vector is always in the null space
        assert np.abs(L @ np.ones(7)).max() == 0

    def test_outside_corner_and_degenerate_faces(self):
        # -1 corner drops its edges; repeated corner gives no self loop
        f = np.array([[0, 1, -1], [1, 1, 2], [2, 0, 1], [0, 1, 2]])
        e = lap.canonical_edges(f, 3)
        assert e.tolist() == [[0, 1], [0, 2], [1, 2]]
        with pytest.raises(lap.IndexError_):
            lap.canonical_edges(np.array([[0, 1, 3]]), 3)
        with pytest.raises(lap.DegenerateError):
            lap.edge_weights(np.array([[0, 1]]), np.zeros((2, 3)), lap.INV_SQ_DIST)

    def test_literal_mixed_form_is_not_a_laplacian(self):
        # reading of Eq. 1-2: D = |N(i)| with weighted C breaks L 1 = 0
        v, f = M.octahedron()
        v = v * np.array([1.0, 2.0, 0.5])
        e = lap.canonical_edges(f, 6)
        w = lap.edge_weights(e, v, lap.INV_SQ_DIST)
        Lm = lap.laplacian_literal_mixed(6, e, w)
        assert np.abs(Lm.sum(1)).max() > 1e-3
        Lw = lap.laplacian_dense(6, e, w)
        assert np.abs(Lw.sum(1)).max() < 1e-12


# ---------------------------------------------------------------- Eq. 3, closed forms

class TestClosedFormSpectra:
    @pytest.mark.parametrize("n", [2, 5, 17, 64])
    def test_path(self, n):
        _, L = comb_L(path_edges(n), n)
        k = np.arange(n)
        ref = np.sort(2 - 2 * np.cos(k * np.pi / n))
        lam, U = S.eigh_lowest(L)
        assert np.abs(lam - ref).max() < 1e-12
        # eigenvectors cos(k pi (i + 1/2) / n): subspace pins for every c
        i = np.arange(n)
        Uref = np.cos(np.pi * np.outer(i + 0.5, k) / n)
        for c in range(1, n):
            assert S.sin_theta_max(Uref[:, :c], U[:, :c]) < 1e-9

    @pytest.mark.parametrize("n", [3, 8, 31])
    def test_cycle(self, n):
        _, L = comb_L(cycle_edges(n), n)
        ref = np.sort(2 - 2 * np.cos(2 * np.pi * np.arange(n) / n))
        assert np.abs(np.linalg.eigvalsh(L) - ref).max() < 1e-12

    @pytest.mark.parametrize("a,b", [(3, 4), (7, 5), (10, 10)])
    def test_grid_product(self, a, b):
        _, L = comb_L(grid_edges(a, b), a * b)
        pa = 2 - 2 * np.cos(np.pi * np.arange(a) / a)
        pb = 2 - 2 * np.cos(np.pi * np.arange(b) / b)
        ref = np.sort((pa[:, None] + pb[None, :]).ravel())
        assert np.abs(np.linalg.eigvalsh(L) - ref).max() < 1e-11

    @pytest.mark.parametrize("a,b", [(3, 3), (7, 9), (12, 5)])
    def test_triangulated_torus_from_faces(self, a, b):
        f = M.torus_faces(a, b)
        _, L = comb_L(f, a * b)
        t1 = 2 * np.pi * np.arange(a)[:, None] / a
        t2 = 2 * np.pi * np.arange(b)[None, :] / b
        ref = np.sort((6 - 2 * np.cos(t1) - 2 * np.cos(t2) - 2 * np.cos(t1 + t2)).ravel())
        assert np.abs(np.linalg.eigvalsh(L) - ref).max() < 1e-11

    def test_platonic_solids(self):
        r5 = 5 ** 0.5
        cases = {
            "tetrahedron": (M.tetrahedron(), [0, 4, 4, 4]),
            "octahedron": (M.octahedron(), [0, 4, 4, 4, 6, 6]),
            "icosahedron": (M.icosahedron(), [0] + [5 - r5] * 3 + [6] * 5 + [5 + r5] * 3),
        }
        for name, ((v, f), ref) in cases.items():
            _, L = comb_L(f, v.shape[0])
            assert np.abs(np.linalg.eigvalsh(L) - np.array(ref)).max() < 1e-12, name

    def test_golden_platonic_fixture(self):
        # tests/golden/platonic_spectra.txt holds the closed forms written out
        import os
        path = os.path.join(os.path.dirname(__file__), "golden", "platonic_spectra.txt")
        got = {}
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            name, vals = line.split(":")
            got[name.strip()] = [float(x) for x in vals.split()]
        for name, (v, f) in {"tetrahedron": M.tetrahedron(), "octahedron": M.octahedron(),
                             "icosahedron": M.icosahedron()}.items():
            _, L = comb_L(f, v.shape[0])
            assert np.abs(np.linalg.eigvalsh(L) - np.array(got[name])).max() < 1e-12


# ---------------------------------------------------------------- brute force, <= 10 vertices

def small_meshes():
    out = {}
    v, f = M.octahedron()
    out["octahedron"] = (6, f)
    v, f = M.grid_mesh(3, 3)
    out["grid3x3"] = (9, f)
    # a fan of 7 triangles around vertex 0 (9 vertices, open)
    fan = np.array([[0, i, i + 1] for i in range(1, 8)])
    out["fan9"] = (9, fan)
    # 10-vertex strip with one -1 corner (a face cut by the block boundary)
    strip = np.array([[i, i + 1, i + 2] for i in range(8)] + [[9, 0, -1]])
    out["strip10"] = (10, strip)
    return out


@pytest.mark.parametrize("name", list(small_meshes().keys()))
def test_exact_charpoly_eigenvalues(name):
    n, f = small_meshes()[name]
    _, L = comb_L(f, n)
    ev_exact = exact.eigenvalues_exact(L.astype(int).tolist())
    lam = np.linalg.eigvalsh(L)
    assert np.abs(np.array(ev_exact) - lam).max() < 1e-10


@pytest.mark.parametrize("name", ["octahedron", "grid3x3", "fan9"])
def test_matrix_tree_theorem(name):
    n, f = small_meshes()[name]
    e, L = comb_L(f, n)
    tau = exact.spanning_trees_bruteforce(n, e.tolist())
    lam = np.linalg.eigvalsh(L)
    prod = np.prod(lam[1:]) / n
    assert abs(prod - tau) < 1e-6 * tau


def test_charpoly_small_known():
    # path on 3 vertices: L = [[1,-1,0],[-1,2,-1],[0,-1,1]], det(xI-L) = x^3 - 4x^2 + 3x
    cp = exact.charpoly([[1, -1, 0], [-1, 2, -1], [0, -1, 1]])
    assert cp == [Fraction(1), Fraction(-4), Fraction(3), Fraction(0)]


# ---------------------------------------------------------------- GFT, Sections 3 and 7

class TestProjection:
    @pytest.fixture(scope="class")
    def setup(self):
        bs = W.grid_single(nx=12, ny=10, c=10, p=15)
        X = bs.coords[0]
        _, L = comb_L(bs.faces[0], X.shape[0])
        lam, U = S.eigh_lowest(L)
        return X, L, lam, U

    def test_full_basis_is_identity(self, setup):
        X, L, lam, U = setup
        assert np.abs(S.encode_decode(U, X) - X).max() < 1e-12

    def test_c1_gives_centroid(self, setup):
        X, L, lam, U = setup
        Xr = S.encode_decode(U[:, :1], X)
        assert np.abs(Xr - X.mean(0)[None, :]).max() < 1e-12

    def test_projector_idempotent_and_pythagoras(self, setup):
        X, L, lam, U = setup
        for c in (3, 17, 60):
            Uc = U[:, :c]
            Xr = S.encode_decode(Uc, X)
            assert np.abs(S.encode_decode(Uc, Xr) - Xr).max() < 1e-12
            E = S.project(Uc, X)
            assert math.isclose((X ** 2).sum(), (E ** 2).sum() + ((X - Xr) ** 2).sum(), rel_tol=1e-12)

    def test_kept_eigenvector_reconstructs_exactly(self):
        n = 40
        _, L = comb_L(path_edges(n), n)
        lam, U = S.eigh_lowest(L)
        i = np.arange(n)
        X = np.stack([np.cos(np.pi * 3 * (i + 0.5) / n), np.cos(np.pi * 5 * (i + 0.5) / n),
                      np.ones(n)], 1)
        assert np.abs(S.encode_decode(U[:, :6], X) - X).max() < 1e-11
        assert np.abs(S.encode_decode(U[:, :5], X)[:, 1]).max() < 1e-11  # k=5 dropped

    def test_principal_angles_known_rotation(self):
        rng = np.random.default_rng(0)
        Q, _ = np.linalg.qr(rng.normal(size=(30, 4)))
        th = np.array([1e-7, 1e-3, 0.2, 1.0])
        # rotate each basis vector towards an orthogonal complement vector by th
        C, _ = np.linalg.qr(rng.normal(size=(30, 4)) - Q @ (Q.T @ rng.normal(size=(30, 4))))
        C = C - Q @ (Q.T @ C)
        C, _ = np.linalg.qr(C)
        B = Q * np.cos(th) + C * np.sin(th)
        ang = S.principal_angles(Q, B)
        assert np.allclose(ang, np.sort(th), rtol=1e-6, atol=1e-12)
        assert math.isclose(S.sin_theta_max(Q, B), np.sin(1.0), rel_tol=1e-12)


# ---------------------------------------------------------------- Eq. 16, Eq. 6, choice of c

class TestMetrics:
    def test_nmsve_hand_example(self):
        # 4-cycle square of side 1 (d = 1 on every edge), one vertex moved.
        X = np.array([[0., 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]])
        e = cycle_edges(4)
        G = met.gl_matrix(4, lap.canonical_edges(e, 4), X)
        Xr = X.copy()
        Xr[0, 2] = 0.3
        # GL(v) - GL(v~) is zero except: vertex 0 gets 0.3*... by hand:
        # GL_0 diff = -0.3 (z), neighbours 1 and 3 each + 0.15 (z)
        d1 = 0.3
        d2 = math.sqrt(0.3 ** 2 + 2 * 0.15 ** 2)
        assert math.isclose(met.nmsve(X, Xr, G), (d1 + d2) / 8, rel_tol=1e-12)

    def test_gl_annihilates_constants(self):
        bs = W.grid_single(nx=6, ny=7, c=5, p=8)
        X = bs.coords[0]
        e = lap.canonical_edges(bs.faces[0], X.shape[0])
        G = met.gl_matrix(X.shape[0], e, X)
        assert np.abs(G @ np.ones(X.shape[0])).max() < 1e-14

    def test_prefix_identity_and_monotone_l2(self):
        bs = W.grid_single(nx=10, ny=9, c=5, p=8)
        X = bs.coords[0]
        _, L = comb_L(bs.faces[0], X.shape[0])
        lam, U = S.eigh_lowest(L)
        E = U.T @ X
        curve = met.l2_residual_curve(U, X, 60)
        pref = np.sqrt(np.maximum((X ** 2).sum() - np.cumsum((E ** 2).sum(1))[:60], 0))
        assert np.abs(curve - pref).max() < 1e-10 * np.linalg.norm(X)
        assert np.all(np.diff(curve) <= 1e-12)

    def test_choose_c_rule(self):
        curve = np.array([5.0, 4.0, 2.0, 0.5, 0.4, 0.1])
        lam = np.array([0.0, 1.0, 2.0, 3.0, 3.0001, 5.0, 6.0])
        assert met.choose_c(curve, lam, 1.0, 0.0) == 4
        # 4 -> lambda_5 - lambda_4 tiny relative gap: snap up to 5
        assert met.choose_c(curve, lam, 1.0, 1e-3) == 5
        assert met.choose_c(curve, lam, 1e-3, 1e-3) == 6  # target unreachable: c_max

    def test_doi_residual_eq6(self):
        rng = np.random.default_rng(1)
        U, _ = np.linalg.qr(rng.normal(size=(20, 20)))
        X = rng.normal(size=(20, 3))
        assert np.abs(met.doi_residual(U, X)).max() < 1e-12
        e = met.doi_residual(U[:, :5], X)
        assert np.allclose(e, (X - U[:, :5] @ (U[:, :5].T @ X)).sum(1))


class TestHandWorkedWeights:
    """Distance weights (Eq. 2 and the GL operator of Eq. 16) and the Eq. 6
    residual on meshes small enough to work out by hand, with unequal edge
    lengths, so that 1/d and 1/d^2 (or a sum and a mean) give different
    numbers."""

    # right triangle with legs 1 and 2: edges (0,1) d = 1, (0,2) d = 2, (1,2) d = sqrt 5
    TRI_X = np.array([[0., 0, 0], [1, 0, 0], [0, 2, 0]])
    TRI_F = np.array([[0, 1, 2]])
    # three vertices on a line at x = 0, 1, 3: edges (0,1) d = 1, (1,2) d = 2
    PATH_X = np.array([[0., 0, 0], [1, 0, 0], [3, 0, 0]])
    PATH_E = np.array([[0, 1], [1, 2]])

    def test_right_triangle_inverse_square_weights(self):
        e = lap.canonical_edges(self.TRI_F, 3)
        assert e.tolist() == [[0, 1], [0, 2], [1, 2]]
        w = lap.edge_weights(e, self.TRI_X, lap.INV_SQ_DIST)
        assert np.allclose(w, [1.0, 0.25, 0.2], rtol=0, atol=1e-15)
        L = lap.laplacian_dense(3, e, w)
        want = np.array([[1.25, -1.0, -0.25],
                         [-1.0, 1.2, -0.2],
                         [-0.25, -0.2, 0.45]])
        assert np.abs(L - want).max() < 1e-15

    def test_right_triangle_inverse_distance_weights(self):
        e = lap.canonical_edges(self.TRI_F, 3)
        w = lap.edge_weights(e, self.TRI_X, lap.INV_DIST)
        assert np.allclose(w, [1.0, 0.5, 1.0 / math.sqrt(5.0)], rtol=0, atol=1e-15)

    def test_gl_on_a_path_with_unequal_lengths(self):
        # GL(v_1) = v_1 - (v_0 / 1 + v_2 / 2) / (1 + 1/2); the ends have one neighbour
        G = met.gl_matrix(3, self.PATH_E, self.PATH_X)
        want = np.array([[1.0, -1.0, 0.0],
                         [-2.0 / 3.0, 1.0, -1.0 / 3.0],
                         [0.0, -1.0, 1.0]])
        assert np.abs(G - want).max() < 1e-15
        Y = np.array([[2.0, -1.0, 0.5], [4.0, 3.0, -2.0], [-6.0, 9.0, 1.0]])
        assert np.abs(met.gl_apply(3, self.PATH_E, self.PATH_X, Y) - want @ Y).max() < 1e-14
        # middle row by hand for the first column: 4 - (2 + (-6)/2) / 1.5
        assert math.isclose(met.gl_apply(3, self.PATH_E, self.PATH_X, Y)[1, 0],
                            4.0 - (2.0 - 3.0) / 1.5, rel_tol=1e-15)

    def test_nmsve_on_a_path_with_unequal_lengths(self):
        # move end vertex 0 by 0.6 along y: the l2 term is 0.6; G times the
        # difference is (0.6, -0.4, 0) along y (row 1 weighs vertex 0 by 2/3)
        Xr = self.PATH_X.copy()
        Xr[0, 1] += 0.6
        want = (0.6 + math.sqrt(0.36 + 0.16)) / (2 * 3)
        G = met.gl_matrix(3, self.PATH_E, self.PATH_X)
        assert math.isclose(met.nmsve(self.PATH_X, Xr, G), want, rel_tol=1e-14)
        assert math.isclose(met.nmsve_mesh(3, self.PATH_E, self.PATH_X, Xr), want, rel_tol=1e-14)

    def test_sparse_nmsve_curve(self):
        # the edge-by-edge GL of the large-block curve against the dense GL
        # matrix (both pinned above by hand) on a grid with noisy heights,
        # a random orthonormal basis; zero at the full basis
        bs = W.grid_single(nx=7, ny=6, c=5, p=8)
        X = bs.coords[0]
        n = X.shape[0]
        e = lap.canonical_edges(bs.faces[0], n)
        Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(n, n)))
        G = met.gl_matrix(n, e, X)
        dense = np.array([met.nmsve(X, Q[:, :c] @ (Q[:, :c].T @ X), G) for c in range(1, n + 1)])
        sparse = met.nmsve_curve_sparse(Q, X, e, X, n)
        assert np.abs(sparse - dense).max() <= 1e-13 * dense.max()
        assert sparse[-1] < 1e-14
        # c = 1 with the constant vector: every coordinate replaced by its mean
        U1 = np.full((n, 1), 1.0 / math.sqrt(n))
        Xm = np.broadcast_to(X.mean(0), X.shape)
        assert math.isclose(met.nmsve_curve_sparse(U1, X, e, X, 1)[0], met.nmsve(X, Xm, G),
                            rel_tol=1e-12)

    def test_eq6_residual_by_hand(self):
        # U = the constant unit vector (c = 1): v_j - U U^T v_j removes each
        # coordinate's mean; Eq. 6 sums the three residual vectors
        U = np.full((3, 1), 1.0 / math.sqrt(3.0))
        X = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
        e = met.doi_residual(U, X)
        assert np.abs(e - np.array([-28.0 / 3.0, -1.0 / 3.0, 29.0 / 3.0])).max() < 1e-14


class TestSubsetEigensolver:
    """The subset driver that the block references use for large blocks
    (k lowest pairs) against the closed form of the path graph, whose
    spectrum is simple: lambda_k = 2 - 2 cos(k pi / n), u_k(i) ~ cos(k pi (i + 1/2) / n)."""

    @pytest.mark.parametrize("n,k", [(40, 7), (64, 33)])
    def test_lowest_pairs_of_a_path(self, n, k):
        e = path_edges(n)
        L = lap.laplacian_dense(n, lap.canonical_edges(e, n), np.ones(n - 1))
        lam, U = S.eigh_lowest(L, k)
        assert lam.shape == (k,) and U.shape == (n, k)
        j = np.arange(k)
        assert np.abs(lam - (2.0 - 2.0 * np.cos(j * np.pi / n))).max() < 1e-13
        i = np.arange(n)[:, None]
        Uc = np.cos(j[None, :] * np.pi * (i + 0.5) / n)
        Uc /= np.linalg.norm(Uc, axis=0)
        # simple spectrum: each column equals the closed form up to sign
        assert np.abs(np.abs(np.sum(U * Uc, axis=0)) - 1.0).max() < 1e-12

    def test_subset_equals_full_solve_on_a_mesh(self):
        bs = W.grid_single(nx=9, ny=8, c=5, p=8)
        X = bs.coords[0]
        _, L = comb_L(bs.faces[0], X.shape[0])
        lam_f, U_f = np.linalg.eigh(L)
        lam_s, U_s = S.eigh_lowest(L, 20)
        assert np.abs(lam_s - lam_f[:20]).max() < 1e-12
        # compare at a cut with a clear gap
        c = next(c for c in range(12, 20) if lam_f[c] - lam_f[c - 1] > 1e-3)
        assert S.sin_theta_max(U_f[:, :c], U_s[:, :c]) < 1e-10


def test_golden_grid32_fixture():
    """tests/golden/grid32_combinatorial.txt (written by make_golden.py from the
    oracle): the 32 x 32 single-submesh workload's sizes, lowest 76 eigenvalues
    (the tracked width p = 75 plus one), NMSVE and l2 residual at c = 50.  A
    regression pin of the oracle and the input generator; the GPU FP64 test
    compares its Ritz values with the same file."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "grid32_combinatorial.txt")
    rec = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        rec[k] = [float(x) for x in v]
    bs = W.grid_single()
    X = bs.coords[0]
    n = X.shape[0]
    e = lap.canonical_edges(bs.faces[0], n)
    assert (n, e.shape[0], n + 2 * e.shape[0]) == (rec["n"][0], rec["edges"][0], rec["nnz"][0])
    _, L = comb_L(bs.faces[0], n)
    lam, U = S.eigh_lowest(L)
    assert np.abs(lam[:76] - np.array(rec["lambda_1_to_76"])).max() < 1e-12
    Xr = S.encode_decode(U[:, :50], X)
    G = met.gl_matrix(n, e, X)
    assert math.isclose(met.nmsve(X, Xr, G), rec["nmsve_c50"][0], rel_tol=1e-10)
    assert math.isclose(float(np.linalg.norm(X - Xr)), rec["l2_residual_c50"][0], rel_tol=1e-10)


# ---------------------------------------------------------------- Alg. 1, Section 4 rate

class TestIterations:
    def test_paper_oi_converges_at_rate_of_R(self):
        bs = W.grid_single(nx=14, ny=12, c=6, p=6)
        X = bs.coords[0]
        n = X.shape[0]
        _, L = comb_L(bs.faces[0], n)
        lam, U = S.eigh_lowest(L)
        c, delta, z = 6, 1e-2, 1
        U0 = M.random_orthonormal(n, c, M.rng_for(77))
        hist = []
        it.paper_oi(L, U0, z, delta, 60, history=hist)
        ang = np.array([S.sin_theta_max(U[:, :c], H) for H in hist])
        # eigenvalues of R = (L + delta)^-1: the rate is mu_{c+1}/mu_c
        rate = ((lam[c - 1] + delta) / (lam[c] + delta)) ** z
        k0, k1 = 20, 40
        measured = (ang[k1] / ang[k0]) ** (1.0 / (k1 - k0))
        assert abs(measured - rate) < 0.02
        assert ang[-1] < ang[0]

    def test_paper_oi_z_power_reaches_svd_subspace(self):
        bs = W.grid_single(nx=10, ny=10, c=8, p=8)
        n = 100
        _, L = comb_L(bs.faces[0], n)
        lam, U = S.eigh_lowest(L)
        # c = 5 sits at a clear gap (lambda_5 = 0.513, lambda_6 = 0.671)
        U0 = M.random_orthonormal(n, 5, M.rng_for(78))
        Uz = it.paper_oi(L, U0, 5, 1e-3, 40)
        assert S.sin_theta_max(U[:, :5], Uz) < 1e-8

    def test_chebyshev_apply_closed_form(self):
        # T_m(t(L)) V = U T_m(t(Lambda)) U^T V with T_m from its trigonometric /
        # hyperbolic closed form
        bs = W.grid_single(nx=8, ny=9, c=5, p=8)
        n = 72
        _, L = comb_L(bs.faces[0], n)
        lam, U = np.linalg.eigh(L)
        a, b, m = 2.0, 9.0, 7
        t = (2 * lam - a - b) / (b - a)
        Tm = np.where(np.abs(t) <= 1, np.cos(m * np.arccos(np.clip(t, -1, 1))),
                      np.sign(t) ** m * np.cosh(m * np.arccosh(np.maximum(np.abs(t), 1))))
        V = np.random.default_rng(2).normal(size=(n, 4))
        ref = U @ (Tm[:, None] * (U.T @ V))
        got = it.chebyshev_apply(L, V, a, b, m)
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()

    def test_chebyshev_span_converges_to_eigenspace(self):
        bs = W.grid_single(nx=12, ny=12, c=10, p=15)
        n = 144
        _, L = comb_L(bs.faces[0], n)
        lam, U = np.linalg.eigh(L)
        V0 = M.random_orthonormal(n, 15, M.rng_for(79))
        Vs = it.chebyshev_span(L, V0, lam[15], lam[-1] + 0.1, 8, 12)
        th, Vr = it.rayleigh_ritz(L, Vs)
        assert S.sin_theta_max(U[:, :10], Vr[:, :10]) < 1e-9
        assert np.abs(th[:10] - lam[:10]).max() < 1e-10

    def test_doi_grows_and_shrinks(self):
        bs = W.grid_single(nx=10, ny=10, c=4, p=4)
        X = bs.coords[0]
        _, L = comb_L(bs.faces[0], 100)
        lam, U = np.linalg.eigh(L)
        U0 = U[:, :4]
        # a band that needs more columns than 4
        target = np.linalg.norm(met.doi_residual(U[:, :12], X))
        eps_l, eps_h = 0.5 * target, 1.01 * target
        Ud, c, traj = it.paper_doi(L, U0, X, 2, 1e-3, eps_l, eps_h, 40)
        assert c > 4
        # Alg. 2 stops once the Eq. 6 residual of its own basis is inside the band
        ne = np.linalg.norm(met.doi_residual(Ud, X))
        assert eps_l <= ne <= eps_h
        assert np.abs(Ud.T @ Ud - np.eye(c)).max() < 1e-12
        # a band below the current error floor shrinks c
        _, c2, _ = it.paper_doi(L, U[:, :30], X, 2, 1e-3, 1e9, 2e9, 40)
        assert c2 < 30

    def _doi_case(self):
        bs = W.grid_single(nx=9, ny=8, c=4, p=4)
        X = bs.coords[0]
        _, L = comb_L(bs.faces[0], 72)
        lam, U = np.linalg.eigh(L)
        return X, L, lam, U

    def test_doi_chebyshev_first_decision_closed_form(self):
        # an eigenvector start is invariant under the filter: the first
        # residual is that of the exact eigenvectors (eigh, no filter code),
        # the same for the paper's operator; inside the band the walk stops
        X, L, lam, U = self._doi_case()
        r6 = float(np.linalg.norm((X - U[:, :6] @ (U[:, :6].T @ X)).sum(1)))
        Ud, c, traj = it.doi_chebyshev(L, U[:, :6], X, 0.5, 8.5, 6, 2, 0.9 * r6, 1.1 * r6, 20, 30)
        assert c == 6 and len(traj) == 1 and traj[0][0] == 6
        assert math.isclose(traj[0][1], r6, rel_tol=1e-9)
        assert S.sin_theta_max(U[:, :6], Ud) < 1e-10
        _, _, tp = it.paper_doi(L, U[:, :6], X, 2, 1e-3, 0.9 * r6, 1.1 * r6, 20, 30)
        assert math.isclose(tp[0][1], r6, rel_tol=1e-9)

    def test_doi_chebyshev_walks_to_the_limits(self):
        X, L, lam, U = self._doi_case()
        # always above the band: one column per iteration up to c_max, then stop
        Ud, c, traj = it.doi_chebyshev(L, U[:, :3], X, 0.5, 8.5, 6, 2, 0.0, 0.0, 9, 30)
        assert [t[0] for t in traj] == list(range(3, 10)) and c == 9
        assert np.abs(Ud.T @ Ud - np.eye(9)).max() < 1e-12
        # one iteration that grows: the new column is the normalised Eq. 6
        # residual of the filtered basis, orthogonal to it (Eq. 7)
        U1, c, traj = it.doi_chebyshev(L, U[:, :3], X, 0.5, 8.5, 6, 2, 0.0, 0.0, 9, 1)
        e = (X - U1[:, :3] @ (U1[:, :3].T @ X)).sum(1)
        assert c == 4 and np.allclose(U1[:, 3], e / np.linalg.norm(e), atol=1e-14)
        assert np.abs(U1[:, :3].T @ U1[:, 3]).max() < 1e-12
        # always below the band: one column fewer per iteration down to 1
        _, c, traj = it.doi_chebyshev(L, U[:, :5], X, 0.5, 8.5, 6, 2, 1e9, 2e9, 9, 30)
        assert [t[0] for t in traj] == [5, 4, 3, 2, 1] and c == 1
        # no iteration: the start comes back
        Ud, c, traj = it.doi_chebyshev(L, U[:, :5], X, 0.5, 8.5, 6, 2, 0.0, 1.0, 9, 0)
        assert c == 5 and traj == [] and np.array_equal(Ud, U[:, :5])

    def test_doi_chebyshev_stops_inside_the_band(self):
        X, L, lam, U = self._doi_case()
        target = float(np.linalg.norm(met.doi_residual(U[:, :14], X)))
        Ud, c, traj = it.doi_chebyshev(L, U[:, :4], X, 1.0, 8.5, 8, 2, 0.5 * target,
                                       1.01 * target, 40, 60)
        assert c > 4 and traj[-1][0] == c
        ne = float(np.linalg.norm(met.doi_residual(Ud, X)))
        assert 0.5 * target <= ne <= 1.01 * target and math.isclose(ne, traj[-1][1], rel_tol=1e-12)
        assert np.abs(Ud.T @ Ud - np.eye(c)).max() < 1e-12


# ---------------------------------------------------------------- Section 4, iteration count

class TestRitzResiduals:
    def test_exact_pairs_have_zero_residual(self):
        bs = W.grid_single(nx=9, ny=8, c=6, p=8)
        _, L = comb_L(bs.faces[0], 72)
        lam, U = np.linalg.eigh(L)
        r = it.ritz_residuals(L, U[:, :8], lam[:8])
        assert r.max() < 1e-12 * lam[-1]

    def test_two_vector_mix_closed_form(self):
        # v = cos(phi) u_i + sin(phi) u_k: theta = cos^2 lam_i + sin^2 lam_k and
        # L v - theta v = sin(phi) cos(phi) (lam_i - lam_k) (sin(phi) u_i - cos(phi) u_k),
        # so r = |sin(phi) cos(phi)| |lam_k - lam_i|
        _, L = comb_L(M.icosahedron()[1], 12)
        lam, U = np.linalg.eigh(L)
        i, k = 1, 9
        assert abs(lam[k] - lam[i]) > 1.0
        for phi in (0.0, 0.1, 0.7, 1.3):
            v = np.cos(phi) * U[:, i] + np.sin(phi) * U[:, k]
            th = np.cos(phi) ** 2 * lam[i] + np.sin(phi) ** 2 * lam[k]
            r = it.ritz_residuals(L, v[:, None], np.array([th]))[0]
            assert abs(r - abs(np.sin(phi) * np.cos(phi)) * abs(lam[k] - lam[i])) < 1e-12

    def test_residual_bounds_distance_to_spectrum(self):
        # symmetric L, unit v: some eigenvalue lies within r of the Rayleigh quotient
        bs = W.grid_single(nx=10, ny=10, c=6, p=10)
        _, L = comb_L(bs.faces[0], 100)
        lam = np.linalg.eigvalsh(L)
        V0 = M.random_orthonormal(100, 10, M.rng_for(5))
        Vs = it.chebyshev_span(L, V0, 1.5, lam[-1] + 0.1, 3, 1)
        th, Vr = it.rayleigh_ritz(L, Vs)
        r = it.ritz_residuals(L, Vr, th)
        assert r.max() > 1e-3  # not converged: the bound is not trivially met
        for j in range(10):
            assert np.abs(lam - th[j]).min() <= r[j] * (1 + 1e-12)


# ---------------------------------------------------------------- gradient of encode/decode

class TestAdjointOracle:
    """The FP64 autograd gradient of the unrolled encode/decode against
    central finite differences, its special cases, and its converged limit."""

    @pytest.fixture(scope="class")
    def case(self):
        from oracle import adjoint as adj
        bs = W.grid_single(nx=6, ny=5, c=4, p=8)
        n = 30
        e = lap.canonical_edges(bs.faces[0], n)
        X = bs.coords[0].astype(np.float64)
        rng = M.rng_for(71)
        V0 = M.random_orthonormal(n, 8, rng)
        G = rng.normal(size=(n, 3))
        uw = rng.uniform(0.5, 2.0, e.shape[0])
        return adj, n, e, X, V0, G, uw

    def _loss(self, adj, n, e, X, mode, V0, G, uw, N, m=3, c=4, b=12.0):
        import torch
        with torch.no_grad():
            Xr = adj.encdec(n, torch.from_numpy(e), torch.from_numpy(X), mode,
                            torch.from_numpy(V0), 0.9, b, m, N, c,
                            torch.from_numpy(uw) if uw is not None else None)
        return float((Xr.numpy() * G).sum())

    def test_user_weights_match_central_differences(self, case):
        adj, n, e, X, V0, G, uw = case
        gX, gw = adj.unrolled_grad(n, e, X, adj.USER, V0, 0.9, 12.0, 3, 3, 4, G, uw)
        h = 1e-6
        for k in (0, 7, 20, e.shape[0] - 1):
            wp, wm = uw.copy(), uw.copy()
            wp[k] += h
            wm[k] -= h
            fd = (self._loss(adj, n, e, X, adj.USER, V0, G, wp, 3)
                  - self._loss(adj, n, e, X, adj.USER, V0, G, wm, 3)) / (2 * h)
            assert abs(fd - gw[k]) <= 1e-6 * max(1.0, abs(gw).max()), (k, fd, gw[k])
        # projection path of X at fixed L
        for (i, d) in ((0, 0), (13, 2), (29, 1)):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, d] += h
            Xm[i, d] -= h
            fd = (self._loss(adj, n, e, Xp, adj.USER, V0, G, uw, 3)
                  - self._loss(adj, n, e, Xm, adj.USER, V0, G, uw, 3)) / (2 * h)
            assert abs(fd - gX[i, d]) <= 1e-6 * max(1.0, abs(gX).max())

    def test_distance_weights_chain_into_coordinates(self, case):
        adj, n, e, X, V0, G, _ = case
        Xz = X.copy()
        Xz[:, 2] += 0.05 * np.sin(3 * X[:, 0])  # non-flat so every direction matters
        gX, _ = adj.unrolled_grad(n, e, Xz, adj.INV_SQ_DIST, V0, 0.9, 40.0, 3, 3, 4, G)
        h = 1e-6
        for (i, d) in ((1, 0), (14, 1), (22, 2)):
            Xp, Xm = Xz.copy(), Xz.copy()
            Xp[i, d] += h
            Xm[i, d] -= h
            fd = (self._loss(adj, n, e, Xp, adj.INV_SQ_DIST, V0, G, None, 3, b=40.0)
                  - self._loss(adj, n, e, Xm, adj.INV_SQ_DIST, V0, G, None, 3, b=40.0)) / (2 * h)
            assert abs(fd - gX[i, d]) <= 1e-5 * max(1.0, abs(gX).max()), (i, d, fd, gX[i, d])

    def test_combinatorial_gradient_is_the_projector(self, case):
        # L does not depend on X: d loss/dX = U_c U_c^T Gbar with U_c the forward's basis
        import torch
        adj, n, e, X, V0, G, _ = case
        gX, _ = adj.unrolled_grad(n, e, X, adj.COMBINATORIAL, V0, 0.9, 12.0, 3, 3, 4, G)
        with torch.no_grad():
            P = adj.encdec(n, torch.from_numpy(e), torch.eye(n, dtype=torch.float64),
                           adj.COMBINATORIAL, torch.from_numpy(V0), 0.9, 12.0, 3, 3, 4).numpy()
        assert np.abs(P - P.T).max() < 1e-12 and np.abs(P @ P - P).max() < 1e-12
        assert abs(np.trace(P) - 4) < 1e-12
        assert np.abs(gX - P @ G).max() < 1e-12

    def test_eigenprojector_formula_matches_central_differences(self, case):
        adj, n, e, X, _, G, uw = case
        L = lap.laplacian_dense(n, e, uw)
        _, gw = adj.eigenprojector_grad(L, e, X, G, 4)

        def f(w):
            lam, U = np.linalg.eigh(lap.laplacian_dense(n, e, w))
            return float((U[:, :4] @ (U[:, :4].T @ X) * G).sum())

        h = 1e-6
        for k in (2, 11, 30):
            wp, wm = uw.copy(), uw.copy()
            wp[k] += h
            wm[k] -= h
            fd = (f(wp) - f(wm)) / (2 * h)
            assert abs(fd - gw[k]) <= 1e-6 * max(1.0, abs(gw).max()), (k, fd, gw[k])

    def test_unrolled_gradient_tends_to_the_converged_limit(self, case):
        adj, n, e, X, V0, G, uw = case
        L = lap.laplacian_dense(n, e, uw)
        lam = np.linalg.eigvalsh(L)
        gXl, gwl = adj.eigenprojector_grad(L, e, X, G, 4)
        errs = []
        for N in (2, 8, 40):
            gX, gw = adj.unrolled_grad(n, e, X, adj.USER, V0, lam[8] + 0.05, lam[-1] + 0.1, 4, N,
                                       4, G, uw)
            errs.append(np.abs(gw - gwl).max() / np.abs(gwl).max())
        assert errs[-1] < 1e-8 and errs[0] > errs[-1], errs


    def test_tracked_map_reduces_to_the_fixed_interval(self, case):
        # one pass per iteration, a given b and no adaptation: the same map as
        # the fixed-interval unrolled iteration
        adj, n, e, X, V0, G, uw = case
        gX0, gw0 = adj.unrolled_grad(n, e, X, adj.USER, V0, 0.9, 12.0, 3, 3, 4, G, uw)
        gX, gw, info = adj.tracked_grad(n, e, X, adj.USER, V0, 4, G, T=3, m=3, passes=1, a0=0.9,
                                        b=12.0, user_w=uw)
        assert info["a"] == [0.9, 0.9, 0.9] and info["b"] == 12.0
        assert np.abs(gw - gw0).max() < 1e-12 * np.abs(gw0).max()
        assert np.abs(gX - gX0).max() < 1e-12 * np.abs(gX0).max()

    def test_tracked_gradient_matches_differences_at_the_frozen_interval(self, case):
        # adaptive a and Gershgorin b recorded at the point, then held fixed
        adj, n, e, X, V0, G, uw = case
        kw = dict(T=3, m=3, passes=2, a0=lambda b: 1.0 * b * 8 / n, adapt=True, orth_start=True)
        gX, gw, info = adj.tracked_grad(n, e, X, adj.USER, V0, 4, G, user_w=uw, **kw)
        assert len(info["a"]) == 3 and len(set(info["a"])) == 3  # the bound moved
        sched = (info["b"], info["a"])

        def f(w):
            return adj.tracked_grad(n, e, X, adj.USER, V0, 4, G, user_w=w, schedule=sched,
                                    **kw)[2]["loss"]

        h = 1e-6
        for k in (1, 9, e.shape[0] - 2):
            wp, wm = uw.copy(), uw.copy()
            wp[k] += h
            wm[k] -= h
            fd = (f(wp) - f(wm)) / (2 * h)
            assert abs(fd - gw[k]) <= 1e-6 * max(1.0, abs(gw).max()), (k, fd, gw[k])

    def test_gershgorin_bound_and_adaptive_bound_on_a_path(self):
        # path P_n: rows of L sum in absolute value to 2 (ends) and 4 (inside);
        # eigenpairs lam_k = 2 - 2 cos(k pi / n), u_k(i) ~ cos(k pi (i + 1/2) / n).
        # Started on the exact lowest p eigenvectors the filter keeps them, so
        # the largest Rayleigh quotient of the basis is lam_{p-1}.
        import torch
        from oracle import adjoint as adj
        n, p = 12, 4
        e = np.array([[i, i + 1] for i in range(n - 1)])
        L = adj.laplacian(n, torch.from_numpy(e), torch.ones(n - 1, dtype=torch.float64))
        assert adj.gershgorin(L) == 4.0
        i = np.arange(n) + 0.5
        U = np.stack([np.cos(k * np.pi * i / n) for k in range(p)], axis=1)
        U /= np.linalg.norm(U, axis=0)
        lam = 2 - 2 * np.cos(np.arange(p) * np.pi / n)
        X = np.stack([np.arange(n), np.zeros(n), np.zeros(n)], axis=1).astype(float)
        _, _, info = adj.tracked_grad(n, e, X, adj.COMBINATORIAL, U, 2, np.ones((n, 3)), T=3,
                                      m=3, passes=1, a0=0.5, adapt=True)
        assert info["b"] == 4.0 and info["a"][0] == 0.5
        assert abs(info["a"][1] - lam[p - 1]) < 1e-12 and abs(info["a"][2] - lam[p - 1]) < 1e-12
        assert np.abs(info["theta"] - lam).max() < 1e-12

    def test_warm_start_layout(self):
        from oracle import adjoint as adj
        Vp = np.arange(8, dtype=float).reshape(4, 2) + 1.0
        S0 = adj.warm_start(Vp, 5, 3)
        # rows 0..3 and columns 0..1 copied, row 4 zero there, column 2 is
        # the unit vector at (997 * 2) mod 5 = 4
        want = np.array([[1, 2, 0], [3, 4, 0], [5, 6, 0], [7, 8, 0], [0, 0, 1]], float)
        assert np.array_equal(S0, want)
        assert np.array_equal(adj.warm_start(Vp, 3, 1), Vp[:3, :1])


# ---------------------------------------------------------------- Section 6.1, Alg. 3

class TestOverlappedMerge:
    """Weighted average of a vertex's reconstructions in the overlapped
    submeshes that hold it, weighted by its degree in each (Alg. 3)."""

    def test_degrees_are_neighbour_counts(self):
        # brute force: neighbour sets from the faces, kept inside the block
        bs = W.icosphere_overlapped(level=3, n_blocks=6, c=4, p=8)
        fg = bs.extra["faces_global"]
        nbr = [set() for _ in range(bs.n_global)]
        for f in fg:
            for a in range(3):
                for b in range(3):
                    if a != b:
                        nbr[f[a]].add(int(f[b]))
        for gid, faces in zip(bs.global_ids, bs.faces):
            inblk = set(int(g) for g in gid)
            deg = mg.submesh_degrees(faces, len(gid))
            for k, g in enumerate(gid):
                assert deg[k] == len(nbr[g] & inblk)

    def test_single_submesh_is_identity(self):
        v, f = M.icosphere(2)
        X = M.rng_for(61).normal(size=v.shape).astype(np.float32)
        deg = mg.submesh_degrees(f, v.shape[0])
        out = mg.weighted_average(v.shape[0], [np.arange(v.shape[0])], [deg], [X])
        assert np.array_equal(out, X)
        assert (deg == np.bincount(f.ravel(), minlength=v.shape[0])).all()  # closed surface: degree = faces per vertex

    def test_disjoint_parts_are_identity(self):
        bs = W.icosphere_blocks(level=3, n_blocks=5, c=4, p=8)
        rng = M.rng_for(62)
        Xb = [rng.normal(size=(len(g), 3)).astype(np.float32) for g in bs.global_ids]
        deg = [mg.submesh_degrees(f, len(g)) for g, f in zip(bs.global_ids, bs.faces)]
        out = mg.weighted_average(bs.n_global, bs.global_ids, deg, Xb)
        ref = np.zeros((bs.n_global, 3), np.float32)
        for g, x in zip(bs.global_ids, Xb):
            ref[g] = x
        assert np.array_equal(out, ref)

    def test_weighted_centroid_balances(self):
        # the paper's example point lies in three submeshes with degrees 4, 5
        # and 6 (Section 6.1, the figure on degree weights): the merged point
        # r satisfies sum_j w_j (r - v_j) = 0, and it moves toward the
        # reconstruction with the largest degree
        pts = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [0.0, 6.0, 1.5]], np.float32)
        gid = [np.array([0]), np.array([0]), np.array([0])]
        deg = [np.array([4]), np.array([5]), np.array([6])]
        r = mg.weighted_average(1, gid, deg, [pts[0:1], pts[1:2], pts[2:3]])[0].astype(np.float64)
        bal = 4 * (r - pts[0]) + 5 * (r - pts[1]) + 6 * (r - pts[2])
        assert np.abs(bal).max() < 1e-5
        r_eq = mg.weighted_average(1, gid, [np.array([1])] * 3, [pts[0:1], pts[1:2], pts[2:3]])[0]
        assert np.allclose(r_eq, pts.mean(0), atol=1e-6)
        # two submeshes: the distances to the two reconstructions are in the
        # inverse ratio of the degrees
        r2 = mg.weighted_average(1, gid[:2], [np.array([2]), np.array([6])], [pts[0:1], pts[1:2]])[0]
        da, db = np.linalg.norm(r2 - pts[0]), np.linalg.norm(r2 - pts[1])
        assert abs(da / db - 3.0) < 1e-6

    def test_equal_reconstructions_are_kept(self):
        bs = W.icosphere_overlapped(level=3, n_blocks=6, c=4, p=8)
        Xg = M.rng_for(63).normal(size=(bs.n_global, 3)).astype(np.float32)
        deg = [mg.submesh_degrees(f, len(g)) for g, f in zip(bs.global_ids, bs.faces)]
        out = mg.weighted_average(bs.n_global, bs.global_ids, deg, [Xg[g] for g in bs.global_ids])
        assert np.abs(out - Xg).max() <= 2 * np.finfo(np.float32).eps * np.abs(Xg).max()

    def test_all_zero_degrees_take_the_mean_and_uncovered_vertices_zero(self):
        gid = [np.array([0, 1]), np.array([0])]
        deg = [np.array([0, 0]), np.array([0])]
        X = [np.array([[1, 2, 3], [5, 5, 5]], np.float32), np.array([[3, 4, 5]], np.float32)]
        out = mg.weighted_average(3, gid, deg, X)
        assert np.array_equal(out[0], [2, 3, 4]) and np.array_equal(out[1], [5, 5, 5])
        assert np.array_equal(out[2], [0, 0, 0])


class TestOverlapGenerator:
    """Equal-size overlapped submeshes of Section 6.1 (input generation)."""

    def test_sizes_cores_and_rings(self):
        bs = W.icosphere_overlapped(level=4, n_blocks=10, c=4, p=8, overlap=0.15)
        lab = bs.extra["label"]
        n_d = bs.extra["n_d"]
        sizes = np.bincount(lab)
        assert n_d == int(np.ceil(1.15 * sizes.max()))
        indptr, indices = M.vertex_adjacency(bs.n_global, bs.extra["faces_global"])
        for b, g in enumerate(bs.global_ids):
            assert len(g) == n_d == len(set(g.tolist()))
            core = set(np.nonzero(lab == b)[0].tolist())
            assert core <= set(g.tolist())
            # every added vertex touches the block: the rings grow outwards
            gs = set(g.tolist())
            for v in gs - core:
                assert any(int(u) in gs for u in indices[indptr[v]:indptr[v + 1]])
        cover = np.bincount(np.concatenate(bs.global_ids), minlength=bs.n_global)
        assert cover.min() >= 1 and cover.max() >= 2


# ---------------------------------------------------------------- Section 8 (compression)

class TestQuantiser:
    """Uniform q-bit quantisation of the feature vectors and the bit rate."""

    def test_levels_are_exact_on_a_grid(self):
        # values already on the 2^q levels of their range come back exactly
        q = 3
        E = np.zeros((8, 3), np.float32)
        E[:, 0] = np.arange(8) * 0.25 - 1.0          # step 0.25, lo -1
        E[:, 1] = np.arange(8)[::-1]                  # step 1, reversed
        E[:, 2] = 2.5                                 # constant axis
        codes, lo, step, deq = cd.quantize_block(E, 8, q)
        assert np.array_equal(codes[:, 0], np.arange(8)) and np.array_equal(codes[:, 1], np.arange(8)[::-1])
        assert (codes[:, 2] == 0).all() and step[2] == 0 and lo[2] == 2.5
        assert np.array_equal(deq, E)

    def test_error_bound_and_extremes(self):
        rng = M.rng_for(81)
        E = rng.normal(scale=3.0, size=(150, 3)).astype(np.float32)
        for q in (4, 8, 12, 16):
            codes, lo, step, deq = cd.quantize_block(E, 100, q)
            assert codes.max() <= (1 << q) - 1
            err = np.abs(deq.astype(np.float64) - E[:100].astype(np.float64))
            # half a step, plus the FP32 rounding of the level's value
            assert (err <= step.astype(np.float64) / 2 * (1 + 1e-5) + 4 * np.finfo(np.float32).eps * np.abs(E[:100]).max(0)).all()
            for k in range(3):  # the range ends map to the first and last level
                assert codes[np.argmin(E[:100, k]), k] == 0
                assert codes[np.argmax(E[:100, k]), k] == (1 << q) - 1

    def test_rate_counts_bits_per_mesh_vertex(self):
        # the paper's bpv = 3 q_c c k / n_d for k equal blocks of n_d vertices
        assert cd.bits_per_vertex(12, np.full(70, 100), 70 * 512) == 3 * 12 * 100 * 70 / (70 * 512)
        assert cd.bits_per_vertex(12, np.array([0, 0]), 10) == 0.0


class TestMeshQuality:
    """Whole-mesh NMSVE (Eq. 16) and the mean face-normal angle theta
    (Section 8) that the quality report computes."""

    def test_nmsve_mesh_hand_example(self):
        # the 4-cycle square of TestMetrics, through the edge-by-edge operator
        X = np.array([[0., 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]])
        Xr = X.copy()
        Xr[0, 2] = 0.3
        e = lap.canonical_edges(cycle_edges(4), 4)
        d2 = math.sqrt(0.3 ** 2 + 2 * 0.15 ** 2)
        assert math.isclose(met.nmsve_mesh(4, e, X, Xr), (0.3 + d2) / 8, rel_tol=1e-12)

    def test_nmsve_of_a_translation(self):
        # GL removes constants, so a rigid shift t leaves only the l2 term:
        # NMSVE = sqrt(n) |t| / (2 n)
        v, f = M.icosphere(2)
        X = M.displaced_sphere(v, M.rng_for(90), 0.05)
        n = X.shape[0]
        t = np.array([0.3, -0.4, 1.2])
        e = lap.canonical_edges(f, n)
        got = met.nmsve_mesh(n, e, X, X + t)
        assert math.isclose(got, math.sqrt(n) * 1.3 / (2 * n), rel_tol=1e-12)
        assert met.nmsve_mesh(n, e, X, X) == 0.0

    def test_sparse_gl_matches_dense_operator(self):
        bs = W.grid_single(nx=7, ny=6, c=5, p=8)
        X = bs.coords[0]
        n = X.shape[0]
        e = lap.canonical_edges(bs.faces[0], n)
        Y = M.rng_for(91).normal(size=(n, 3))
        assert np.abs(met.gl_apply(n, e, X, Y) - met.gl_matrix(n, e, X) @ Y).max() < 1e-13
        # an isolated vertex keeps its value
        e2 = e[(e != n - 1).all(1)]
        assert np.array_equal(met.gl_apply(n, e2, X, Y)[n - 1], Y[n - 1])

    def test_angle_hand_example(self):
        # normal (0,0,1) against (1,0,0) x (0,1,1) = (0,-1,1): 45 degrees
        f = np.array([[0, 1, 2]])
        X = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0]])
        Xr = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 1]])
        th, used = met.mean_normal_angle(f, X, Xr)
        assert used == 1 and math.isclose(th, 45.0, rel_tol=1e-12)
        # two faces at 45 and 90 degrees average to 67.5
        f2 = np.array([[0, 1, 2], [3, 4, 5]])
        X2 = np.concatenate([X, X + 5])
        Xr2 = np.concatenate([Xr, np.array([[5., 5, 5], [6, 5, 5], [5, 5, 6]])])  # normal (0,-1,0)
        th, used = met.mean_normal_angle(f2, X2, Xr2)
        assert used == 2 and math.isclose(th, 67.5, rel_tol=1e-12)

    def test_angle_of_rotated_and_mirrored_plane(self):
        # every normal of a flat mesh is (0,0,1); a rotation about the x axis
        # by alpha turns each by alpha, a mirror in x flips each
        v, f = M.grid_mesh(9, 8)
        v[:, 2] = 0.0
        a = math.radians(31.0)
        R = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
        th, used = met.mean_normal_angle(f, v, v @ R.T)
        assert used == len(f) and math.isclose(th, 31.0, rel_tol=1e-10)
        th, _ = met.mean_normal_angle(f, v, v * np.array([-1.0, 1.0, 1.0]))
        assert math.isclose(th, 180.0, rel_tol=1e-12)
        th, _ = met.mean_normal_angle(f, v, v)
        assert th == 0.0

    def test_zero_area_faces_are_left_out(self):
        f = np.array([[0, 1, 2], [0, 1, 3]])
        X = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [2, 0, 0]])  # face 1 collinear
        Xr = np.array([[0., 0, 0], [1, 0, 0], [0, 1, 1], [0, 0, 1]])
        th, used = met.mean_normal_angle(f, X, Xr)
        assert used == 1 and math.isclose(th, 45.0, rel_tol=1e-12)
        assert met.mean_normal_angle(f[1:], X, Xr) == (0.0, 0)
