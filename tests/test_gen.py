"""Pins of the seeded input generators (frontal matrices of Sec. 2.2 / Sec. 6).

The fronts are Schur complements of sparse grid operators onto a middle
plane.  They are pinned against a closed form (unit Laplacian), against the
brute-force dense Schur complement, and against properties of the
discretisations (Q1 element null space, patch test, SPD).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.special import eval_chebyu

from gen import fronts, grids


def brute_front(A, m, zs):
    A = A.toarray()
    s = np.arange(zs * m, (zs + 1) * m)
    rest = np.setdiff1d(np.arange(A.shape[0]), s)
    Ass = A[np.ix_(s, s)]
    Asi = A[np.ix_(s, rest)]
    Aii = A[np.ix_(rest, rest)]
    return Ass - Asi @ np.linalg.solve(Aii, Asi.T)


def test_laplace_front_closed_form():
    """Unit 7-point Laplacian, 32x32x31 cells, plane z=15: the 2D sine transform
    diagonalises each plane and the per-mode Schur value of a chain of m=15
    planes per side is a - 2 U_{m-1}(a/2) / U_m(a/2) (Chebyshev U)."""
    f = fronts.make_workload("laplace1024")
    K = f.K.numpy()
    n1 = 32
    j = np.arange(1, n1 + 1)
    S = np.sqrt(2.0 / (n1 + 1)) * np.sin(np.outer(j, j) * np.pi / (n1 + 1))
    lam = 2.0 - 2.0 * np.cos(j * np.pi / (n1 + 1))
    a = 2.0 + lam[:, None] + lam[None, :]          # [y-mode, x-mode]
    m = 15
    sig = a - 2.0 * eval_chebyu(m - 1, a / 2.0) / eval_chebyu(m, a / 2.0)
    Q = np.kron(S, S)                               # index y*32 + x
    Kc = Q @ np.diag(sig.ravel()) @ Q.T
    assert np.abs(Kc - K).max() / np.abs(K).max() < 1e-13
    assert f.n == 1024


def test_tpfa_unit_is_7pt():
    A = grids.tpfa_matrix((4, 3, 5))
    d = A.diagonal()
    assert np.all(d == 6.0)
    off = A - sp.diags(d)
    assert set(np.unique(off.data)) <= {-1.0, 0.0}
    assert np.all(np.asarray((A != 0).sum(axis=1)).ravel() <= 7)


@pytest.mark.parametrize("shape,zs", [((5, 4, 7), 3), ((3, 6, 6), 2)])
def test_tpfa_plane_sweep_matches_brute_force(shape, zs):
    kappa = grids.lognormal_coeff(shape, sigma=1.0, seed=3)
    A = grids.tpfa_matrix(shape, kappa)
    m = shape[0] * shape[1]
    f = fronts.tpfa_front(shape, zs=zs, sigma=1.0, seed=3)
    Kb = brute_front(A, m, zs)
    assert np.abs(f.K.numpy() - Kb).max() <= 1e-12 * np.abs(Kb).max()
    # symmetric M-matrix with positive row sums (diagonally dominant)
    K = f.K.numpy()
    assert np.allclose(K, K.T, atol=0)
    off = K - np.diag(np.diag(K))
    assert off.max() <= 1e-14
    assert np.all(K.sum(axis=1) > 0)


def test_q1_element_nullspace_and_patch():
    Ke = grids.q1_element_stiffness(E=1.0, nu=0.3)
    assert np.allclose(Ke, Ke.T, atol=1e-14)
    w = np.linalg.eigvalsh(Ke)
    assert np.all(w > -1e-12)
    assert int(np.sum(np.abs(w) < 1e-10)) == 6  # rigid-body modes
    # patch test: a linear displacement field gives equal and opposite nodal forces
    corners = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float)
    G = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.3], [0.1, 0.2, -0.2]])
    u = (corners @ G.T).ravel()
    f = Ke @ u
    assert abs(f.reshape(8, 3).sum(axis=0)).max() < 1e-12


def test_q1_patch_interior_zero():
    """Globally linear displacement -> zero residual at nodes not touching the
    clamped boundary (assembled operator on a larger box, interior rows)."""
    fx, fy, fz = 5, 5, 5
    A = grids.q1_elasticity_matrix((fx, fy, fz))
    z, y, x = np.meshgrid(np.arange(fz) + 1, np.arange(fy) + 1, np.arange(fx) + 1, indexing="ij")
    X = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(float)
    G = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.3], [0.1, 0.2, -0.2]])
    u = (X @ G.T + np.array([0.1, -0.2, 0.3])).ravel()
    r = (A @ u).reshape(fz, fy, fx, 3)
    inner = r[1:-1, 1:-1, 1:-1]
    assert np.abs(inner).max() < 1e-12


def test_elasticity_front_matches_brute_force_and_spd():
    fs = (3, 3, 5)
    A = grids.q1_elasticity_matrix(fs)
    m = 3 * fs[0] * fs[1]
    f = fronts.elasticity_front(fs, zs=2)
    Kb = brute_front(A, m, 2)
    assert np.abs(f.K.numpy() - Kb).max() <= 1e-12 * np.abs(Kb).max()
    assert np.linalg.eigvalsh(f.K.numpy()).min() > 0


def test_permuted_front_consistent():
    fs = (3, 2, 3)
    f = fronts.elasticity_front(fs, zs=1)
    g = fronts.elasticity_front(fs, zs=1, perm_seed=0)
    perm = np.random.default_rng(0).permutation(f.n)
    assert np.array_equal(g.K.numpy(), f.K.numpy()[np.ix_(perm, perm)])
    assert np.array_equal(g.coords, f.coords[perm])
    Gf = sp.csr_matrix((np.ones(f.indices.size), f.indices, f.indptr), shape=(f.n, f.n)).toarray()
    Gg = sp.csr_matrix((np.ones(g.indices.size), g.indices, g.indptr), shape=(g.n, g.n)).toarray()
    assert np.array_equal(Gg, Gf[np.ix_(perm, perm)])


def test_separator_graph_symmetric():
    f = fronts.tpfa_front((6, 5, 5), zs=2, sigma=1.0, seed=1)
    G = sp.csr_matrix((np.ones(f.indices.size), f.indices, f.indptr), shape=(f.n, f.n))
    assert (G != G.T).nnz == 0
    assert G.diagonal().sum() == 0
    deg = np.diff(f.indptr)
    assert deg.max() == 4 and deg.min() == 2


def test_rhs_deterministic():
    a = fronts.rhs(10, 3, seed=0).numpy()
    b = np.random.default_rng(0).uniform(-1, 1, size=(10, 3))
    assert np.array_equal(a, b)


def test_nd_fronts_are_box_schur_complements():
    """Every nested-dissection front equals the dense Schur complement of its
    box's operator onto its separator (brute force), and the tree has the
    expected separators."""
    import scipy.linalg as sla
    from gen import grids
    N = 6
    fr = fronts.nd_fronts(N, levels=3, sigma=1.0, seed=4)
    assert [f.meta["level"] for f in fr] == [0, 1, 1, 2, 2, 2, 2]
    assert fr[0].n == N * N and fr[1].n == N * (N // 2)
    kap = grids.lognormal_coeff((N, N, N), sigma=1.0, seed=4).reshape(N, N, N)
    for f in fr:
        x0, x1, y0, y1, z0, z1 = f.meta["box"]
        shape = (x1 - x0, y1 - y0, z1 - z0)
        A = grids.tpfa_matrix(shape, kap[z0:z1, y0:y1, x0:x1].ravel()).toarray()
        # separator cells in the box's x-fastest numbering
        c = f.coords.astype(int)
        sep = (c[:, 0] - x0) + shape[0] * ((c[:, 1] - y0) + shape[1] * (c[:, 2] - z0))
        rest = np.setdiff1d(np.arange(A.shape[0]), sep)
        S = A[np.ix_(sep, sep)]
        if rest.size:
            S = S - A[np.ix_(sep, rest)] @ sla.solve(A[np.ix_(rest, rest)], A[np.ix_(rest, sep)])
        np.testing.assert_allclose(f.K.numpy(), S, rtol=1e-10, atol=1e-12)
        # the separator cuts the box in its middle along the level's axis
        ax = {"x": 0, "y": 1, "z": 2}[f.meta["axis"]]
        lo, hi = f.meta["box"][2 * ax], f.meta["box"][2 * ax + 1]
        assert np.all(c[:, ax] == lo + (hi - lo) // 2)


# ---------------------------------------------------------------------------
# unstructured tetrahedral meshes (gen/meshes.py)
# ---------------------------------------------------------------------------
def test_p1_reference_element():
    """The P1 stiffness of the unit right tetrahedron, by hand: |T| = 1/6 and
    the basis gradients (-1,-1,-1), e_x, e_y, e_z."""
    from gen import meshes
    pts = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    A = meshes.p1_laplacian(pts, np.array([[0, 1, 2, 3]])).toarray()
    want = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    assert np.allclose(A, want, atol=1e-15)


def test_p1_constants_and_linear_patch():
    """Rows sum to zero (constants are harmonic) and a linear function is
    discretely harmonic at every vertex off the boundary."""
    from gen import meshes
    pts, tets = meshes.tet_mesh(1500, seed=3)
    A = meshes.p1_laplacian(pts, tets)
    scale = abs(A).max()
    assert np.abs(A @ np.ones(pts.shape[0])).max() <= 1e-12 * scale
    u = pts @ np.array([0.3, -1.2, 0.7]) + 2.0
    inner = np.setdiff1d(np.arange(pts.shape[0]), meshes.hull_vertices(pts))
    assert np.abs((A @ u)[inner]).max() <= 1e-11 * scale


def test_tet_front_is_the_schur_complement_and_spd():
    from gen import meshes
    f = meshes.tet_front(1500, seed=4)
    pts, tets = meshes.tet_mesh(1500, seed=4)
    A = meshes.p1_laplacian(pts, tets)
    free = np.setdiff1d(np.arange(pts.shape[0]), meshes.hull_vertices(pts))
    S = meshes.mid_separator(pts, A, free)
    I = np.setdiff1d(free, S)
    D = A.toarray()
    want = D[np.ix_(S, S)] - D[np.ix_(S, I)] @ np.linalg.solve(D[np.ix_(I, I)], D[np.ix_(I, S)])
    K = f.K.numpy()
    assert np.abs(K - want).max() <= 1e-11 * np.abs(want).max()
    assert np.linalg.eigvalsh(K).min() > 0
    # the separator disconnects the two halves: no edge joins I below to I above
    below = pts[I, 2] < 0.5
    C = A[I][:, I].tocoo()
    assert not np.any((below[C.row] != below[C.col]) & (C.data != 0.0))
    # graph = pattern of A_SS, symmetric, no self loops
    G = sp.csr_matrix((np.ones(f.indices.size), f.indices, f.indptr), shape=(f.n, f.n)).toarray()
    P = (np.abs(D[np.ix_(S, S)]) > 0).astype(float)
    np.fill_diagonal(P, 0)
    assert np.array_equal(G, P) and np.array_equal(G, G.T)
    assert np.allclose(f.coords, pts[S].astype(np.float32))
