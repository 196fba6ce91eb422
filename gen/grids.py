"""Seeded sparse finite-element / finite-volume operators on structured grids.

These build the sparse matrices whose nested-dissection separators give the
dense frontal matrices the solver works on (the paper's frontal matrices come
from 3D elliptic problems eliminated with a multifrontal method, Sec. 2.2 and
Sec. 6).  Nothing here touches the HODLR method itself: it is problem set-up,
shared by the oracle and the GPU path as input only.

Cell / node numbering is x-fastest: ``idx = x + nx*(y + ny*z)``; a "plane"
is one fixed z.  Elasticity numbers dofs node-major (ux, uy, uz).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Cell-centred two-point-flux diffusion (7-point stencil)
# ---------------------------------------------------------------------------

def lognormal_coeff(shape, sigma=1.0, seed=0):
    """Cell coefficient kappa = exp(N(0, sigma^2)), drawn x-fastest.

    ``shape`` is (nx, ny, nz); the draw order is the flat cell index.
    """
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(nx * ny * nz)
    return np.exp(sigma * g)


def tpfa_matrix(shape, kappa=None):
    """Sparse SPD two-point-flux matrix on an nx*ny*nz cell grid, unit spacing.

    Interior face between cells a, b: transmissibility 2/(1/k_a + 1/k_b).
    Dirichlet boundary face of cell c: transmissibility k_c.  With k == 1 this
    is the 7-point Laplacian (diagonal 6, off-diagonals -1).
    Returns a CSR matrix with x-fastest cell numbering.
    """
    nx, ny, nz = shape
    N = nx * ny * nz
    k = np.ones(N) if kappa is None else np.asarray(kappa, dtype=np.float64)
    assert k.shape == (N,)
    idx = np.arange(N).reshape(nz, ny, nx)
    kk = k.reshape(nz, ny, nx)
    diag = np.zeros((nz, ny, nx))
    rows, cols, vals = [], [], []
    for axis in range(3):  # axis 0 = z, 1 = y, 2 = x in the (nz, ny, nx) array
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        ka, kb = kk[tuple(lo)], kk[tuple(hi)]
        t = 2.0 / (1.0 / ka + 1.0 / kb)
        diag[tuple(lo)] += t
        diag[tuple(hi)] += t
        a = idx[tuple(lo)].ravel()
        b = idx[tuple(hi)].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t.ravel(), -t.ravel()]
        # Dirichlet faces on both ends of this axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = slice(0, 1)
        last[axis] = slice(-1, None)
        diag[tuple(first)] += kk[tuple(first)]
        diag[tuple(last)] += kk[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A


# ---------------------------------------------------------------------------
# Trilinear (Q1, 8-node) hexahedral linear elasticity
# ---------------------------------------------------------------------------

def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def q1_element_stiffness(E=1.0, nu=0.3, h=1.0):
    """24x24 stiffness of a cube of side h, 2x2x2 Gauss, isotropic material.

    Local node (a, b, c) in {0,1}^3 has index a + 2b + 4c; local dof
    3*node + component.  Strains in Voigt order xx, yy, zz, yz, xz, xy with
    engineering shears.
    """
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    g = 1.0 / np.sqrt(3.0)
    corners = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float)
    sgn = 2.0 * corners - 1.0  # node reference coordinates in {-1, 1}
    Ke = np.zeros((24, 24))
    detJ = (h / 2.0) ** 3
    for gz in (-g, g):
        for gy in (-g, g):
            for gx in (-g, g):
                xi = np.array([gx, gy, gz])
                # dN/dxi for each node
                dN = np.zeros((8, 3))
                for n in range(8):
                    f = (1.0 + sgn[n] * xi) / 2.0
                    dN[n, 0] = sgn[n, 0] / 2.0 * f[1] * f[2]
                    dN[n, 1] = sgn[n, 1] / 2.0 * f[0] * f[2]
                    dN[n, 2] = sgn[n, 2] / 2.0 * f[0] * f[1]
                dNdx = dN * (2.0 / h)
                B = np.zeros((6, 24))
                for n in range(8):
                    bx, by, bz = dNdx[n]
                    c = 3 * n
                    B[0, c] = bx
                    B[1, c + 1] = by
                    B[2, c + 2] = bz
                    B[3, c + 1] = bz
                    B[3, c + 2] = by
                    B[4, c] = bz
                    B[4, c + 2] = bx
                    B[5, c] = by
                    B[5, c + 1] = bx
                Ke += B.T @ D @ B * detJ
    return Ke


def q1_elasticity_matrix(free_shape, E=1.0, nu=0.3):
    """Sparse stiffness of a box of (fx+1)*(fy+1)*(fz+1) unit hexes, clamped on
    all faces; the unknowns are the fx*fy*fz interior nodes (3 dofs each).

    Free node (x, y, z), 0-based, sits at grid point (x+1, y+1, z+1); its
    index is x + fx*(y + fy*z) and its dofs are 3*index + {0,1,2}.
    """
    fx, fy, fz = free_shape
    ex, ey, ez = fx + 1, fy + 1, fz + 1  # elements per axis
    Ke = q1_element_stiffness(E, nu)
    # global grid-point -> free node index (or -1 on the clamped boundary)
    gx, gy, gz = fx + 2, fy + 2, fz + 2
    gmap = -np.ones((gz, gy, gx), dtype=np.int64)
    gmap[1:-1, 1:-1, 1:-1] = np.arange(fx * fy * fz).reshape(fz, fy, fx)
    rows, cols, vals = [], [], []
    ez_i, ey_i, ex_i = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
    ez_i, ey_i, ex_i = ez_i.ravel(), ey_i.ravel(), ex_i.ravel()
    # free node index of each local node of every element
    loc = np.empty((ex_i.size, 8), dtype=np.int64)
    for n in range(8):
        a, b, c = n & 1, (n >> 1) & 1, (n >> 2) & 1
        loc[:, n] = gmap[ez_i + c, ey_i + b, ex_i + a]
    ldof = np.empty((ex_i.size, 24), dtype=np.int64)
    for n in range(8):
        for comp in range(3):
            ldof[:, 3 * n + comp] = np.where(loc[:, n] >= 0, 3 * loc[:, n] + comp, -1)
    for i in range(24):
        for j in range(24):
            if Ke[i, j] == 0.0:
                continue
            m = (ldof[:, i] >= 0) & (ldof[:, j] >= 0)
            rows.append(ldof[m, i])
            cols.append(ldof[m, j])
            vals.append(np.full(int(m.sum()), Ke[i, j]))
    N = 3 * fx * fy * fz
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A
