"""Seeded synthetic sparse s.p.d. problems in CSR form.

This module only assembles matrices and draws random vectors.  It contains none of
the solver's arithmetic, so both the serial oracle and the GPU path can be fed
from it.  Every matrix comes back as ``(rowptr int32[n+1], col int32[nnz],
val float64[nnz])`` with columns sorted ascending in every row, the diagonal
present, and values bitwise symmetric (``a_ij`` and ``a_ji`` are the same
double), which is what the setup's matching needs for the weight of an edge to
be identical from both of its ends.

The workloads stand in for the paper's test sets (Section 5: anisotropic
diffusion, linear elasticity and the Parflow Darcy systems), which are not
available; they follow the shapes and value distributions of those problems:
cell-centred finite volumes with log-normal coefficients, Q1 elasticity with a
clamped face, and constant-coefficient Poisson stencils.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "laplace1d", "poisson2d", "poisson3d", "diffusion3d", "elasticity3d",
    "random_spd", "uniform_rhs", "config", "CONFIGS", "default_max_coarse",
]


def _finish(A) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def _tridiag(m: int):
    """1-D Dirichlet second-difference matrix T_m = tridiag(-1, 2, -1)."""
    e = np.ones(m)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplace1d(m: int):
    return _finish(_tridiag(m))


def poisson2d(nx: int, ny: int | None = None):
    """5-point Laplacian, Dirichlet, index k = x + nx*y; diagonal 4, neighbours -1."""
    ny = nx if ny is None else ny
    Ix, Iy = sp.identity(nx, format="csr"), sp.identity(ny, format="csr")
    A = sp.kron(Iy, _tridiag(nx)) + sp.kron(_tridiag(ny), Ix)
    return _finish(A)


def poisson3d(nx: int, ny: int | None = None, nz: int | None = None):
    """7-point Laplacian, Dirichlet, index k = x + nx*y + nx*ny*z; diagonal 6, neighbours -1."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    Ix, Iy, Iz = (sp.identity(k, format="csr") for k in (nx, ny, nz))
    A = (sp.kron(Iz, sp.kron(Iy, _tridiag(nx)))
         + sp.kron(Iz, sp.kron(_tridiag(ny), Ix))
         + sp.kron(_tridiag(nz), sp.kron(Iy, Ix)))
    return _finish(A)


def diffusion3d(nx: int, sigma: float, seed: int, z_scale: float = 1.0,
                ny: int | None = None, nz: int | None = None):
    """Cell-centred finite-volume diffusion on an nx*ny*nz grid of unit cells.

    Cell coefficients kappa = exp(sigma * xi), xi ~ N(0, 1) i.i.d. from ``seed``
    (sigma is the standard deviation of ln kappa).  Interior face
    transmissibility is the harmonic mean 2 ka kb / (ka + kb) times a direction
    scale (``z_scale`` on z faces, 1 on x and y faces).  Every boundary face
    carries a Dirichlet half-cell term 2 kappa_c * scale, so the matrix is s.p.d.
    Off-diagonals are -T, stored with the same double at (i, j) and (j, i).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)
    kap = np.exp(sigma * rng.standard_normal(nz * ny * nx)).reshape(nz, ny, nx)
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    diag = np.zeros((nz, ny, nx))
    rows, cols, vals = [], [], []
    for axis, s in ((2, 1.0), (1, 1.0), (0, z_scale)):
        ka = np.moveaxis(kap, axis, 0)
        T = 2.0 * ka[:-1] * ka[1:] / (ka[:-1] + ka[1:]) * s
        Tb_lo = 2.0 * ka[0] * s
        Tb_hi = 2.0 * ka[-1] * s
        d = np.moveaxis(diag, axis, 0)  # view: writes land in diag
        d[0] += Tb_lo
        d[:-1] += T
        d[1:] += T
        d[-1] += Tb_hi
        ii = np.moveaxis(idx, axis, 0)
        a, b = ii[:-1].ravel(), ii[1:].ravel()
        t = -T.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [t, t]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _finish(A)


def _q1_element_stiffness(E: float, nu: float, h: float) -> np.ndarray:
    """24x24 trilinear hexahedron stiffness of a cube of side h, 2x2x2 Gauss rule.

    Local node a = ax + 2 ay + 4 az (ax, ay, az in {0, 1}), local dof 3 a + component.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3:, 3:] = np.diag([mu, mu, mu])
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    sgn = 2.0 * corners - 1.0  # reference coordinates of the corners in [-1, 1]^3
    g = 1.0 / np.sqrt(3.0)
    K = np.zeros((24, 24))
    for gp in np.array(np.meshgrid([-g, g], [-g, g], [-g, g], indexing="ij")).reshape(3, -1).T:
        # d N_a / d xi_k for N_a = prod_k (1 + s_ak xi_k) / 8
        dN = np.empty((8, 3))
        for k in range(3):
            o = [m for m in range(3) if m != k]
            dN[:, k] = sgn[:, k] * (1 + sgn[:, o[0]] * gp[o[0]]) * (1 + sgn[:, o[1]] * gp[o[1]]) / 8.0
        dN *= 2.0 / h  # d xi / d x
        B = np.zeros((6, 24))
        for a in range(8):
            bx, by, bz = dN[a]
            B[0, 3 * a + 0] = bx
            B[1, 3 * a + 1] = by
            B[2, 3 * a + 2] = bz
            B[3, 3 * a + 1], B[3, 3 * a + 2] = bz, by
            B[4, 3 * a + 0], B[4, 3 * a + 2] = bz, bx
            B[5, 3 * a + 0], B[5, 3 * a + 1] = by, bx
        K += B.T @ D @ B * (h / 2.0) ** 3
    return 0.5 * (K + K.T)


def elasticity3d(ne: int, seed: int, nu: float = 0.3, nu_soft: float = 0.45,
                 frac_soft: float = 0.2, E: float = 1.0):
    """Q1 linear elasticity on the unit cube with ne^3 hexahedra.

    Exactly ``round(frac_soft * ne^3)`` elements (a seeded permutation) get
    Poisson ratio ``nu_soft``; the others ``nu``.  Nodes on the x = 0 face are
    clamped and their dofs eliminated; the remaining dofs are numbered
    3 * (free node, lexicographic x fastest) + component.  Returns
    ``(rowptr, col, val, f)`` where f is the consistent load of the body force
    (0, 0, -1).
    """
    h = 1.0 / ne
    N = ne + 1
    nel = ne ** 3
    rng = np.random.default_rng(seed)
    soft = np.zeros(nel, dtype=bool)
    soft[rng.permutation(nel)[: int(round(frac_soft * nel))]] = True
    K0 = _q1_element_stiffness(E, nu, h)
    K1 = _q1_element_stiffness(E, nu_soft, h)
    ex, ey, ez = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    ex, ey, ez = (a.transpose(2, 1, 0).ravel() for a in (ex, ey, ez))  # element id x fastest
    loc = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)])
    nodes = ((ex[:, None] + loc[None, :, 0]) + N * (ey[:, None] + loc[None, :, 1])
             + N * N * (ez[:, None] + loc[None, :, 2]))  # [nel, 8]
    free = np.ones(N ** 3, dtype=bool)
    free[np.arange(N ** 3) % N == 0] = False  # x = 0 face
    newnode = np.full(N ** 3, -1, dtype=np.int64)
    newnode[free] = np.arange(int(free.sum()))
    nfree = int(free.sum())
    gn = newnode[nodes]  # [nel, 8]
    gd = (3 * gn[:, :, None] + np.arange(3)[None, None, :]).reshape(nel, 24)
    gd[np.repeat(gn < 0, 3, axis=1)] = -1
    Ke = np.where(soft[:, None, None], K1[None], K0[None])  # [nel, 24, 24]
    r = np.broadcast_to(gd[:, :, None], (nel, 24, 24)).ravel()
    c = np.broadcast_to(gd[:, None, :], (nel, 24, 24)).ravel()
    v = Ke.ravel()
    keep = (r >= 0) & (c >= 0)
    n = 3 * nfree
    A = sp.coo_matrix((v[keep], (r[keep], c[keep])), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    # (A + A^T) / 2 on A's own pattern, every structural entry kept -- also the
    # couplings whose element contributions cancel to exactly 0 (scipy's sparse
    # addition would drop them).  a_ij + a_ji is commutative: bitwise symmetric.
    AT = A.T.tocsr()
    AT.sort_indices()
    assert np.array_equal(A.indptr, AT.indptr) and np.array_equal(A.indices, AT.indices)
    A = sp.csr_matrix(((A.data + AT.data) * 0.5, A.indices.copy(), A.indptr.copy()), shape=(n, n))
    f = np.zeros(n)
    zdofs = gd[:, 2::3].ravel()
    zdofs = zdofs[zdofs >= 0]
    np.add.at(f, zdofs, -(h ** 3) / 8.0)
    rp, ci, va = _finish(A)
    return rp, ci, va, f


def random_spd(n: int, density: float, seed: int, equal_weights: bool = False):
    """Random sparse symmetric matrix with negative off-diagonals and a strictly
    dominant diagonal (an s.p.d. M-matrix); a connected path is always included."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="coo")
    r, c = M.row, M.col
    path = np.arange(n - 1)
    r = np.concatenate([r, path])
    c = np.concatenate([c, path + 1])
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    keep = lo != hi
    lo, hi = lo[keep], hi[keep]
    key = np.unique(lo.astype(np.int64) * n + hi)
    lo, hi = key // n, key % n
    if equal_weights:
        v = np.ones(len(lo))
    else:
        v = rng.uniform(0.1, 1.0, len(lo))
    W = sp.coo_matrix((np.concatenate([-v, -v]), (np.concatenate([lo, hi]), np.concatenate([hi, lo]))),
                      shape=(n, n)).tocsr()
    d = -np.asarray(W.sum(axis=1)).ravel() + rng.uniform(0.05, 0.5, n)
    return _finish(W + sp.diags(d))


def uniform_rhs(n: int, seed: int) -> np.ndarray:
    """b ~ U[-1, 1) from numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def grid_sine_vector(nx: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """sin(pi x) sin(pi y) sin(pi z) at the nodes (x = (i+1)/(nx+1), ...) of an
    nx*ny*nz grid in lexicographic order (x fastest): the eigenvector of the
    smallest eigenvalue of the 7-point Dirichlet Laplacian, a user-supplied
    smooth vector for that operator."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    fx = np.sin(np.pi * np.arange(1, nx + 1) / (nx + 1))
    fy = np.sin(np.pi * np.arange(1, ny + 1) / (ny + 1))
    fz = np.sin(np.pi * np.arange(1, nz + 1) / (nz + 1))
    return (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).ravel()


def default_max_coarse(n: int) -> int:
    """The paper's coarsest-size bound maxcoarseset * n^(1/3) with maxcoarseset = 40,
    rounded to the nearest integer (Section 5, experimental settings)."""
    return int(round(40.0 * float(np.cbrt(n))))


def _g1(scale: float = 1.0):
    nx = max(4, int(round(64 * scale)))
    rp, ci, va = poisson2d(nx)
    n = nx * nx
    return dict(name=f"poisson2d_{nx}x{nx}", n=n, rowptr=rp, col=ci, val=va,
                b=uniform_rhs(n, 0), w=np.ones(n), max_coarse=default_max_coarse(n), tol=1e-8)


def _g2(scale: float = 1.0):
    nx = max(4, int(round(100 * scale)))
    rp, ci, va = poisson3d(nx)
    n = nx ** 3
    return dict(name=f"poisson3d_{nx}^3", n=n, rowptr=rp, col=ci, val=va,
                b=uniform_rhs(n, 1), w=np.ones(n), max_coarse=99, tol=1e-8)


def _g3(scale: float = 1.0):
    nx = max(4, int(round(160 * scale)))
    rp, ci, va = diffusion3d(nx, sigma=2.0, seed=2, z_scale=1e-2)
    n = nx ** 3
    return dict(name=f"hetero_diffusion3d_{nx}^3", n=n, rowptr=rp, col=ci, val=va,
                b=uniform_rhs(n, 3), w=np.ones(n), max_coarse=default_max_coarse(n), tol=1e-8)


def _g4(scale: float = 1.0):
    ne = max(2, int(round(48 * scale)))
    rp, ci, va, f = elasticity3d(ne, seed=4)
    n = len(rp) - 1
    return dict(name=f"elasticity3d_q1_{ne}^3", n=n, rowptr=rp, col=ci, val=va,
                b=f, w=np.ones(n), max_coarse=default_max_coarse(n), tol=1e-8)


def _g5(scale: float = 1.0):
    nx = max(4, int(round(128 * scale)))
    rp, ci, va = diffusion3d(nx, sigma=1.0, seed=5)
    n = nx ** 3
    return dict(name=f"diffusion3d_{nx}^3", n=n, rowptr=rp, col=ci, val=va,
                b=uniform_rhs(n, 6), w=np.ones(n), xstar=uniform_rhs(n, 7),
                max_coarse=default_max_coarse(n), tol=1e-10)


CONFIGS = {"G1": _g1, "G2": _g2, "G3": _g3, "G4": _g4, "G5": _g5}


def config(name: str, scale: float = 1.0) -> dict:
    """One of the five workloads, optionally shrunk by ``scale`` along each grid axis.

    G1  2-D Poisson 64^2, b ~ U[-1,1) seed 0, w = 1, coarsest <= 40 n^(1/3)
    G2  3-D Poisson 100^3, b seed 1, coarsest < 100 rows
    G3  3-D heterogeneous FV diffusion 160^3, ln kappa ~ N(0, 2^2) seed 2, z faces x1e-2, b seed 3
    G4  3-D Q1 elasticity 48^3 elements, nu = 0.45 on 20% of elements (seed 4), body force
    G5  3-D FV diffusion 128^3, ln kappa ~ N(0, 1) seed 5, b seed 6, target x* seed 7, tol 1e-10
    """
    return CONFIGS[name](scale)
