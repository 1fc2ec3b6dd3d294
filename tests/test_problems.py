"""The seeded input generators: shapes, symmetry and the closed forms they
promise (no method arithmetic here)."""
import numpy as np
import scipy.sparse as sp

from paper_1810_04221_amd import problems as P


def _A(rp, ci, va):
    n = len(rp) - 1
    return sp.csr_matrix((va, ci, rp), shape=(n, n))


def test_grid_sine_vector_is_the_lowest_poisson_mode():
    nx = 9
    A = _A(*P.poisson3d(nx))
    w = P.grid_sine_vector(nx)
    lam = 3 * (2.0 - 2.0 * np.cos(np.pi / (nx + 1)))
    assert np.allclose(A @ w, lam * w, rtol=0, atol=1e-13)
    assert (w > 0).all()
    ev = np.linalg.eigvalsh(A.toarray())
    assert abs(ev[0] - lam) < 1e-12


def test_generators_are_symmetric_and_sorted():
    for name, scale in [("G1", 0.25), ("G2", 0.1), ("G3", 0.1), ("G4", 0.1), ("G5", 0.1)]:
        c = P.config(name, scale)
        A = _A(c["rowptr"], c["col"], c["val"])
        assert (A != A.T).nnz == 0
        for i in range(0, c["n"], max(1, c["n"] // 50)):
            row = c["col"][c["rowptr"][i]:c["rowptr"][i + 1]]
            assert (np.diff(row) > 0).all()
        assert len(c["b"]) == c["n"] and len(c["w"]) == c["n"]


def test_elasticity_keeps_every_structural_entry():
    # Q1 elements couple every pair of nodes within one element of each other
    # (3 x 3 x 3 neighbourhood), 3 x 3 dofs per node pair: with the x = 0 face
    # clamped there are (3 ne - 2) (3 (ne + 1) - 2)^2 free node pairs, and every
    # one of them is stored -- also those whose element contributions cancel
    # to exactly 0 (the full-size 48^3 count is 26,869,950)
    ne = 8
    rp, ci, va, f = P.elasticity3d(ne, seed=4)
    assert len(ci) == 9 * (3 * ne - 2) * (3 * (ne + 1) - 2) ** 2
    assert (va == 0).sum() > 0
    A = _A(rp, ci, va)
    assert np.array_equal(A.T.tocsr().sorted_indices().indices, ci)
    assert 9 * (3 * 48 - 2) * (3 * 49 - 2) ** 2 == 26869950
