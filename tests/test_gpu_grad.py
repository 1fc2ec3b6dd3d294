"""Differentiable solve on the GPU: adjoint solve with the same hierarchy,
sampled outer product dL/dA_ij = -lambda_i x_j on A's pattern, and the
torch.autograd.Function built on them.

References: the oracle (adjoint solve, sampled outer product), numpy dense
solves (dense reference gradient) and central finite differences of the loss
L = 1/2 ||x - x*||^2 along symmetric directions on the pattern.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1810_04221_amd import problems as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1810_04221_amd import bcm
    bcm.load_library()
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 GPU"
    return bcm


@pytest.mark.parametrize("name,scale,group", [("G5", 0.15, 0), ("G4", 0.21, 0), ("G5", 0.15, 4)])
def test_sampled_outer_bitexact(B, ora, name, scale, group):
    # group 4: rows longer than the lane group (a second pass over each row)
    c = P.config(name, scale)
    say(f"sampled outer {c['name']} group={group}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], group=group)
    lam, x = P.uniform_rhs(c["n"], 21), P.uniform_rhs(c["n"], 22)
    G = h.sampled_outer(lam, x).cpu().numpy()
    Go = ora.sampled_outer(c["rowptr"], c["col"], lam, x)
    assert np.array_equal(G.view(np.uint64), Go.view(np.uint64))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_matches_oracle(B, ora, precision):
    c = P.config("G5", 0.15)
    say(f"adjoint {precision} {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], precision=precision)
    x = h.solve(c["b"], tol=1e-12)
    g = x.cpu().numpy() - c["xstar"]
    lam = h.solve_adjoint(g).cpu().numpy()
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    xo, _ = ho.solve(c["b"], tol=1e-12)
    lo, _ = ho.solve(xo - c["xstar"], tol=1e-12)
    assert np.linalg.norm(lam - lo) <= 1e-9 * np.linalg.norm(lo)
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    assert np.linalg.norm(A @ lam - g) <= 1e-12 * np.linalg.norm(g) * 1.01


def _dense_problem(scale=0.08):
    c = P.config("G5", scale)
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    return c, A


@pytest.mark.parametrize("save_x", [True, False])
def test_autograd_matches_dense_reference(B, save_x):
    import torch
    c, A = _dense_problem()
    say(f"autograd dense reference n={c['n']} save_x={save_x}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], adjoint_tol=1e-13)
    val = torch.tensor(c["val"], device="cuda", requires_grad=True)
    b = torch.tensor(c["b"], device="cuda", requires_grad=True)
    xs = torch.tensor(c["xstar"], device="cuda")
    x = B.solve(val, b, h, tol=1e-13, save_x=save_x)
    loss = 0.5 * ((x - xs) ** 2).sum()
    loss.backward()
    D = A.toarray()
    xd = np.linalg.solve(D, c["b"])
    ld = np.linalg.solve(D, xd - c["xstar"])
    rows = np.repeat(np.arange(c["n"]), np.diff(c["rowptr"]))
    Gd = -ld[rows] * xd[c["col"]]
    assert np.linalg.norm(b.grad.cpu().numpy() - ld) <= 1e-9 * np.linalg.norm(ld)
    assert np.linalg.norm(val.grad.cpu().numpy() - Gd) <= 1e-9 * np.linalg.norm(Gd)


def test_autograd_finite_differences(B):
    import torch
    c, A = _dense_problem()
    n = c["n"]
    rng = np.random.default_rng(31)
    say(f"autograd finite differences n={n}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], adjoint_tol=1e-13)
    val = torch.tensor(c["val"], device="cuda", requires_grad=True)
    b = torch.tensor(c["b"], device="cuda", requires_grad=True)
    xs = torch.tensor(c["xstar"], device="cuda")
    x = B.solve(val, b, h, tol=1e-13)
    (0.5 * ((x - xs) ** 2).sum()).backward()
    G = val.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()

    def loss(vals, bb):
        xx = np.linalg.solve(sp.csr_matrix((vals, c["col"], c["rowptr"]), shape=(n, n)).toarray(), bb)
        return 0.5 * np.sum((xx - c["xstar"]) ** 2)

    rows = np.repeat(np.arange(n), np.diff(c["rowptr"]))
    E = sp.csr_matrix((rng.standard_normal(len(c["col"])), c["col"], c["rowptr"]), shape=(n, n))
    E = ((E + E.T) * 0.5).tocsr()
    # relative perturbation of every stored entry, symmetric on the pattern
    e = np.asarray(E[rows, c["col"]]).ravel() * np.abs(c["val"])

    def richardson(f, h):
        # central differences at h and h/2 combined: truncation error O(h^4)
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    fd = richardson(lambda t: loss(c["val"] + t * e, c["b"]), 1e-3)
    assert abs(fd - G @ e) <= 1e-6 * abs(fd)
    d = rng.standard_normal(n)
    fdb = richardson(lambda t: loss(c["val"], c["b"] + t * d), 1e-3)
    assert abs(fdb - gb @ d) <= 1e-6 * abs(fdb)


def test_fp32_cycle_gradient_error(B):
    # FP32 cycle inside FP64 CG: gradients converge to the same FP64 tolerance
    import torch
    c, A = _dense_problem()
    say("fp32 cycle gradient")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], precision="fp32",
                    adjoint_tol=1e-12)
    val = torch.tensor(c["val"], device="cuda", requires_grad=True)
    b = torch.tensor(c["b"], device="cuda", requires_grad=True)
    x = B.solve(val, b, h, tol=1e-12)
    (0.5 * ((x - torch.tensor(c["xstar"], device="cuda")) ** 2).sum()).backward()
    D = A.toarray()
    ld = np.linalg.solve(D, np.linalg.solve(D, c["b"]) - c["xstar"])
    assert np.linalg.norm(b.grad.cpu().numpy() - ld) <= 1e-8 * np.linalg.norm(ld)


def test_autograd_rejects_values_the_hierarchy_was_not_built_from(B):
    # the solve uses the hierarchy's copy of A: values changed after the
    # setup (an optimiser step) must not be silently ignored
    import torch
    c = P.config("G5", 0.1)
    say("autograd stale values")
    val = torch.tensor(c["val"], dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(c["b"], dtype=torch.float64, device="cuda")
    h = B.Hierarchy(c["rowptr"], c["col"], val.detach(), max_coarse=c["max_coarse"])
    x = B.solve(val, b, h, 1e-10)
    x.sum().backward()
    assert val.grad is not None and torch.isfinite(val.grad).all().item()
    with torch.no_grad():
        val.mul_(1.01)
    with pytest.raises(ValueError):
        B.solve(val, b, h, 1e-10)
    h2 = B.Hierarchy(c["rowptr"], c["col"], val.detach(), max_coarse=c["max_coarse"])
    x2 = B.solve(val, b, h2, 1e-10)
    assert torch.allclose(x2 * 1.01, x.detach(), rtol=1e-6, atol=1e-12)
