"""GPU parity against the serial oracle, through the C ABI.

Bars: matchings, aggregates, prolongators and coarse matrices bit-exact (the
weights are FP64 without FMA contraction; the Galerkin sums run in one fixed
order on both sides); l1 diagonals within (row length) ulp; one FP64 cycle within 1e-12
relative; FP64 solves reach the true residual with the iteration count within
+-1 of the oracle's; the FP32-cycle form reaches the same FP64 residual and its
cycle error against the FP64 oracle is bounded as stated below.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1810_04221_amd import problems as P

pytestmark = pytest.mark.gpu
ULP = np.finfo(np.float64).eps


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1810_04221_amd import bcm
    bcm.load_library()
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 GPU"
    return bcm


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def _close_entries(z, zo, rtol):
    # entry by entry: |z_i - zo_i| <= rtol (|zo_i| + mean |zo|).  The scale
    # mean |zo| stands for the size of the terms a rounding error in entry i
    # is relative to (the cycle mixes neighbouring entries at every level).
    z, zo = np.asarray(z, dtype=np.float64), np.asarray(zo, dtype=np.float64)
    bound = rtol * (np.abs(zo) + np.mean(np.abs(zo)))
    err = np.abs(z - zo)
    worst = int(np.argmax(err / bound))
    say(f"entry-wise: worst |dz| / (|zo| + mean |zo|) = {err[worst] / bound[worst] * rtol:.2e} (bound {rtol:.0e})")
    assert np.all(err <= bound), f"entry {worst}: |dz| = {err[worst]:.3e} > bound {bound[worst]:.3e}"


# Entry-wise bounds of one preconditioner application against the FP64
# oracle, on the scale |zo_i| + mean |zo|.  FP64: the two sides differ only in
# the order of the sums (dense folded operators, sliced-ELL rows, block
# partials), a few ulp per operation carried through the levels; FP32: float32
# storage and accumulation, eps 6e-8 per operation carried the same way.  The
# norm-wise bounds (1e-12 and 1e-5 relative) are checked beside these.
ENTRY_FP64, ENTRY_FP32 = 1e-11, 1e-4


# FP32 cycle: a perturbed preconditioner; the iteration count may differ from
# the FP64 oracle's either way, by at most this much
def _fp32_allowance(it):
    return max(2, it // 20)


def _star(n):
    A = sp.lil_matrix((n, n))
    for j in range(1, n):
        A[0, j] = A[j, 0] = -1.0
    A.setdiag([n + 1.0] + [2.0] * (n - 1))
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def _clique(n):
    A = sp.csr_matrix(-np.ones((n, n)) + (n + 1.0) * np.eye(n))
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


MATCH_CASES = {
    "path9": lambda: (*P.laplace1d(9), None),
    "path4097": lambda: (*P.laplace1d(4097), None),
    "star65": lambda: (*_star(65), None),
    "clique40": lambda: (*_clique(40), None),
    "rand500_eq": lambda: (*P.random_spd(500, 0.01, 3, equal_weights=True), None),
    "rand5000_w": lambda: (*P.random_spd(5000, 0.002, 4), np.random.default_rng(9).uniform(0.2, 3, 5000)),
    "G1": lambda: (*[P.config("G1")[k] for k in ("rowptr", "col", "val")], None),
    "G2_30": lambda: (*[P.config("G2", 0.3)[k] for k in ("rowptr", "col", "val")], None),
    "G3_32": lambda: (*[P.config("G3", 0.2)[k] for k in ("rowptr", "col", "val")], None),
    "G4_10": lambda: (*[P.config("G4", 0.21)[k] for k in ("rowptr", "col", "val")], None),
}


@pytest.mark.parametrize("case", list(MATCH_CASES))
def test_matching_bitexact(B, ora, case):
    rp, ci, va, w = MATCH_CASES[case]()
    n = len(rp) - 1
    w = np.ones(n) if w is None else w
    c_ref = ora.weights(rp, ci, va, w)
    mate_ref = ora.match(rp, ci, c_ref)
    for rep in range(3):
        say(f"match {case} n={n} nnz={len(ci)} rep={rep}")
        mate, c = B.match(rp, ci, va, w)
        assert np.array_equal(_bits(c.cpu().numpy()), _bits(c_ref)), "edge weights differ"
        assert np.array_equal(mate.cpu().numpy(), mate_ref), "matching differs from greedy"


HIER_CASES = [("G1", 1.0), ("G2", 0.3), ("G3", 0.2), ("G4", 0.21), ("G5", 0.2), ("G2", 1.0), ("G5", 0.5),
              ("G3", 0.5)]


def _compare_hierarchy(h, ho):
    inf = h.info()
    assert inf["nl"] == ho.nl
    assert inf["n"] == ho.sizes() and inf["nnz"] == ho.nnzs()
    for k in range(ho.nl):
        g, o = h.level(k), ho.level(k)
        assert np.array_equal(g["rowptr"], o["rowptr"]), f"level {k} row_ptr"
        assert np.array_equal(g["col"], o["col"]), f"level {k} col"
        assert np.array_equal(_bits(g["val"]), _bits(o["val"])), f"level {k} values"
        assert np.array_equal(_bits(g["w"]), _bits(o["w"])), f"level {k} smooth vector"
        # sum of |a_ij| in another order: error bound (row length) ulp
        rl = np.diff(o["rowptr"]).astype(float)
        err = np.abs(g["dinv"] - o["dinv"]) / (rl * ULP * np.abs(o["dinv"]))
        assert err.max() <= 1.0, f"level {k} dinv: {err.max():.2f} x bound"
        if k < ho.nl - 1:
            assert np.array_equal(g["agg"], o["agg"]), f"level {k} aggregates"
            assert np.array_equal(_bits(g["p"]), _bits(o["p"])), f"level {k} prolongator"


@pytest.mark.parametrize("name,scale", HIER_CASES)
def test_hierarchy_bitexact(B, ora, name, scale):
    c = P.config(name, scale)
    say(f"setup {c['name']} n={c['n']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    _compare_hierarchy(h, ho)
    h.close()


def test_hierarchy_sweeps_1_and_3_and_random_w(B, ora):
    c = P.config("G3", 0.15)
    w = np.random.default_rng(1).uniform(0.5, 2.0, c["n"])
    for sweeps in (1, 3, 4):
        say(f"setup sweeps={sweeps} {c['name']}")
        h = B.Hierarchy(c["rowptr"], c["col"], c["val"], w, max_coarse=30, sweeps=sweeps)
        ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], w, max_coarse=30, sweeps=sweeps)
        _compare_hierarchy(h, ho)


@pytest.mark.parametrize("name,scale", [("G1", 1.0), ("G2", 0.3), ("G4", 0.21), ("G3", 0.2)])
def test_precond_fp64_parity(B, ora, name, scale):
    c = P.config(name, scale)
    say(f"precond fp64 {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    r = P.uniform_rhs(c["n"], 11)
    z = h.precond(r).cpu().numpy()
    zo = ho.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP64)


@pytest.mark.parametrize("name,scale", [("G1", 1.0), ("G2", 0.3), ("G4", 0.21)])
def test_precond_fp32_cycle_error_bound(B, ora, name, scale):
    # FP32 storage and accumulation: error vs the FP64 oracle stated as 1e-5 relative
    c = P.config(name, scale)
    say(f"precond fp32 {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], precision="fp32")
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    r = P.uniform_rhs(c["n"], 12)
    z = h.precond(r).cpu().numpy()
    zo = ho.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-5 * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP32)


@pytest.mark.parametrize("name,scale", [("G1", 1.0), ("G2", 0.3), ("G5", 0.2), ("G4", 0.21)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cycle,klevels", [("V", 0), ("W", 0), ("K", 1)])
def test_folded_coarse_levels(B, ora, name, scale, precision, cycle, klevels):
    # the small levels' cycle applied as one precomputed float64 operator
    # (the default) against the level-by-level cycle and the oracle: the same
    # linear map, rounded differently (fold from level 1 in G1 and G4, from
    # level 2 over four levels in G2).  W: each folded level's coarse problem
    # is 2T - T A T of the level below; K on the finest level: its two Krylov
    # steps use the folded cycle of level 1 and below.
    c = P.config(name, scale)
    say(f"folded levels {cycle} {precision} {c['name']}")
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], cycle=cycle,
                       kcycle_levels=klevels)
    r = P.uniform_rhs(c["n"], 21)
    zo = ho.vcycle(r)
    zs = []
    for fold in (True, False):
        h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], precision=precision,
                        fold=fold, cycle=cycle, kcycle_levels=klevels)
        zs.append(h.precond(r).cpu().numpy())
        h.close()
    bound = 1e-12 if precision == "fp64" else 1e-5
    for z in zs:
        assert np.linalg.norm(z - zo) <= bound * np.linalg.norm(zo)
        _close_entries(z, zo, ENTRY_FP64 if precision == "fp64" else ENTRY_FP32)
    assert np.linalg.norm(zs[0] - zs[1]) <= bound * np.linalg.norm(zo)


SOLVE_CASES = [("G1", 1.0), ("G2", 0.3), ("G3", 0.2), ("G4", 0.21), ("G2", 1.0), ("G5", 0.5)]


@pytest.mark.parametrize("name,scale", SOLVE_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_parity(B, ora, name, scale, precision):
    c = P.config(name, scale)
    say(f"solve {precision} {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], precision=precision)
    x = h.solve(c["b"], tol=c["tol"]).cpu().numpy()
    inf = h.info()
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    rel = np.linalg.norm(c["b"] - A @ x) / np.linalg.norm(c["b"])
    assert rel <= c["tol"], rel
    assert abs(inf["relres"] - rel) <= 1e-3 * rel + 1e-15
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    xo, io = ho.solve(c["b"], tol=c["tol"])
    say(f"solve {precision} {c['name']} iters gpu={inf['iters']} oracle={io['iters']} relres={rel:.3e}")
    allow = 1 if precision == "fp64" else _fp32_allowance(io["iters"])
    assert abs(inf["iters"] - io["iters"]) <= allow, (inf["iters"], io["iters"])


def test_solve_edge_cases(B):
    c = P.config("G1", 0.5)
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], itmax=1)
    say("solve zero rhs")
    x = h.solve(np.zeros(c["n"]))
    assert not x.any().item() and h.info()["iters"] == 0
    say("solve itmax=1")
    x = h.solve(c["b"], tol=1e-12, allow_maxit=True)
    assert h.info()["status"] == B.BCM_MAXIT and h.info()["iters"] == 1
    with pytest.raises(B.BcmError):
        h.solve(c["b"], tol=1e-12)
    say("solve with exact initial guess")
    h2 = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"])
    x = h2.solve(c["b"], tol=1e-10)
    x2 = h2.solve(c["b"], x0=x, tol=1e-8)
    assert h2.info()["iters"] == 0 and np.array_equal(x.cpu().numpy(), x2.cpu().numpy())


def test_single_level_and_tiny(B, ora):
    rp, ci, va = P.laplace1d(7)
    say("single level n=7")
    h = B.Hierarchy(rp, ci, va, max_coarse=100)
    ho = ora.Hierarchy(rp, ci, va, np.ones(7), max_coarse=100)
    assert h.info()["nl"] == 1
    r = P.uniform_rhs(7, 1)
    assert np.allclose(h.precond(r).cpu().numpy(), ho.vcycle(r), rtol=1e-13, atol=1e-15)
    x = h.solve(r, tol=1e-10).cpu().numpy()
    assert np.allclose(x, np.linalg.solve(sp.csr_matrix((va, ci, rp)).toarray(), r), rtol=1e-8)
    say("n=1")
    h1 = B.Hierarchy(np.array([0, 1]), np.array([0]), np.array([3.0]))
    assert np.allclose(h1.solve(np.array([6.0]), tol=1e-12).cpu().numpy(), [2.0])


def test_large_coarsest_level_global_sweeps(B, ora):
    # coarsest level above the one-workgroup LDS bound: global Jacobi sweeps
    c = P.config("G2", 0.4)  # 40^3 -> 16000 rows after one double-pairwise level
    say(f"large coarsest {c['name']} n={c['n']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=20000)
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=20000)
    assert h.info()["n"][-1] > 8192
    r = P.uniform_rhs(c["n"], 3)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP64)


def test_invalid_inputs_rejected(B):
    rp, ci, va = P.poisson2d(6)
    n = 36
    bad = []
    v = va.copy(); v[5] = np.nan; bad.append(("nan", rp, ci, v, None))
    v = va.copy(); v[0] = -4.0; bad.append(("diag<=0", rp, ci, v, None))
    v = va.copy(); v[1] = -0.5; bad.append(("asym", rp, ci, v, None))
    c2 = ci.copy(); c2[1], c2[2] = c2[2], c2[1]; bad.append(("unsorted", rp, c2, va, None))
    c3 = ci.copy(); c3[3] = 99; bad.append(("col range", rp, c3, va, None))
    r2 = rp.copy(); r2[4] = r2[5] + 1; bad.append(("rowptr", r2, ci, va, None))
    w = np.ones(n); w[7] = 0.0; bad.append(("w=0", rp, ci, va, w))
    for name, a, b_, c_, w_ in bad:
        say(f"invalid input {name}")
        with pytest.raises(B.BcmError) as e:
            B.Hierarchy(a, b_, c_, w_)
        assert e.value.code == B.BCM_EINVAL


def test_indefinite_matrix_breakdown(B):
    rp, ci, va = P.poisson2d(8)
    v = va.copy()
    v[np.repeat(np.arange(64), np.diff(rp)) == ci] = 0.6  # diagonal too small: indefinite
    say("indefinite")
    try:
        h = B.Hierarchy(rp, ci, v, max_coarse=100)
    except B.BcmError as e:  # a coarse level may already fail the s.p.d. checks
        assert e.code == B.BCM_EINVAL
        return
    with pytest.raises(B.BcmError) as e:
        h.solve(P.uniform_rhs(64, 0), tol=1e-10)
    assert e.value.code in (B.BCM_EBREAKDOWN,)


# ----------------------------------------------------------------------------- lane width (miniwarp)
@pytest.mark.parametrize("name,scale,group,sell", [("G2", 0.3, 4, False), ("G2", 0.3, 64, False),
                                                   ("G4", 0.21, 16, True), ("G4", 0.21, 64, False),
                                                   ("G3", 0.2, -1, False), ("G2", 0.3, -1, True)])
def test_lane_width_and_sell_settings(B, ora, name, scale, group, sell):
    # the hierarchy is bit-identical for every lane width (setup sums in a fixed
    # order); the cycle, with or without the sliced-ELL copies, within rounding
    c = P.config(name, scale)
    say(f"lane width {group} sell={sell} {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], group=group, sell=sell)
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
    _compare_hierarchy(h, ho)
    r = P.uniform_rhs(c["n"], 16)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP64)
    x = h.solve(c["b"], tol=c["tol"]).cpu().numpy()
    _, io = ho.solve(c["b"], tol=c["tol"])
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    assert np.linalg.norm(c["b"] - A @ x) <= c["tol"] * np.linalg.norm(c["b"])
    assert abs(h.info()["iters"] - io["iters"]) <= 1


def _cliques_and_hubs(nb=120, b=30, hubs=3, hub_deg=700, seed=5):
    # dense diagonal blocks (average row length >= 24: the sort-based rank,
    # candidate and Galerkin kernels) plus hub rows much longer than any lane
    # group's LDS slots (their direct-counting fallbacks)
    rng = np.random.default_rng(seed)
    n = nb * b + hubs
    rows, cols, vals = [], [], []
    for k in range(nb):
        idx = np.arange(k * b, (k + 1) * b)
        I, J = np.meshgrid(idx, idx, indexing="ij")
        off = I != J
        rows.append(I[off]); cols.append(J[off])
        vals.append(-rng.uniform(0.5, 1.5, off.sum()))
    for h in range(hubs):
        hub = nb * b + h
        nbrs = rng.choice(nb * b, hub_deg, replace=False)
        a = -rng.uniform(0.2, 0.8, hub_deg)
        rows += [np.full(hub_deg, hub), nbrs]; cols += [nbrs, np.full(hub_deg, hub)]; vals += [a, a]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A = (A + A.T) * 0.5
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


@pytest.mark.parametrize("group", [0, 4, 16])
def test_hierarchy_dense_blocks_and_hub_rows(B, ora, group):
    rp, ci, va = _cliques_and_hubs()
    n = len(rp) - 1
    assert len(ci) >= 24 * n and np.diff(rp).max() > 16 * 32
    say(f"dense blocks and hubs n={n} nnz={len(ci)} group={group}")
    h = B.Hierarchy(rp, ci, va, max_coarse=40, group=group)
    ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=40)
    _compare_hierarchy(h, ho)
    h.close()


def test_sell_uniform_and_mixed_slices(B, ora):
    # a 7-point grid (slices whose rows share one offset list: offsets read once
    # per slice) with a few long couplings added (their slices store offsets per
    # entry); both kinds in one matrix, against the oracle
    rp, ci, va = P.poisson3d(40)
    n = len(rp) - 1
    A = sp.csr_matrix((va, ci, rp), shape=(n, n)).tolil()
    rng = np.random.default_rng(31)
    for _ in range(60):
        i = int(rng.integers(0, n - 20000))
        j = i + int(rng.integers(2, 20000))  # offsets within int16: the copy keeps int16 offsets
        a = -rng.uniform(0.1, 0.5)
        A[i, j] = A[j, i] = a
        A[i, i] = A[i, i] - a
        A[j, j] = A[j, j] - a
    A = A.tocsr()
    A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()
    say(f"sliced ELL uniform and mixed slices n={n}")
    for precision, bound in (("fp64", 1e-12), ("fp32", 1e-5)):
        h = B.Hierarchy(rp, ci, va, max_coarse=100, precision=precision)
        ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=100)
        if precision == "fp64":
            _compare_hierarchy(h, ho)
        r = P.uniform_rhs(n, 23)
        z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
        assert np.linalg.norm(z - zo) <= bound * np.linalg.norm(zo)
        _close_entries(z, zo, ENTRY_FP64 if precision == "fp64" else ENTRY_FP32)
        b = P.uniform_rhs(n, 24)
        x = h.solve(b, tol=1e-8).cpu().numpy()
        assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
        _, io = ho.solve(b, tol=1e-8)
        assert abs(h.info()["iters"] - io["iters"]) <= (1 if precision == "fp64" else _fp32_allowance(io["iters"]))
        h.close()


def test_sell_int32_columns_for_long_range_couplings(B, ora):
    # offsets |col - row| beyond int16: the sliced-ELL copies keep int32 columns
    rp, ci, va = P.random_spd(70000, 4e-5, 23)
    n = len(rp) - 1
    assert np.abs(ci - np.repeat(np.arange(n), np.diff(rp))).max() > 32767
    say(f"sliced ELL with int32 columns n={n}")
    h = B.Hierarchy(rp, ci, va, max_coarse=200)
    ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=200)
    _compare_hierarchy(h, ho)
    r = P.uniform_rhs(n, 18)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-12 * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP64)
    b = P.uniform_rhs(n, 19)
    x = h.solve(b, tol=1e-8).cpu().numpy()
    _, io = ho.solve(b, tol=1e-8)
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert abs(h.info()["iters"] - io["iters"]) <= 1


def test_wide_rows_int32_columns_split_kernels(B, ora):
    # 70,000 rows averaging 38 entries, couplings beyond int16 offsets: the
    # finest level takes the slot-split kernels (residual, smoother and the
    # flexible-CG product with one partial per slice) on int32 columns and gets
    # dinv o r from the update; level 1 (17,928 rows, about 2M entries) runs
    # split legs too, its dinv o b formed by the restriction
    rp, ci, va = P.random_spd(70000, 2.5e-4, 29)
    n = len(rp) - 1
    assert len(ci) >= 16 * n and np.abs(ci - np.repeat(np.arange(n), np.diff(rp))).max() > 32767
    say(f"wide rows, int32 columns n={n} nnz={len(ci)}")
    h = B.Hierarchy(rp, ci, va, max_coarse=200)
    ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=200)
    _compare_hierarchy(h, ho)
    r = P.uniform_rhs(n, 18)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    _close_entries(z, zo, ENTRY_FP64)
    b = P.uniform_rhs(n, 19)
    _, io = ho.solve(b, tol=1e-8)
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    for precision, rtol in (("fp64", 1e-12), ("fp32", 1e-5)):
        say(f"wide rows: three iterations {precision}")
        h3 = B.Hierarchy(rp, ci, va, max_coarse=200, precision=precision, itmax=3)
        x3 = h3.solve(b, tol=1e-30, allow_maxit=True).cpu().numpy()
        h3.close()
        xo3, _ = ho.solve(b, tol=1e-30, itmax=3)
        _close_entries(x3, xo3, rtol)
        hs = B.Hierarchy(rp, ci, va, max_coarse=200, precision=precision)
        x = hs.solve(b, tol=1e-8).cpu().numpy()
        assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
        allow = 1 if precision == "fp64" else _fp32_allowance(io["iters"])
        assert abs(hs.info()["iters"] - io["iters"]) <= allow, (hs.info()["iters"], io["iters"])
        hs.close()


# ----------------------------------------------------------------------------- W-cycle
@pytest.mark.parametrize("name,scale,precision", [("G1", 1.0, "fp64"), ("G2", 0.3, "fp64"), ("G4", 0.21, "fp64"),
                                                  ("G2", 0.3, "fp32")])
def test_w_cycle_parity(B, ora, name, scale, precision):
    c = P.config(name, scale)
    say(f"W-cycle {precision} {c['name']}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], cycle="W",
                    precision=precision)
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], cycle="W")
    r = P.uniform_rhs(c["n"], 13)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    bound = 1e-12 if precision == "fp64" else 1e-5
    assert np.linalg.norm(z - zo) <= bound * np.linalg.norm(zo)
    _close_entries(z, zo, ENTRY_FP64 if precision == "fp64" else ENTRY_FP32)
    x = h.solve(c["b"], tol=c["tol"]).cpu().numpy()
    xo, io = ho.solve(c["b"], tol=c["tol"])
    inf = h.info()
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    assert np.linalg.norm(c["b"] - A @ x) <= c["tol"] * np.linalg.norm(c["b"])
    say(f"W-cycle {precision} {c['name']} iters gpu={inf['iters']} oracle={io['iters']}")
    allow = 1 if precision == "fp64" else _fp32_allowance(io["iters"])
    assert abs(inf["iters"] - io["iters"]) <= allow, (inf["iters"], io["iters"])


# ----------------------------------------------------------------------------- K-cycle
@pytest.mark.parametrize("name,scale,precision,klevels", [("G1", 1.0, "fp64", 0), ("G2", 0.3, "fp64", 0),
                                                          ("G2", 0.3, "fp64", 1), ("G3", 0.2, "fp64", 2),
                                                          ("G4", 0.21, "fp64", 0), ("G2", 0.3, "fp32", 0)])
def test_k_cycle_parity(B, ora, name, scale, precision, klevels):
    c = P.config(name, scale)
    say(f"K-cycle {precision} {c['name']} kcycle_levels={klevels}")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], cycle="K",
                    kcycle_levels=klevels, precision=precision)
    ho = ora.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], cycle="K",
                       kcycle_levels=klevels)
    r = P.uniform_rhs(c["n"], 14)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    say(f"K-cycle {precision} {c['name']} precond rel err {err:.2e}")
    assert err <= (1e-11 if precision == "fp64" else 1e-4)
    # the K-cycle is nonlinear (its coarse steps divide by dot products): ten
    # times the linear cycles' entry-wise bounds
    _close_entries(z, zo, 10 * (ENTRY_FP64 if precision == "fp64" else ENTRY_FP32))
    x = h.solve(c["b"], tol=c["tol"]).cpu().numpy()
    xo, io = ho.solve(c["b"], tol=c["tol"])
    inf = h.info()
    A = sp.csr_matrix((c["val"], c["col"], c["rowptr"]), shape=(c["n"], c["n"]))
    assert np.linalg.norm(c["b"] - A @ x) <= c["tol"] * np.linalg.norm(c["b"])
    say(f"K-cycle {precision} {c['name']} iters gpu={inf['iters']} oracle={io['iters']}")
    if precision == "fp64":
        assert abs(inf["iters"] - io["iters"]) <= max(1, int(0.03 * io["iters"])), (inf["iters"], io["iters"])


def test_k_cycle_zero_and_scaled_rhs(B):
    # b = 0 ends the coarse flexible CG at once (rho = 0): B(0) = 0; the cycle
    # is homogeneous: B(2r) = 2 B(r) bit for bit
    c = P.config("G2", 0.3)
    say("K-cycle zero and scaled right-hand side")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], cycle="K")
    assert not h.precond(np.zeros(c["n"])).any().item()
    r = P.uniform_rhs(c["n"], 15)
    z1 = h.precond(r).cpu().numpy()
    z2 = h.precond(2.0 * r).cpu().numpy()
    assert np.array_equal(z2, 2.0 * z1)


# ----------------------------------------------------------------------------- HIP graph replay
@pytest.mark.parametrize("cycle,precision", [("V", "fp64"), ("V", "fp32"), ("W", "fp64"), ("K", "fp64"),
                                             ("K", "fp32")])
def test_graph_replay_equals_eager(B, cycle, precision):
    # the captured iteration is replayed across several solves, with eager work in
    # between; every result must equal the eager solve bit for bit
    c = P.config("G2", 0.3)
    say(f"graph replay {cycle} {precision}")
    he = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], cycle=cycle,
                     precision=precision, graph=False)
    hg = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], cycle=cycle,
                     precision=precision, graph=True)
    for seed in (1, 2, 1):
        b = P.uniform_rhs(c["n"], seed)
        xe = he.solve(b, tol=1e-9).cpu().numpy()
        ie = he.info()["iters"]
        z = hg.precond(b)  # eager work on the same handle between replays
        xg = hg.solve(b, tol=1e-9).cpu().numpy()
        assert hg.info()["iters"] == ie
        assert np.array_equal(xg.view(np.uint64), xe.view(np.uint64))
        assert z.isfinite().all().item()


@pytest.mark.parametrize("cls", ["spmv_dots", "down0", "coarse"])
def test_graph_profiling_times_one_class(B, cls):
    # with a one-class profile mask the iteration still runs from the graph; the
    # class is timed by event nodes inside it and the result is unchanged
    c = P.config("G2", 0.3)
    say(f"graph profiling {cls}")
    b = P.uniform_rhs(c["n"], 3)
    he = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], graph=False)
    hg = B.Hierarchy(c["rowptr"], c["col"], c["val"], max_coarse=c["max_coarse"], graph=True,
                     profile=B.PROF[cls])
    xe = he.solve(b, tol=1e-9).cpu().numpy()
    xg = hg.solve(b, tol=1e-9).cpu().numpy()
    assert np.array_equal(xg.view(np.uint64), xe.view(np.uint64))
    launches, ms, by = hg.profile(cls)
    # the eager first iteration plus at least one replay sample
    assert 2 <= launches <= hg.info()["iters"]
    assert ms > 0.0 and by > 0.0


# ----------------------------------------------------------------------------- long (hub) rows
def _hubs(n_leaf=60000, hubs=(0,), path=True, seed=3, frac=1.0):
    # hub rows coupled to (a fraction of) all other rows with random weights,
    # plus a path through the non-hub rows: rows far longer than any lane
    # group's bound (the per-row kernels hand them to the long-row path)
    rng = np.random.default_rng(seed)
    n = n_leaf + len(hubs)
    hub_set = set(hubs)
    others = np.array([i for i in range(n) if i not in hub_set])
    rows, cols, vals = [], [], []
    for h in hubs:
        nb = others if frac >= 1.0 else rng.choice(others, int(frac * len(others)), replace=False)
        a = -rng.uniform(0.1, 1.0, len(nb))
        rows += [np.full(len(nb), h), nb]; cols += [nb, np.full(len(nb), h)]; vals += [a, a]
    if path:
        a = -rng.uniform(0.1, 1.0, len(others) - 1)
        rows += [others[:-1], others[1:]]; cols += [others[1:], others[:-1]]; vals += [a, a]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A = (A + A.T) * 0.5
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + rng.uniform(0.05, 0.5, n))
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def _two_hubs_paired(n_leaf=30000, seed=4):
    # two hubs coupled to every leaf and, most strongly, to each other: the
    # greedy matching pairs them, so one aggregate holds two long rows
    rp, ci, va = _hubs(n_leaf=n_leaf, hubs=(0, 1), path=True, seed=seed)
    A = sp.csr_matrix((va, ci, rp), shape=(len(rp) - 1, len(rp) - 1)).tolil()
    A[0, 1] = A[1, 0] = -5000.0
    A[0, 0] = A[0, 0] + 5000.0
    A[1, 1] = A[1, 1] + 5000.0
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


LONG_CASES = {
    "star60k": lambda: _hubs(path=False),
    "star60k_equal": lambda: (lambda rp, ci, va: (rp, ci, np.where(va < 0, -0.5, va)))(*_hubs(path=False)),
    "hubs3_path": lambda: _hubs(n_leaf=40000, hubs=(0, 17000, 40002), frac=0.5),
}


@pytest.mark.parametrize("case", list(LONG_CASES))
def test_long_rows_matching_bitexact(B, ora, case):
    rp, ci, va = LONG_CASES[case]()
    n = len(rp) - 1
    w = np.ones(n)
    c_ref = ora.weights(rp, ci, va, w)
    mate_ref = ora.match(rp, ci, c_ref)
    say(f"long rows match {case} n={n} longest={np.diff(rp).max()}")
    mate, c = B.match(rp, ci, va, w)
    assert np.array_equal(_bits(c.cpu().numpy()), _bits(c_ref)), "edge weights differ"
    assert np.array_equal(mate.cpu().numpy(), mate_ref), "matching differs from greedy"


@pytest.mark.parametrize("case,group,precision", [("hubs3_path", 0, "fp64"), ("hubs3_path", 64, "fp64"),
                                                  ("star60k", 0, "fp64"), ("star60k", 0, "fp32"),
                                                  ("hubs2_paired", 0, "fp64"), ("hubs2_paired", 0, "fp32")])
def test_long_rows_hierarchy_cycle_solve(B, ora, case, group, precision):
    # the row-wise cycle legs (up leg, coarsest sweeps) of levels with long
    # rows run the rows' chunks in the row kernel's own launch (one finishing
    # block per long row); the down leg sums them in a pre-pass (hubs2_paired:
    # one aggregate holds two long rows)
    rp, ci, va = (LONG_CASES[case] if case in LONG_CASES else _two_hubs_paired)()
    n = len(rp) - 1
    say(f"long rows hierarchy {case} group={group} {precision} n={n}")
    h = B.Hierarchy(rp, ci, va, max_coarse=50, group=group, precision=precision)
    ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=50)
    if precision == "fp64":
        _compare_hierarchy(h, ho)
    else:
        assert h.info()["n"] == ho.sizes()
    if case == "hubs2_paired":
        agg0 = h.level(0)["agg"]
        assert agg0[0] == agg0[1], "the two hubs should share an aggregate"
    r = P.uniform_rhs(n, 31)
    z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
    _close_entries(z, zo, 1e-11 if precision == "fp64" else ENTRY_FP32)
    b = P.uniform_rhs(n, 32)
    x = h.solve(b, tol=1e-8).cpu().numpy()
    _, io = ho.solve(b, tol=1e-8)
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    allow = 1 if precision == "fp64" else _fp32_allowance(io["iters"])
    assert abs(h.info()["iters"] - io["iters"]) <= allow, (h.info()["iters"], io["iters"])
    h.close()


def _random_star(n, seed):
    # one hub (row 0) coupled to every other row, each of which holds only its
    # diagonal and the hub entry; random couplings and diagonal dominance
    rng = np.random.default_rng(seed)
    a = -rng.uniform(0.1, 1.0, n - 1)
    rows = np.concatenate([np.zeros(n - 1, int), np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(1, n), np.zeros(n - 1, int), np.arange(n)])
    diag = np.concatenate([[1.1 * np.abs(a).sum()], np.abs(a) * rng.uniform(1.0, 2.0, n - 1)])
    A = sp.csr_matrix((np.concatenate([a, a, diag]), (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_star_coarsest_level_recurrence(B, ora, precision):
    # a coarsest level shaped as a star (too large for the dense operator, its
    # hub a long row) takes the hub recurrence instead of one launch per
    # sweep: the same 20 sweeps up to the rounding of the hub's sums
    n = 6000
    rp, ci, va = _random_star(n, 5)
    say(f"star coarsest level {precision} n={n}")
    h = B.Hierarchy(rp, ci, va, max_coarse=2 * n, precision=precision)
    ho = ora.Hierarchy(rp, ci, va, np.ones(n), max_coarse=2 * n)
    assert h.info()["nl"] == 1 and h.info()["long_rows"] >= 1
    for seed in (41, 42):
        r = P.uniform_rhs(n, seed)
        z, zo = h.precond(r).cpu().numpy(), ho.vcycle(r)
        _close_entries(z, zo, 1e-12 if precision == "fp64" else ENTRY_FP32)
    b = P.uniform_rhs(n, 43)
    x = h.solve(b, tol=1e-9).cpu().numpy()
    _, io = ho.solve(b, tol=1e-9)
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b)
    allow = 1 if precision == "fp64" else _fp32_allowance(io["iters"])
    assert abs(h.info()["iters"] - io["iters"]) <= allow, (h.info()["iters"], io["iters"])
    h.close()


def test_true_residual_stagnation_status(B):
    # a tolerance below the rounding floor of b - A x: the recurrence residual
    # keeps falling, the true one cannot follow; after three restarts the solve
    # reports BCM_STAGNATED (not BCM_MAXIT: far fewer than itmax iterations ran)
    c = P.config("G1", 1.0)
    say("stagnation below the rounding floor")
    h = B.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"], precision="fp32")
    h.solve(c["b"], tol=1e-17, allow_maxit=True)
    inf = h.info()
    assert inf["status"] == B.BCM_STAGNATED and inf["iters"] < 1000, inf
    assert 1e-17 < inf["relres"] < 1e-12
    with pytest.raises(B.BcmError) as e:
        h.solve(c["b"], tol=1e-17)
    assert e.value.code == B.BCM_STAGNATED and "stagnated" in str(e.value)
