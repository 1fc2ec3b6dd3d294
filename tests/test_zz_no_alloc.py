"""The allocation-free matching entry point (bcm_match_noalloc) against
bcm_match, through the C ABI: mate and the edge weights bit for bit, on two
calls in a row (the second on a smaller graph, so it runs over what the first
left in the shared static scratch), on a graph with a hub row (the long-row
path takes its sort keys from the same array), and the size limit.
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


def _star(n):
    A = sp.lil_matrix((n, n))
    for j in range(1, n):
        A[0, j] = A[j, 0] = -1.0
    A.setdiag([n + 1.0] + [2.0] * (n - 1))
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def _both(B, rp, ci, va, w=None):
    m0, c0 = B.match(rp, ci, va, w)
    m1, c1 = B.match(rp, ci, va, w, noalloc=True)
    m0, c0, m1, c1 = (t.cpu().numpy() for t in (m0, c0, m1, c1))
    assert np.array_equal(m0, m1), "mate differs"
    assert np.array_equal(c0.view(np.uint64), c1.view(np.uint64)), "weights differ"
    return m1


def test_noalloc_match_equals_match_two_calls(B):
    c = P.config("G2", 0.5)  # 50^3 Poisson, then 2-D Poisson 64^2
    say(f"noalloc match {c['name']} n={c['n']}")
    mate = _both(B, c["rowptr"], c["col"], c["val"])
    assert (mate >= 0).sum() > 0
    c2 = P.config("G1")
    say(f"noalloc match {c2['name']} n={c2['n']} (smaller, second call)")
    _both(B, c2["rowptr"], c2["col"], c2["val"])
    w = np.random.default_rng(3).uniform(0.5, 1.5, c2["n"])
    say("noalloc match G1 with random w")
    _both(B, c2["rowptr"], c2["col"], c2["val"], w)


def test_noalloc_match_long_rows_and_without_weights(B):
    rp, ci, va = _star(20000)
    say("noalloc match star 20000 (hub row)")
    mate = _both(B, rp, ci, va)
    assert mate[0] >= 0
    rp2, ci2, va2 = P.laplace1d(4097)
    say("noalloc match path 4097, weights not returned")
    m0, _ = B.match(rp2, ci2, va2)
    m1, c1 = B.match(rp2, ci2, va2, noalloc=True, weights=False)
    assert c1 is None
    assert np.array_equal(m0.cpu().numpy(), m1.cpu().numpy())


def test_noalloc_match_size_limit(B):
    # 20 n + 12 nnz (+ 8 nnz without a caller weight array) beyond 64 MiB:
    # rejected before any kernel runs
    nx = 128  # 128^3 Poisson: n = 2.1e6, nnz = 1.46e7
    rp, ci, va = P.poisson3d(nx)
    say(f"noalloc match size limit poisson3d_{nx}^3")
    with pytest.raises(B.BcmError) as e:
        B.match(rp, ci, va, noalloc=True)
    assert e.value.code == -1 and "static" in str(e.value)
