"""ctypes shim over the serial FP64 oracle (bcm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing in the GPU library imports,
links or calls this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bcm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.c_void_p
        I = C.c_int
        D = C.c_double
        L.ora_weights.argtypes = [I, P, P, P, P, P]
        L.ora_match.argtypes = [I, P, P, P, P]
        L.ora_aggregate.argtypes = [I, P, P, P, P]
        L.ora_prolong.argtypes = [I, P, I, P, P, P]
        L.ora_galerkin.argtypes = [I, P, P, P, P, P, I, P, P, P]
        L.ora_l1_dinv.argtypes = [I, P, P, P, P]
        L.ora_setup.argtypes = [I, P, P, P, P, I, I, I, I, I, I, D, C.POINTER(I)]
        L.ora_setup.restype = P
        L.ora_free.argtypes = [P]
        L.ora_nlevels.argtypes = [P]
        L.ora_level_n.argtypes = [P, I]
        L.ora_level_nnz.argtypes = [P, I]
        L.ora_level_npairs.argtypes = [P, I, I]
        L.ora_level_get.argtypes = [P, I, P, P, P, P, P, P, P]
        L.ora_vcycle.argtypes = [P, P, P]
        L.ora_fcg.argtypes = [P, I, P, P, D, I, C.POINTER(I), C.POINTER(D)]
        L.ora_sampled_outer.argtypes = [I, P, P, P, P, P]
        L.ora_spmv.argtypes = [I, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def weights(rp, ci, va, w):
    rp, ci, va, w = _i32(rp), _i32(ci), _f64(va), _f64(w)
    c = np.empty(len(ci))
    lib().ora_weights(len(rp) - 1, _p(rp), _p(ci), _p(va), _p(w), _p(c))
    return c


def match(rp, ci, c):
    rp, ci, c = _i32(rp), _i32(ci), _f64(c)
    mate = np.empty(len(rp) - 1, dtype=np.int32)
    lib().ora_match(len(rp) - 1, _p(rp), _p(ci), _p(c), _p(mate))
    return mate


def aggregate(mate):
    mate = _i32(mate)
    agg = np.empty(len(mate), dtype=np.int32)
    npairs, nsing = C.c_int(), C.c_int()
    nc = lib().ora_aggregate(len(mate), _p(mate), _p(agg), C.byref(npairs), C.byref(nsing))
    return agg, nc, npairs.value, nsing.value


def prolong(agg, nc, w):
    agg, w = _i32(agg), _f64(w)
    p = np.empty(len(agg))
    wc = np.empty(nc)
    if lib().ora_prolong(len(agg), _p(agg), nc, _p(w), _p(p), _p(wc)) != 0:
        raise ValueError("aggregates are not pairs")
    return p, wc


def galerkin(rp, ci, va, agg, p, nc):
    rp, ci, va, agg, p = _i32(rp), _i32(ci), _f64(va), _i32(agg), _f64(p)
    n = len(rp) - 1
    nnz = lib().ora_galerkin(n, _p(rp), _p(ci), _p(va), _p(agg), _p(p), nc, None, None, None)
    crp = np.empty(nc + 1, dtype=np.int32)
    cci = np.empty(nnz, dtype=np.int32)
    cva = np.empty(nnz)
    lib().ora_galerkin(n, _p(rp), _p(ci), _p(va), _p(agg), _p(p), nc, _p(crp), _p(cci), _p(cva))
    return crp, cci, cva


def l1_dinv(rp, ci, va):
    rp, ci, va = _i32(rp), _i32(ci), _f64(va)
    d = np.empty(len(rp) - 1)
    lib().ora_l1_dinv(len(rp) - 1, _p(rp), _p(ci), _p(va), _p(d))
    return d


def spmv(rp, ci, va, x):
    rp, ci, va, x = _i32(rp), _i32(ci), _f64(va), _f64(x)
    y = np.empty(len(rp) - 1)
    lib().ora_spmv(len(rp) - 1, _p(rp), _p(ci), _p(va), _p(x), _p(y))
    return y


def sampled_outer(rp, ci, lam, x):
    rp, ci, lam, x = _i32(rp), _i32(ci), _f64(lam), _f64(x)
    G = np.empty(len(ci))
    lib().ora_sampled_outer(len(rp) - 1, _p(rp), _p(ci), _p(lam), _p(x), _p(G))
    return G


PRECOND = {"identity": 0, "amg": 1, "jacobi": 2}
CYCLES = {"V": 1, "W": 2, "K": 3}


class Hierarchy:
    """Oracle hierarchy (Section 2.1): levels A^k, smooth vectors w^k, l1 diagonals
    and the composed prolongators P^k (column agg, value p)."""

    def __init__(self, rp, ci, va, w, max_levels=40, max_coarse=None, sweeps=2,
                 coarse_sweeps=20, cycle="V", kcycle_levels=0, min_ratio=0.0):
        self._keep = [_i32(rp), _i32(ci), _f64(va), _f64(w)]
        rp, ci, va, w = self._keep
        n = len(rp) - 1
        if max_coarse is None:
            max_coarse = int(round(40.0 * float(np.cbrt(n))))
        st = C.c_int()
        self.h = lib().ora_setup(n, _p(rp), _p(ci), _p(va), _p(w), max_levels, max_coarse,
                                 sweeps, coarse_sweeps, CYCLES[cycle], kcycle_levels, float(min_ratio),
                                 C.byref(st))
        if not self.h:
            raise ValueError(f"oracle setup rejected the input (status {st.value})")
        self.n = n
        self.nl = lib().ora_nlevels(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().ora_free(self.h)
            self.h = None

    def level(self, k: int) -> dict:
        n = lib().ora_level_n(self.h, k)
        nnz = lib().ora_level_nnz(self.h, k)
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        va = np.empty(nnz)
        w = np.empty(n)
        dinv = np.empty(n)
        agg = np.empty(n, dtype=np.int32)
        p = np.empty(n)
        lib().ora_level_get(self.h, k, _p(rp), _p(ci), _p(va), _p(w), _p(dinv), _p(agg), _p(p))
        out = dict(n=n, nnz=nnz, rowptr=rp, col=ci, val=va, w=w, dinv=dinv)
        if k < self.nl - 1:
            out["agg"], out["p"] = agg, p
        return out

    def npairs(self, k: int, s: int) -> int:
        return lib().ora_level_npairs(self.h, k, s)

    def sizes(self):
        return [lib().ora_level_n(self.h, k) for k in range(self.nl)]

    def nnzs(self):
        return [lib().ora_level_nnz(self.h, k) for k in range(self.nl)]

    def vcycle(self, b):
        b = _f64(b)
        x = np.empty(self.n)
        lib().ora_vcycle(self.h, _p(b), _p(x))
        return x

    def solve(self, b, tol=1e-8, itmax=5000, x0=None, precond="amg"):
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        it, rr = C.c_int(), C.c_double()
        st = lib().ora_fcg(self.h, PRECOND[precond], _p(b), _p(x), tol, itmax,
                           C.byref(it), C.byref(rr))
        return x, dict(status=st, iters=it.value, relres=rr.value)
