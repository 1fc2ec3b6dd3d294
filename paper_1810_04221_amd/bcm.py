"""Python binding of the gfx950 library (libbcm.so): argument marshalling only.

Every step of setup and solve runs in the library's HIP kernels; PyTorch
supplies device memory (its caching allocator is handed to the library as the
device allocator) and the stream.  There is no fallback: without the built
library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcm.so")

BCM_OK, BCM_MAXIT, BCM_STAGNATED, BCM_EINVAL, BCM_EBREAKDOWN, BCM_ENOMEM, BCM_EHIP = 0, 1, 2, -1, -2, -3, -4
BCM_FP64, BCM_FP32_CYCLE = 0, 1
CYCLES = {"V": 1, "W": 2, "K": 3}  # BCM_VCYCLE, BCM_WCYCLE, BCM_KCYCLE
PROF = {"down0": 1, "up0": 2, "spmv_dots": 4, "update": 8, "coarse": 16, "mid": 32,
        "setup_match": 64, "setup_suitor": 128, "setup_galerkin": 256}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class BcmCsr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class BcmParams(C.Structure):
    _fields_ = [("max_levels", C.c_int32), ("max_coarse", C.c_int32), ("sweeps", C.c_int32),
                ("coarse_sweeps", C.c_int32), ("pre", C.c_int32), ("post", C.c_int32), ("cycle", C.c_int32),
                ("kcycle_levels", C.c_int32), ("precision", C.c_int32), ("itmax", C.c_int32),
                ("check", C.c_int32), ("profile", C.c_int32), ("graph", C.c_int32), ("group", C.c_int32),
                ("sell", C.c_int32), ("fold", C.c_int32), ("adjoint_tol", C.c_double), ("min_ratio", C.c_double), ("alloc", ALLOC_FN),
                ("dealloc", DEALLOC_FN), ("alloc_ctx", C.c_void_p), ("stream", C.c_void_p)]


class BcmInfo(C.Structure):
    _fields_ = [("nl", C.c_int32), ("precision", C.c_int32), ("iters", C.c_int32), ("status", C.c_int32),
                ("n", C.c_int32 * 64), ("nnz", C.c_int64 * 64), ("vcmplx", C.c_double), ("cratio", C.c_double),
                ("cratio_nl", C.c_double), ("relres", C.c_double), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("cycle_bytes", C.c_double), ("iter_bytes", C.c_double),
                ("setup_bytes", C.c_double), ("sweeps_run", C.c_int32), ("long_rows", C.c_int32)]


EXPORTS = ["bcm_default_params", "bcm_setup", "bcm_solve", "bcm_precond", "bcm_solve_adjoint", "bcm_sampled_outer", "bcm_info",
           "bcm_level_copy", "bcm_match", "bcm_match_noalloc", "bcm_profile", "bcm_free", "bcm_last_error"]

_lib = None


class BcmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bcm error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Loads libbcm.so and declares the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1810_04221_amd.build`")
    L = C.CDLL(path)
    P, I32 = C.c_void_p, C.c_int32
    L.bcm_default_params.argtypes = [C.POINTER(BcmParams)]
    L.bcm_default_params.restype = None
    L.bcm_setup.argtypes = [C.POINTER(BcmCsr), P, C.POINTER(BcmParams), C.POINTER(P)]
    L.bcm_solve.argtypes = [P, P, P, C.c_double]
    L.bcm_precond.argtypes = [P, P, P]
    L.bcm_solve_adjoint.argtypes = [P, P, P]
    L.bcm_sampled_outer.argtypes = [P, P, P, P]
    L.bcm_info.argtypes = [P, C.POINTER(BcmInfo)]
    L.bcm_level_copy.argtypes = [P, I32, P, P, P, P, P, P, P]
    L.bcm_match.argtypes = [C.POINTER(BcmCsr), P, C.POINTER(BcmParams), P, P]
    L.bcm_match_noalloc.argtypes = [C.POINTER(BcmCsr), P, C.POINTER(BcmParams), P, P]
    L.bcm_profile.argtypes = [P, I32, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.bcm_free.argtypes = [P]
    L.bcm_free.restype = None
    L.bcm_last_error.restype = C.c_char_p
    _lib = L
    return L


def _gpu_lib():
    L = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the library runs only on a gfx950 device")
    return L


def _check(rc: int, allow=(BCM_OK,)):
    if rc not in allow:
        raise BcmError(rc, load_library().bcm_last_error().decode())
    return rc


def _dev(t, dtype, device):
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


class _TorchAllocator:
    """The library's device allocator, backed by PyTorch's caching allocator."""

    def __init__(self, device: torch.device, stream: int):
        self.device, self.stream = device, stream

        def alloc(size, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), self.device, self.stream)
            except Exception:  # reported to the library as an allocation failure
                return None

        def dealloc(ptr, size, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = ALLOC_FN(alloc)
        self.dealloc = DEALLOC_FN(dealloc)


def make_params(precision="fp64", max_levels=40, max_coarse=0, sweeps=2, coarse_sweeps=20, itmax=5000,
                check=True, adjoint_tol=0.0, profile=0, stream=None, allocator=None, cycle="V",
                graph=False, kcycle_levels=0, group=0, sell=True, min_ratio=0.0, fold=True) -> BcmParams:
    p = BcmParams()
    load_library().bcm_default_params(C.byref(p))
    p.cycle = CYCLES[cycle]
    p.kcycle_levels = kcycle_levels
    p.group, p.sell, p.fold = group, int(bool(sell)), int(bool(fold))
    p.min_ratio = float(min_ratio)
    p.graph = int(bool(graph))
    p.max_levels, p.max_coarse, p.sweeps, p.coarse_sweeps = max_levels, max_coarse, sweeps, coarse_sweeps
    p.precision = {"fp64": BCM_FP64, "fp32": BCM_FP32_CYCLE}[precision]
    p.itmax, p.check, p.adjoint_tol, p.profile = itmax, int(bool(check)), adjoint_tol, profile
    p.stream = stream
    if allocator is not None:
        p.alloc, p.dealloc = allocator.alloc, allocator.dealloc
    return p


class Hierarchy:
    """AMG hierarchy built on the GPU by ``bcm_setup`` from a CSR matrix and a
    smooth vector ``w`` (defaults to ones).  Inputs may be numpy arrays or
    tensors; they are copied to the device as int32 / float64."""

    def __init__(self, rowptr, col, val, w=None, *, precision="fp64", max_levels=40, max_coarse=0, sweeps=2,
                 coarse_sweeps=20, itmax=5000, check=True, adjoint_tol=0.0, profile=0, device=None, cycle="V",
                 graph=False, kcycle_levels=0, group=0, sell=True, min_ratio=0.0, fold=True):
        L = _gpu_lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device).cuda_stream
        self.rowptr = _dev(rowptr, torch.int32, self.device)
        self.col = _dev(col, torch.int32, self.device)
        # a copy of its own: the values the hierarchy was built from, for
        # check_values (a device tensor passed in would otherwise be aliased)
        self.val = _dev(val, torch.float64, self.device).clone()
        self.n = self.rowptr.numel() - 1
        self.nnz = self.col.numel()
        w = torch.ones(self.n, dtype=torch.float64, device=self.device) if w is None else _dev(w, torch.float64, self.device)
        self._alloc = _TorchAllocator(self.device, self.stream)
        self.params = make_params(precision, max_levels, max_coarse, sweeps, coarse_sweeps, itmax, check,
                                  adjoint_tol, profile, self.stream, self._alloc, cycle, graph, kcycle_levels,
                                  group, sell, min_ratio, fold)
        A = BcmCsr(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr())
        h = C.c_void_p()
        _check(L.bcm_setup(C.byref(A), C.c_void_p(w.data_ptr()), C.byref(self.params), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load_library().bcm_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # The library works on the stream captured at construction.  Inputs made on
    # the caller's current stream are waited for before a call, and outputs are
    # made visible to that stream after it.
    def _enter(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream == self.stream:
            return cur, None
        lib = torch.cuda.ExternalStream(self.stream, device=self.device)
        lib.wait_stream(cur)
        return cur, lib

    def _leave(self, cur, lib):
        if lib is not None:
            cur.wait_stream(lib)

    def solve(self, b, x0=None, tol=1e-8, allow_maxit=False):
        b = _dev(b, torch.float64, self.device)
        x = torch.zeros(self.n, dtype=torch.float64, device=self.device) if x0 is None else _dev(x0, torch.float64, self.device).clone()
        cur, lib = self._enter()
        rc = load_library().bcm_solve(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol))
        self._leave(cur, lib)
        _check(rc, (BCM_OK, BCM_MAXIT, BCM_STAGNATED) if allow_maxit else (BCM_OK,))
        return x

    def precond(self, r):
        """z = B(r): one cycle of the preconditioner."""
        r = _dev(r, torch.float64, self.device)
        z = torch.empty(self.n, dtype=torch.float64, device=self.device)
        cur, lib = self._enter()
        rc = load_library().bcm_precond(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()))
        self._leave(cur, lib)
        _check(rc)
        return z

    def solve_adjoint(self, g, allow_maxit=False):
        g = _dev(g, torch.float64, self.device)
        lam = torch.empty(self.n, dtype=torch.float64, device=self.device)
        cur, lib = self._enter()
        rc = load_library().bcm_solve_adjoint(self.h, C.c_void_p(g.data_ptr()), C.c_void_p(lam.data_ptr()))
        self._leave(cur, lib)
        _check(rc, (BCM_OK, BCM_MAXIT, BCM_STAGNATED) if allow_maxit else (BCM_OK,))
        return lam

    def sampled_outer(self, lam, x):
        lam = _dev(lam, torch.float64, self.device)
        x = _dev(x, torch.float64, self.device)
        out = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        cur, lib = self._enter()
        rc = load_library().bcm_sampled_outer(self.h, C.c_void_p(lam.data_ptr()), C.c_void_p(x.data_ptr()),
                                              C.c_void_p(out.data_ptr()))
        self._leave(cur, lib)
        _check(rc)
        return out

    def check_values(self, val):
        """Raises ValueError unless ``val`` holds exactly the values the
        hierarchy was built from (the solve uses the hierarchy's copy of A)."""
        v = val.detach() if isinstance(val, torch.Tensor) else torch.as_tensor(val)
        v = v.to(device=self.device, dtype=torch.float64)
        if v.numel() != self.nnz or not torch.equal(v.reshape(-1), self.val):
            raise ValueError("val differs from the matrix values this Hierarchy was built from: "
                             "build a new Hierarchy for the new values")

    def info(self) -> dict:
        i = BcmInfo()
        _check(load_library().bcm_info(self.h, C.byref(i)))
        nl = i.nl
        return dict(nl=nl, n=list(i.n[:nl]), nnz=list(i.nnz[:nl]), vcmplx=i.vcmplx, cratio=i.cratio,
                    cratio_nl=i.cratio_nl, iters=i.iters, status=i.status, relres=i.relres,
                    t_setup_ms=i.t_setup_ms, t_solve_ms=i.t_solve_ms, cycle_bytes=i.cycle_bytes,
                    iter_bytes=i.iter_bytes, precision=i.precision, setup_bytes=i.setup_bytes,
                    sweeps_run=i.sweeps_run, long_rows=i.long_rows)

    def level(self, k: int) -> dict:
        """Level k copied to host numpy arrays."""
        import numpy as np
        inf = self.info()
        n, nnz = inf["n"][k], inf["nnz"][k]
        out = dict(n=n, nnz=nnz, rowptr=np.empty(n + 1, np.int32), col=np.empty(nnz, np.int32),
                   val=np.empty(nnz), w=np.empty(n), dinv=np.empty(n))
        last = k == inf["nl"] - 1
        agg = None if last else np.empty(n, np.int32)
        p = None if last else np.empty(n)
        ptr = lambda a: C.c_void_p(a.ctypes.data) if a is not None else None
        _check(load_library().bcm_level_copy(self.h, k, ptr(out["rowptr"]), ptr(out["col"]), ptr(out["val"]),
                                             ptr(out["w"]), ptr(out["dinv"]), ptr(agg), ptr(p)))
        if not last:
            out["agg"], out["p"] = agg, p
        return out

    def profile(self, kclass: str):
        launches, ms, nbytes = C.c_int64(), C.c_double(), C.c_double()
        _check(load_library().bcm_profile(self.h, PROF[kclass], C.byref(launches), C.byref(ms), C.byref(nbytes)))
        return launches.value, ms.value, nbytes.value


def match(rowptr, col, val, w=None, check=True, device=None, noalloc=False, weights=True):
    """One matching sweep on the GPU: returns (mate int32[n], weights float64[nnz]
    or None when weights=False).  noalloc=True calls bcm_match_noalloc, whose
    scratch is the library's static device array (no allocation inside the
    call; calls on one GPU must not overlap)."""
    L = _gpu_lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    rp, ci, va = _dev(rowptr, torch.int32, device), _dev(col, torch.int32, device), _dev(val, torch.float64, device)
    n = rp.numel() - 1
    w = torch.ones(n, dtype=torch.float64, device=device) if w is None else _dev(w, torch.float64, device)
    stream = torch.cuda.current_stream(device).cuda_stream
    alloc = None if noalloc else _TorchAllocator(device, stream)
    p = make_params(check=check, stream=stream, allocator=alloc)
    mate = torch.empty(n, dtype=torch.int32, device=device)
    c = torch.empty(ci.numel(), dtype=torch.float64, device=device) if weights else None
    A = BcmCsr(n, ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    fn = L.bcm_match_noalloc if noalloc else L.bcm_match
    _check(fn(C.byref(A), C.c_void_p(w.data_ptr()), C.byref(p), C.c_void_p(mate.data_ptr()),
              C.c_void_p(c.data_ptr() if c is not None else None)))
    return mate, c


class BcmSolve(torch.autograd.Function):
    """x = A^{-1} b through the GPU hierarchy, differentiable in the stored
    values of A and in b.  Backward solves A lambda = dL/dx with the same
    hierarchy (A symmetric) and returns dL/db = lambda and
    dL/da_ij = -lambda_i x_j on A's pattern.  ``val`` must hold the values the
    hierarchy was built from: forward compares them with the hierarchy's copy
    and raises ValueError when they differ (after an optimiser step, build a
    new Hierarchy).  With save_x=False the solution is recomputed in backward
    instead of being kept."""

    @staticmethod
    def forward(ctx, val, b, hier: Hierarchy, tol: float = 1e-10, save_x: bool = True):
        hier.check_values(val)
        x = hier.solve(b, tol=tol)
        ctx.hier, ctx.tol, ctx.save_x = hier, tol, save_x
        if save_x:
            ctx.save_for_backward(x)
        else:
            ctx.save_for_backward(b.detach())
        return x

    @staticmethod
    def backward(ctx, gx):
        hier = ctx.hier
        (saved,) = ctx.saved_tensors
        x = saved if ctx.save_x else hier.solve(saved, tol=ctx.tol)
        lam = hier.solve_adjoint(gx)
        gval = hier.sampled_outer(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gval, gb, None, None, None


def solve(val, b, hier: Hierarchy, tol: float = 1e-10, save_x: bool = True):
    return BcmSolve.apply(val, b, hier, tol, save_x)
