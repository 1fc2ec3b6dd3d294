"""The C ABI library loads without a GPU, exports every function that
include/bcm.h declares, and the Python binding's struct layouts match the C
compiler's (no compute call is made here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bcm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1810_04221_amd import bcm
    if not os.path.exists(bcm.LIB_PATH):
        from paper_1810_04221_amd import build
        build.build()
    return bcm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    from paper_1810_04221_amd import bcm
    assert sorted(bcm.EXPORTS) == names


def test_default_params_and_error_string(lib):
    from paper_1810_04221_amd import bcm
    p = bcm.BcmParams()
    lib.bcm_default_params(C.byref(p))
    assert (p.max_levels, p.max_coarse, p.sweeps, p.coarse_sweeps, p.pre, p.post) == (40, 0, 2, 20, 1, 1)
    assert (p.itmax, p.precision, p.check) == (5000, bcm.BCM_FP64, 1)
    assert (p.cycle, p.kcycle_levels, p.graph, p.group, p.sell, p.min_ratio, p.fold) == (1, 0, 0, 0, 1, 0.0, 1)
    assert lib.bcm_last_error() == b""


def test_null_arguments_rejected_without_gpu_work(lib):
    from paper_1810_04221_amd import bcm
    h = C.c_void_p()
    assert lib.bcm_setup(None, None, None, C.byref(h)) == bcm.BCM_EINVAL
    assert b"NULL" in lib.bcm_last_error()
    assert lib.bcm_solve(None, None, None, 1e-8) == bcm.BCM_EINVAL
    assert lib.bcm_precond(None, None, None) == bcm.BCM_EINVAL
    assert lib.bcm_solve_adjoint(None, None, None) == bcm.BCM_EINVAL
    assert lib.bcm_sampled_outer(None, None, None, None) == bcm.BCM_EINVAL
    lib.bcm_free(None)


@pytest.mark.parametrize("field,value", [("group", 3), ("group", 128), ("cycle", 4), ("cycle", 0),
                                         ("kcycle_levels", -1), ("sweeps", 5), ("precision", 2)])
def test_unsupported_parameters_rejected_before_gpu_work(lib, field, value):
    # parameter checks run before any HIP call: the pointers are never touched
    from paper_1810_04221_amd import bcm
    p = bcm.BcmParams()
    lib.bcm_default_params(C.byref(p))
    setattr(p, field, value)
    A = bcm.BcmCsr(4, 4, 8, 8, 8)  # dummy non-null device addresses, never dereferenced
    h = C.c_void_p()
    assert lib.bcm_setup(C.byref(A), C.c_void_p(8), C.byref(p), C.byref(h)) == bcm.BCM_EINVAL
    assert b"unsupported parameters" in lib.bcm_last_error()
    assert not h.value


def test_struct_layouts_match_c(tmp_path):
    from paper_1810_04221_amd import bcm
    probe = tmp_path / "probe.c"
    probe.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "bcm.h"\n'
        "int main(void){\n"
        + "".join(f'printf("%zu ", offsetof(bcm_params, {f}));\n' for f, _ in bcm.BcmParams._fields_)
        + 'printf("\\n");\n'
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(bcm_params), offsetof(bcm_params, adjoint_tol),'
        " offsetof(bcm_params, alloc), offsetof(bcm_params, stream), sizeof(bcm_csr));\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(bcm_info_t), offsetof(bcm_info_t, nnz),'
        " offsetof(bcm_info_t, vcmplx), offsetof(bcm_info_t, iter_bytes), offsetof(bcm_info_t, setup_bytes),"
        " offsetof(bcm_info_t, long_rows));\n"
        "return 0;}\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    f, a, b = subprocess.check_output([str(exe)]).decode().split("\n")[:3]
    P, I = bcm.BcmParams, bcm.BcmInfo
    assert [int(t) for t in f.split()] == [getattr(P, name).offset for name, _ in P._fields_]
    assert [int(t) for t in a.split()] == [C.sizeof(P), P.adjoint_tol.offset, P.alloc.offset, P.stream.offset,
                                           C.sizeof(bcm.BcmCsr)]
    assert [int(t) for t in b.split()] == [C.sizeof(I), I.nnz.offset, I.vcmplx.offset, I.iter_bytes.offset,
                                           I.setup_bytes.offset, I.long_rows.offset]

