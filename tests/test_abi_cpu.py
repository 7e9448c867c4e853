"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/gpr.h declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

from paper_2602_19683_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gpr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), f"libgpr.so does not export {name}"
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_abi_version_and_strerror():
    lib = _lib.load()
    assert lib.gpr_abi_version() == 10
    for code in [0, 1, -1, -2, -3, -4, -5]:
        assert lib.gpr_strerror(code)
    assert b"unknown" in lib.gpr_strerror(12345)


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-GPU path")
def test_ctx_create_reports_no_device():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.gpr_ctx_create(ctypes.byref(h), 0, 2, 0) == _lib.GPR_ENODEV
    assert not h.value


def test_host_argument_validation():
    lib = _lib.load()
    H = _lib.Hyper(1.0, 1.0, 0.1)
    h = ctypes.c_void_p()
    assert lib.gpr_ctx_create(None, 0, 2, 0) == _lib.GPR_EINVAL
    assert lib.gpr_ctx_create(ctypes.byref(h), 0, 0, 0) == _lib.GPR_EINVAL
    assert lib.gpr_ctx_create(ctypes.byref(h), 0, 2, 7) == _lib.GPR_EINVAL
    # null context / pointers, bad sizes, bad tile, bad hyperparameters
    assert lib.gpr_assemble(None, None, 10, 8, H, 32, ctypes.byref(h), None) == _lib.GPR_EINVAL
    assert lib.gpr_cholesky(None, None, 0, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_cholesky_dense(None, None, 10, 32, 0, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_predict(None, None, None, None, 10, None, 5, 8, H, None, None, None,
                           None) == _lib.GPR_EINVAL
    assert lib.gpr_nlml_grad(None, None, None, 10, 8, H, 32, 0, None, None, None,
                             None) == _lib.GPR_EINVAL
    assert lib.gpr_solve(None, None, None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_solve_noalloc(None, None, None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_fit_predict(None, None, None, 10, None, 5, 8, H, 32, 0, None, None, None,
                               None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_predict_var(None, None, None, None, 10, None, 5, 8, H, None, None, None, None,
                               None) == _lib.GPR_EINVAL
    assert lib.gpr_fit_predict_var(None, None, None, 10, None, 5, 8, H, 32, 0, None, None, None,
                                   None, None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_tiled_info(None, None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_tiled_to_dense(None, None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_tiled_free(None) == _lib.GPR_EINVAL
    assert lib.gpr_sync(None, None, None) == _lib.GPR_EINVAL
    assert lib.gpr_profile_enable(None, 1) == _lib.GPR_EINVAL
    assert lib.gpr_profile_read(None, 0, None, None, None, None, 0) == _lib.GPR_EINVAL
    assert lib.gpr_ctx_destroy(None) == _lib.GPR_EINVAL


def test_schedule_describe_argument_errors():
    lib = _lib.load()
    nt, nl = ctypes.c_int64(), ctypes.c_int64()
    assert lib.gpr_schedule_describe(0, 0, 0, None, 0, ctypes.byref(nt), None, 0,
                                     ctypes.byref(nl)) == _lib.GPR_EINVAL
    assert lib.gpr_schedule_describe(4, 0, 1, None, 0, ctypes.byref(nt), None, 0,
                                     ctypes.byref(nl)) == _lib.GPR_EINVAL
    # too-small capacity: counts are still reported
    assert lib.gpr_schedule_describe(4, 0, 0, None, 0, ctypes.byref(nt), None, 0,
                                     ctypes.byref(nl)) == _lib.GPR_EINVAL
    assert nt.value == 4 + 6 + 6 + 4


def test_adjoint_describe_argument_errors():
    lib = _lib.load()
    nt, nr, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.gpr_adjoint_describe(0, 2, None, 0, ctypes.byref(nt), None, 0, ctypes.byref(nr),
                                    None, 0, ctypes.byref(nl)) == _lib.GPR_EINVAL
    assert lib.gpr_adjoint_describe(4, 0, None, 0, ctypes.byref(nt), None, 0, ctypes.byref(nr),
                                    None, 0, ctypes.byref(nl)) == _lib.GPR_EINVAL
    # too-small capacity: counts are still reported
    assert lib.gpr_adjoint_describe(1, 2, None, 0, ctypes.byref(nt), None, 0, ctypes.byref(nr),
                                    None, 0, ctypes.byref(nl)) == _lib.GPR_EINVAL
    assert (nt.value, nr.value, nl.value) == (3, 3, 3)  # M = 1: the three POTRF-adjoint products


def test_fit_hyper_rejects_bad_arguments():
    import ctypes
    from paper_2602_19683_amd import _lib
    lib = _lib.load()
    th = (ctypes.c_double * 3)(0.3, 2.0, 0.5)
    out = (ctypes.c_double * 3)()
    # no context
    assert lib.gpr_fit_hyper(None, None, None, 8, 1, 32, th, 5, 0.05, 0.9, 0.999, 1e-8, 0.0,
                             out, None, None, None) == -1
