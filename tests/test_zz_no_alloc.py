"""gpr_solve_noalloc (the solve for callers that cannot allocate device
memory) against gpr_solve, through the C ABI: bitwise equal on two calls in
a row, the second with a smaller problem (so the fixed work array still holds
the first call's longer vectors), and within 1e-10 of the oracle's
alpha = K^{-1} y."""
import ctypes

import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir_train_test

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


@pytest.mark.timeout(300)
def test_solve_noalloc_matches_solve_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19683_amd import Context, _lib
    lib = _lib.load()
    X, y, _ = nfir_train_test(3000, 16)
    with Context(0) as ctx:
        for n, tile in ((3000, 256), (1000, 128)):
            say(f"gpr_solve_noalloc vs gpr_solve: n={n} tile={tile}")
            Xd, yd = dev(X[:n]), dev(y[:n])
            K = ctx.assemble(Xd, DEFAULT_HYPER, tile)
            ctx.cholesky(K)
            x_ref = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
            x_new = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            h = ctx._h
            rc = lib.gpr_solve(h, K.handle, ctypes.c_void_p(yd.data_ptr()),
                               ctypes.c_void_p(x_ref.data_ptr()), None)
            assert rc == _lib.GPR_OK
            rc = lib.gpr_solve_noalloc(h, K.handle, ctypes.c_void_p(yd.data_ptr()),
                                       ctypes.c_void_p(x_new.data_ptr()), None)
            assert rc == _lib.GPR_OK
            assert ctx.sync()[0] == 0
            a_ref, a_new = x_ref.cpu().numpy(), x_new.cpu().numpy()
            np.testing.assert_array_equal(a_new, a_ref)
            ref = oracle.predict(X[:n], y[:n], X[:1], DEFAULT_HYPER, want=("alpha",))
            e = oracle.rel_err(a_new, ref["alpha"])
            say(f"  bitwise equal; rel(alpha) vs oracle = {e:.3e}")
            assert e <= 1e-10
            K.free()
