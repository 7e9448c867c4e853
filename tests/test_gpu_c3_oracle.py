"""The benchmarked configuration against the oracle, element by element.

n = 16384 training points, n_test = 4096, D = 8, tile 512, FP64, through the
fused call the benchmark times (gpr_fit_predict: assembly, factorisation and
covariance rows in one sweep), on both executors, and in the left-looking
task order. The oracle computes the
plain definitions (Sec. 4.1, eqs. (1)-(3)) on the host cores once for the
module (about a minute on 16 cores, about 6 GB of host memory).

Compared, with the normwise reading of the 1e-10 bar (Frobenius over the
lower triangle for L, 2-norm for alpha and the mean, Frobenius for the
covariance; max|A - B| / max|B| also asserted for the covariance):
  L, alpha = K^{-1} y (through gpr_solve with the fused call's factor),
  the mean and the full covariance.
"""
import time

import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir_train_test

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N, NS, D, TILE = 16384, 4096, 8, 512
TOL = 1e-10


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X, y, Xs = nfir_train_test(N, NS, D)
    say(f"oracle predict n={N} n_test={NS} D={D} (host cores)")
    t = time.perf_counter()
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER, want=("L", "alpha", "mean", "cov"))
    say(f"  oracle done in {time.perf_counter() - t:.1f} s")
    return X, y, Xs, ref


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("executor", ["streams", "persistent", "streams-left"])
def test_c3_fused_fp64_matches_oracle(data, executor):
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, GPR_EXEC_STREAMS, Context
    X, y, Xs, ref = data
    say(f"gpr_fit_predict fp64 n={N} n_test={NS} tile={TILE} executor={executor}")
    ex = GPR_EXEC_PERSISTENT if executor == "persistent" else GPR_EXEC_STREAMS
    variant = "left" if executor.endswith("left") else "right"
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    with Context(0, executor=ex, variant=variant) as ctx:
        Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
        mean_d, cov_d, K = ctx.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, TILE, "fp64", info=info)
        assert ctx.sync()[0] == 0 and int(info.item()) == 0
        mean, cov = host(mean_d), host(cov_d)
        del cov_d
        alpha = host(ctx.solve(K, yd))
        Ld = ctx.to_dense(K)
        L = host(Ld)
        del Ld
        K.free()
    torch.cuda.empty_cache()
    np.testing.assert_array_equal(np.triu(L, 1), 0.0)
    np.testing.assert_array_equal(cov, cov.T)
    errs = {
        "rel(L)": oracle.rel_err_lower(L, ref["L"]),
        "rel(alpha)": oracle.rel_err(alpha, ref["alpha"]),
        "rel(mean)": oracle.rel_err(mean, ref["mean"]),
        "rel(cov)": oracle.rel_err(cov, ref["cov"]),
        "maxrel(cov)": oracle.max_rel(cov, ref["cov"]),
    }
    say("  " + "  ".join(f"{k} = {v:.3e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL, f"{k} = {v:.3e} above {TOL}"
