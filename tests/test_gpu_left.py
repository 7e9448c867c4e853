"""The left-looking variant of the tiled Cholesky (Sec. 4.2) on the GPU,
through the C ABI, against the oracle (FP64: normwise 1e-10; L, the mean,
the covariance, the variances, alpha and the NLML with its gradient), and
against the right-looking order of the same library (equal up to rounding).

The sizes make every code path run: multi-term update tasks, tasks split
along k into parts that a second kernel adds in order (tiles of 256 and 512,
where a bulk launch has few 128 x 128 blocks), the fused POTRF + TRSM and
SYRK launches of the critical stream, test rows and the test block, a
ragged n, and the mixed precisions (mean within 1e-8 after refinement)."""
import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir_train_test

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19683_amd import Context
    left = Context(0, variant="left")
    right = Context(0)
    yield left, right
    left.close()
    right.close()


@pytest.mark.parametrize("n,tile", [(1000, 128), (4096, 256), (4096, 512), (3000, 256),
                                    (2048, 64), (640, 32)])
def test_left_cholesky_matches_oracle(ctxs, n, tile):
    left, right = ctxs
    say(f"left-looking cholesky n={n} tile={tile}")
    X, y, _ = nfir_train_test(n, 8)
    Xd = dev(X)
    K = left.assemble(Xd, DEFAULT_HYPER, tile)
    left.cholesky(K)
    assert left.sync()[0] == 0
    L = host(left.to_dense(K))
    K2 = right.assemble(Xd, DEFAULT_HYPER, tile)
    right.cholesky(K2)
    assert right.sync()[0] == 0
    L2 = host(right.to_dense(K2))
    Lref, _ = oracle.cholesky(oracle.assemble_K(X, DEFAULT_HYPER))
    e, e2 = oracle.rel_err_lower(L, Lref), oracle.rel_err_lower(L, L2)
    say(f"  rel(L) vs oracle {e:.3e}, vs right-looking {e2:.3e}")
    np.testing.assert_array_equal(np.triu(L, 1), 0.0)
    assert e <= TOL and e2 <= 1e-12
    # the solve with the left-looking factor
    alpha = host(left.solve(K, dev(y)))
    ref = oracle.predict(X, y, X[:1], DEFAULT_HYPER, want=("alpha",))
    assert oracle.rel_err(alpha, ref["alpha"]) <= TOL
    K.free()
    K2.free()


@pytest.mark.parametrize("n,ns,tile", [(4096, 1024, 256), (4096, 1024, 512), (2500, 700, 128),
                                       (128, 128, 32)])
def test_left_fit_predict_matches_oracle(ctxs, n, ns, tile):
    left, _ = ctxs
    say(f"left-looking fit_predict n={n} n_test={ns} tile={tile}")
    X, y, Xs = nfir_train_test(n, ns)
    mean, cov, K = left.fit_predict(dev(X), dev(y), dev(Xs), DEFAULT_HYPER, tile, "fp64")
    assert left.sync()[0] == 0
    mean, cov = host(mean), host(cov)
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER, want=("mean", "cov"))
    em, ec = oracle.rel_err(mean, ref["mean"]), oracle.rel_err(cov, ref["cov"])
    say(f"  rel(mean) {em:.3e}, rel(cov) {ec:.3e}")
    np.testing.assert_array_equal(cov, cov.T)
    assert em <= TOL and ec <= TOL and oracle.max_rel(cov, ref["cov"]) <= TOL
    # the covariance rows with the given factor (left-looking solve of V)
    mean2, cov2 = left.predict(K, dev(X), dev(y), dev(Xs), DEFAULT_HYPER)
    assert left.sync()[0] == 0
    assert oracle.rel_err(host(cov2), ref["cov"]) <= TOL
    assert oracle.rel_err(host(mean2), ref["mean"]) <= TOL
    K.free()


@pytest.mark.parametrize("fused", [True, False])
def test_left_variances(ctxs, fused):
    left, _ = ctxs
    n, ns, tile = 3000, 600, 256
    say(f"left-looking variances fused={fused}")
    X, y, Xs = nfir_train_test(n, ns)
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER, want=("mean", "cov"))
    if fused:
        mean, var, _, K = left.fit_predict_var(dev(X), dev(y), dev(Xs), DEFAULT_HYPER, tile,
                                               "fp64")
    else:
        K = left.assemble(dev(X), DEFAULT_HYPER, tile)
        left.cholesky(K)
        mean, var = left.predict_var(K, dev(X), dev(y), dev(Xs), DEFAULT_HYPER)[:2]
    assert left.sync()[0] == 0
    ev = oracle.rel_err(host(var), np.diag(ref["cov"]))
    say(f"  rel(var) {ev:.3e}")
    assert ev <= TOL and oracle.rel_err(host(mean), ref["mean"]) <= TOL
    K.free()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_left_mixed_mean(ctxs, precision):
    left, _ = ctxs
    n, ns, tile = 4096, 512, 256
    say(f"left-looking mixed {precision} n={n} tile={tile}")
    X, y, Xs = nfir_train_test(n, ns)
    mean, cov, K, ir = left.fit_predict(dev(X), dev(y), dev(Xs), DEFAULT_HYPER, tile, precision,
                                        ir_stats=True)
    assert left.sync()[0] == 0
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER, want=("mean", "cov"))
    em, ec = oracle.rel_err(host(mean), ref["mean"]), oracle.rel_err(host(cov), ref["cov"])
    say(f"  {ir}, rel(mean) {em:.3e}, rel(cov) {ec:.3e}")
    assert em <= 1e-8
    K.free()


def test_left_nlml_grad(ctxs):
    left, _ = ctxs
    n, tile, h = 2048, 256, (0.3, 2.0, 0.5)
    say(f"left-looking nlml_grad n={n} tile={tile}")
    X, y, _ = nfir_train_test(n, 8)
    nl, g, _ = left.nlml_grad(dev(X), dev(y), h, tile)
    left.sync()
    nl_ref, g_ref = oracle.nlml_grad(X, y, h)
    enl = abs(float(host(nl)[0]) - nl_ref) / abs(nl_ref)
    eg = oracle.rel_err(host(g), g_ref)
    say(f"  rel(nlml) {enl:.3e}, rel(grad) {eg:.3e}")
    assert enl <= 1e-12 and eg <= 1e-9


def test_left_persistent_context_runs_on_streams(ctxs):
    """A persistent-executor context runs left-looking sweeps on the streams:
    bitwise the left-looking result of a stream context."""
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, Context
    left, _ = ctxs
    n, ns, tile = 2048, 512, 256
    X, y, Xs = nfir_train_test(n, ns)
    m1, c1, K1 = left.fit_predict(dev(X), dev(y), dev(Xs), DEFAULT_HYPER, tile, "fp64")
    with Context(0, executor=GPR_EXEC_PERSISTENT, variant="left") as p:
        m2, c2, K2 = p.fit_predict(dev(X), dev(y), dev(Xs), DEFAULT_HYPER, tile, "fp64")
        assert p.sync()[0] == 0
        np.testing.assert_array_equal(host(c2), host(c1))
        np.testing.assert_array_equal(host(m2), host(m1))
        K2.free()
    K1.free()
