"""Predictive variances (the diagonal of eq. (3)) through gpr_fit_predict_var /
gpr_predict_var, against the oracle and against the full covariance.

* var only (no covariance): the sweep forms V^T and skips the test block;
  var_i = v - ||V^T_i||^2. Normwise relative error <= 1e-10 against the
  diagonal of the oracle's covariance; mean bitwise equal to the full path.
* var with the covariance: var is the diagonal of cov, bit for bit, and cov
  equals gpr_fit_predict's.
* given factor (gpr_predict_var) equals the fused call bitwise; the
  persistent executor equals the streams bitwise.
* n = 16384, n_test = 4096, tile 512: var only against the diagonal of the
  full covariance (two routes: row sums of squares of V^T, and the diagonal
  of K_** - V^T V accumulated tile by tile), and 0 <= var <= v.
"""
import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir_train_test

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19683_amd import GPR_EXEC_PERSISTENT, Context
    s = Context(0)
    p = Context(0, executor=GPR_EXEC_PERSISTENT)
    yield s, p
    p.close()
    s.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n,ns,tile,h", [(128, 128, 32, DEFAULT_HYPER), (70, 5, 32, DEFAULT_HYPER),
                                         (1000, 300, 128, (0.3, 2.0, 0.5)),
                                         (512, 512, 128, (2.0, 0.7, 0.01)),
                                         (777, 333, 96, DEFAULT_HYPER)])
def test_variance_matches_oracle(ctxs, n, ns, tile, h):
    say(f"variance n={n} n_test={ns} tile={tile} h={h}")
    s, p = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    mean, var, cov, K = s.fit_predict_var(Xd, yd, Xsd, h, tile)
    assert cov is None
    m1, v1 = host(mean), host(var)
    assert s.sync()[0] == 0
    ref = oracle.predict(X, y, Xs, h)
    ev = oracle.rel_err(v1, np.diag(ref["cov"]))
    em = oracle.rel_err(m1, ref["mean"])
    say(f"  rel(var) {ev:.3e} rel(mean) {em:.3e}")
    assert ev <= TOL and em <= TOL
    # given factor: the same bits
    m2, v2, c2 = s.predict_var(K, Xd, yd, Xsd, h)
    np.testing.assert_array_equal(host(m2), m1)
    np.testing.assert_array_equal(host(v2), v1)
    # with the covariance: var is its diagonal; mean and cov as gpr_fit_predict
    m3, v3, c3, K3 = s.fit_predict_var(Xd, yd, Xsd, h, tile, full_cov=True)
    c3 = host(c3)
    np.testing.assert_array_equal(host(v3), np.diag(c3))
    np.testing.assert_array_equal(host(m3), m1)
    m4, c4, K4 = s.fit_predict(Xd, yd, Xsd, h, tile)
    np.testing.assert_array_equal(host(c4), c3)
    # persistent executor, variances only: the same bits as the streams
    mp, vp, _, Kp = p.fit_predict_var(Xd, yd, Xsd, h, tile)
    np.testing.assert_array_equal(host(vp), v1)
    np.testing.assert_array_equal(host(mp), m1)
    assert s.sync()[0] == 0 and p.sync()[0] == 0
    for k in (K, K3, K4, Kp):
        k.free()


def test_variance_full_size(ctxs):
    n, ns, tile = 16384, 4096, 512
    say(f"variance full size n={n} n_test={ns} tile={tile}")
    s, _ = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    mean, var, _, K = s.fit_predict_var(Xd, yd, Xsd, DEFAULT_HYPER, tile)
    v1, m1 = host(var), host(mean)
    m2, v2, c2, K2 = s.fit_predict_var(Xd, yd, Xsd, DEFAULT_HYPER, tile, full_cov=True)
    d = host(v2)
    assert s.sync()[0] == 0
    e = oracle.rel_err(v1, d)
    say(f"  rel(var only vs diag of the covariance) {e:.3e}; var in [{v1.min():.3e}, {v1.max():.3e}]")
    assert e <= TOL
    np.testing.assert_array_equal(host(m2), m1)
    v = DEFAULT_HYPER[1]
    assert v1.min() >= -1e-12 * v and v1.max() <= v * (1 + 1e-12)
    K.free()
    K2.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_variance_mixed(ctxs, prec):
    """Mixed-precision updates with the variances only: the mean meets the
    mixed bar (1e-8) against the oracle after refinement, the variances carry
    the error of the low-precision V^T (stated, not pinned; bounded loosely),
    and with the covariance as well, var is its diagonal bit for bit."""
    n, ns, tile = 4000, 500, 256
    say(f"variance mixed {prec} n={n} n_test={ns} tile={tile}")
    s, _ = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER)
    mean, var, _, K, st = s.fit_predict_var(Xd, yd, Xsd, DEFAULT_HYPER, tile, precision=prec,
                                            ir_stats=True)
    em = oracle.rel_err(host(mean), ref["mean"])
    ev = oracle.rel_err(host(var), np.diag(ref["cov"]))
    say(f"  refinement {st['iters']} ({st['method']}), precision used {st['precision']}; "
        f"rel(mean) {em:.2e} rel(var) {ev:.2e}")
    assert em <= 1e-8
    assert ev <= (1e-3 if st["precision"] == 1 else 1e-1)
    m2, v2, c2, K2 = s.fit_predict_var(Xd, yd, Xsd, DEFAULT_HYPER, tile, precision=prec,
                                       full_cov=True)
    np.testing.assert_array_equal(host(v2), np.diag(host(c2)))
    assert s.sync()[0] == 0
    K.free()
    K2.free()
