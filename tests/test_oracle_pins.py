"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, never against the oracle itself.

* closed forms of eq. (1) (Sec. 4.1) at hand-chosen points;
* LAPACK (numpy/scipy) where a step reduces to a library routine;
* 50-digit mpmath brute force of eqs. (2)-(3) at tiny n;
* Gauss-Jordan inversion (an independent route) at n <= 64;
* exact identities of GP regression (test set equal to training set,
  noise -> 0, far field), symmetry and positive semi-definiteness;
* closed forms of the negative log marginal likelihood at n = 1 and 2,
  finite differences and torch autograd for its gradient.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir, nfir_train_test, random_spd

U = np.finfo(np.float64).eps / 2  # unit roundoff


# --------------------------------------------------------------------------
# Input generator
# --------------------------------------------------------------------------

def test_generator_shapes_and_lags():
    X, y = nfir(100, 8, seed=0)
    assert X.shape == (100, 8) and y.shape == (100,)
    assert X.flags.c_contiguous and X.dtype == np.float64
    # each row is the previous one shifted by one lag (newest force first)
    np.testing.assert_array_equal(X[1:, 1:], X[:-1, :-1])
    assert np.all(np.abs(X) <= 1.0)
    X2, y2 = nfir(100, 8, seed=0)
    np.testing.assert_array_equal(X, X2)
    np.testing.assert_array_equal(y, y2)
    X3, _ = nfir(100, 8, seed=1)
    assert not np.array_equal(X, X3)


def test_generator_noise_level():
    X, y = nfir(20000, 8, seed=0)
    resid = y - np.tanh(X @ (0.5 ** np.arange(8)))
    assert abs(resid.std() - 0.1) < 0.005       # N(0, 0.01) read as a variance
    assert abs(resid.mean()) < 0.005


# --------------------------------------------------------------------------
# Assembly, eq. (1)
# --------------------------------------------------------------------------

def test_kernel_closed_form_points():
    # a = 0, b = e_0 + 2 e_3: squared distance 1 + 4 = 5 exactly.
    a = np.zeros((1, 8))
    b = np.zeros((1, 8))
    b[0, 0], b[0, 3] = 1.0, 2.0
    for (l, v) in [(0.5, 2.0), (1.0, 1.0), (0.3, 1.7), (2.5, 0.25)]:
        k = oracle.kernel_matrix(a, b, (l, v, 0.1))[0, 0]
        exact = float(mpmath.mpf(v) * mpmath.exp(-mpmath.mpf(5) / (2 * mpmath.mpf(l))))
        assert abs(k - exact) <= 2 * U * exact
    # s = 1, l = 0.3: v e^{-1/0.6}
    b2 = np.zeros((1, 8)); b2[0, 7] = 1.0
    k = oracle.kernel_matrix(a, b2, (0.3, 1.0, 0.1))[0, 0]
    assert abs(k - math.exp(-1 / 0.6)) <= 2 * U


def test_kernel_matrix_structure():
    X, _ = nfir(97, 8)
    l, v, s2 = 0.7, 1.3, 0.05
    K = oracle.assemble_K(X, (l, v, s2))
    np.testing.assert_array_equal(K, K.T)                     # exact symmetry
    np.testing.assert_allclose(np.diag(K), v + s2, rtol=0, atol=0)
    off = K[~np.eye(97, dtype=bool)]
    assert np.all(off > 0) and np.all(off <= v)
    # cross and test covariances carry no noise (index delta on training set only)
    Kc = oracle.kernel_matrix(X, X, (l, v, s2))
    np.testing.assert_allclose(np.diag(Kc), v, rtol=0, atol=0)
    np.testing.assert_allclose(Kc + s2 * np.eye(97), K, rtol=2 * U, atol=0)


def test_kernel_vs_numpy_definition():
    X, _ = nfir(50, 8, seed=3)
    Xs, _ = nfir(30, 8, seed=4)
    l, v = 0.4, 2.0
    s = ((Xs[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    np.testing.assert_allclose(oracle.kernel_matrix(Xs, X, (l, v, 0.1)),
                               v * np.exp(-s / (2 * l)), rtol=1e-14, atol=0)


def test_far_field_underflows_to_zero():
    X, _ = nfir(16, 8)
    Kc = oracle.kernel_matrix(X + 100.0, X, (1.0, 1.0, 0.1))
    assert np.all(Kc == 0.0)


# --------------------------------------------------------------------------
# Cholesky and substitutions (library special cases, backward stability)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 129])
def test_cholesky_vs_lapack(n):
    A = random_spd(n, seed=n)
    L, info = oracle.cholesky(A)
    assert info == 0
    np.testing.assert_array_equal(np.triu(L, 1), 0)
    assert np.all(np.diag(L) > 0)
    Lref = np.linalg.cholesky(A)
    assert oracle.rel_err(L, Lref) <= 50 * n * U
    assert np.linalg.norm(L @ L.T - A) <= 4 * n * U * np.linalg.norm(A)


def test_cholesky_2x2_closed_form():
    a, b, c = 4.0, 2.0, 5.0
    L, info = oracle.cholesky(np.array([[a, b], [b, c]]))
    assert info == 0
    np.testing.assert_allclose(L, [[2.0, 0.0], [1.0, 2.0]], rtol=0, atol=0)


def test_cholesky_backward_error_nfir():
    X, _ = nfir(300, 8)
    K = oracle.assemble_K(X, DEFAULT_HYPER)
    L, info = oracle.cholesky(K)
    assert info == 0
    assert np.linalg.norm(L @ L.T - K) / np.linalg.norm(K) <= 300 * U


def test_cholesky_failure_column():
    A = np.diag([1.0, 2.0, -1.0, 4.0])
    _, info = oracle.cholesky(A)
    assert info == 3
    X, _ = nfir(10, 8)
    K = oracle.assemble_K(X, (1.0, 1.0, -2.0))   # diagonal v + s2 = -1
    _, info = oracle.cholesky(K)
    assert info == 1


def test_substitutions_vs_scipy():
    n = 80
    A = random_spd(n, seed=5)
    L = np.linalg.cholesky(A)
    b = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_allclose(oracle.forward(L, b),
                               scipy.linalg.solve_triangular(L, b, lower=True),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.backward(L, b),
                               scipy.linalg.solve_triangular(L, b, lower=True, trans="T"),
                               rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# Independent routes for eqs. (2)-(3)
# --------------------------------------------------------------------------

def test_gauss_jordan_vs_numpy_inverse():
    A = random_spd(40, seed=2)
    Ai = oracle.gauss_jordan_inverse(A)
    np.testing.assert_allclose(Ai, np.linalg.inv(A), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(A @ Ai, np.eye(40), atol=1e-12)
    # with pivoting it also inverts a non-symmetric matrix needing row swaps
    B = np.array([[0.0, 1.0, 2.0], [1.0, 0.0, 3.0], [4.0, -3.0, 8.0]])
    np.testing.assert_allclose(oracle.gauss_jordan_inverse(B) @ B, np.eye(3), atol=1e-14)


@pytest.mark.parametrize("n,ns", [(4, 3), (8, 5), (64, 64)])
def test_predict_vs_gauss_jordan(n, ns):
    X, y, Xs = nfir_train_test(n, ns)
    h = (0.8, 1.2, 0.1)
    r = oracle.predict(X, y, Xs, h)
    g = oracle.predict_gauss_jordan(X, y, Xs, h)
    assert oracle.rel_err(r["alpha"], g["alpha"]) <= 1e-12
    assert oracle.rel_err(r["mean"], g["mean"]) <= 1e-12
    assert oracle.rel_err(r["cov"], g["cov"]) <= 1e-12


def _mp_predict(X, y, Xs, h, dps=50):
    """50-digit brute force of eqs. (1)-(3) through mpmath's own LU solver."""
    with mpmath.workdps(dps):
        return _mp_predict_body(X, y, Xs, h)


def _mp_predict_body(X, y, Xs, h):
    l, v, s2 = (mpmath.mpf(t) for t in h)
    n, D = X.shape
    ns = Xs.shape[0]

    def k(a, b):
        s = mpmath.fsum((mpmath.mpf(a[d]) - mpmath.mpf(b[d])) ** 2 for d in range(D))
        return v * mpmath.exp(-s / (2 * l))

    K = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            K[i, j] = k(X[i], X[j]) + (s2 if i == j else 0)
    Ks = mpmath.matrix(ns, n)
    for i in range(ns):
        for j in range(n):
            Ks[i, j] = k(Xs[i], X[j])
    Kss = mpmath.matrix(ns, ns)
    for i in range(ns):
        for j in range(ns):
            Kss[i, j] = k(Xs[i], Xs[j])
    alpha = mpmath.lu_solve(K, mpmath.matrix([mpmath.mpf(t) for t in y]))
    mean = Ks * alpha
    W = mpmath.matrix(n, ns)
    for c in range(ns):
        col = mpmath.lu_solve(K, Ks.T[:, c])
        for r in range(n):
            W[r, c] = col[r]
    cov = Kss - Ks * W
    to_np = lambda M: np.array([[float(M[i, j]) for j in range(M.cols)] for i in range(M.rows)])
    return {"alpha": to_np(alpha).ravel(), "mean": to_np(mean).ravel(), "cov": to_np(cov)}


@pytest.mark.parametrize("h", [(1.0, 1.0, 0.1), (0.3, 2.0, 0.5), (2.0, 0.7, 0.01)])
def test_predict_vs_mpmath_bruteforce(h):
    X, y, Xs = nfir_train_test(6, 4)
    r = oracle.predict(X, y, Xs, h)
    m = _mp_predict(X, y, Xs, h)
    assert oracle.rel_err(r["alpha"], m["alpha"]) <= 1e-12
    assert oracle.rel_err(r["mean"], m["mean"]) <= 1e-13
    assert oracle.rel_err(r["cov"], m["cov"]) <= 1e-13


# --------------------------------------------------------------------------
# Exact identities of GP regression
# --------------------------------------------------------------------------

def test_mean_identity_test_equals_train():
    # Xs = X: K_{X*,X} = K - s2 I, so y - mean = s2 alpha.
    X, y = nfir(150, 8)
    s2 = 0.1
    r = oracle.predict(X, y, X, (1.0, 1.0, s2))
    np.testing.assert_allclose(y - r["mean"], s2 * r["alpha"],
                               rtol=0, atol=1e-10 * np.abs(y).max())
    # mean = V^T beta with V solved from L V = K_{X,X*}
    Vt = np.stack([oracle.forward(r["L"], row)
                   for row in oracle.kernel_matrix(X, X, (1.0, 1.0, s2))])
    np.testing.assert_allclose(Vt @ r["beta"], r["mean"], rtol=1e-11, atol=1e-12)


def test_interpolation_as_noise_vanishes():
    X, y = nfir(40, 8)
    errs = []
    for s2 in [1e-2, 1e-4, 1e-6]:
        r = oracle.predict(X, y, X, (1.0, 1.0, s2))
        e = np.linalg.norm(r["mean"] - y)
        np.testing.assert_allclose(e, s2 * np.linalg.norm(r["alpha"]), rtol=1e-6)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4 * np.linalg.norm(y)


def test_cov_identity_test_equals_train():
    # Xs = X: Sigma = s2 I - s2^2 K^{-1}
    X, y = nfir(48, 8)
    s2 = 0.1
    h = (1.0, 1.0, s2)
    r = oracle.predict(X, y, X, h)
    Kinv = oracle.gauss_jordan_inverse(oracle.assemble_K(X, h))
    np.testing.assert_allclose(r["cov"], s2 * np.eye(48) - s2 * s2 * Kinv,
                               rtol=0, atol=1e-12)


def test_cov_structure():
    X, y, Xs = nfir_train_test(200, 120)
    h = (1.0, 1.0, 0.1)
    r = oracle.predict(X, y, Xs, h)
    S = r["cov"]
    np.testing.assert_array_equal(S, S.T)
    Kss = oracle.kernel_matrix(Xs, Xs, h)
    lam = np.linalg.eigvalsh(S)
    assert lam.min() >= -50 * U * np.linalg.norm(Kss, 2)
    d = np.diag(S)
    assert np.all(d >= 0) and np.all(d <= h[1])


def test_far_field_prediction():
    X, y = nfir(32, 8)
    Xs = X[:8] + 100.0
    h = (1.0, 1.0, 0.1)
    r = oracle.predict(X, y, Xs, h)
    assert np.all(r["mean"] == 0.0)
    np.testing.assert_array_equal(r["cov"], oracle.kernel_matrix(Xs, Xs, h))


def test_long_double_agreement():
    X, y, Xs = nfir_train_test(256, 64)
    h = (1.0, 1.0, 0.1)
    a = oracle.predict(X, y, Xs, h)
    b = oracle.predict(X, y, Xs, h, real="long double")
    assert oracle._lib("long double").orc_real_bytes() > 8
    assert oracle.rel_err_lower(a["L"], b["L"]) <= 1e-14
    assert oracle.rel_err(a["mean"], b["mean"]) <= 1e-12
    assert oracle.rel_err(a["cov"], b["cov"]) <= 1e-12


def test_predict_raises_on_not_pd():
    X, y = nfir(8, 8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.predict(X, y, X, (1.0, 1.0, -2.0))
    assert e.value.info == 1


# --------------------------------------------------------------------------
# Negative log marginal likelihood and gradient
# --------------------------------------------------------------------------

def test_nlml_closed_form_n1():
    X = np.array([[0.3, -0.2]])
    y = np.array([0.7])
    l, v, s2 = 0.6, 1.5, 0.2
    f, g = oracle.nlml_grad(X, y, (l, v, s2))
    c = v + s2
    assert abs(f - (0.5 * y[0] ** 2 / c + 0.5 * math.log(c) + 0.5 * math.log(2 * math.pi))) <= 1e-15
    dv = 0.5 * (1 / c - y[0] ** 2 / c ** 2)
    np.testing.assert_allclose(g, [0.0, dv, dv], rtol=1e-14, atol=1e-16)


def test_nlml_closed_form_n2():
    X = np.array([[0.0, 0.0], [1.0, 1.0]])   # squared distance 2
    y = np.array([0.4, -0.9])
    l, v, s2 = 0.5, 1.3, 0.3
    e = math.exp(-2 / (2 * l))
    a, b = v + s2, v * e
    det = a * a - b * b
    Kinv = np.array([[a, -b], [-b, a]]) / det
    alpha = Kinv @ y
    f_exact = 0.5 * y @ alpha + 0.5 * math.log(det) + math.log(2 * math.pi)
    A = Kinv - np.outer(alpha, alpha)
    dK_dv = np.array([[1, e], [e, 1]])
    dK_dl = np.array([[0, v * e * 2 / (2 * l * l)], [v * e * 2 / (2 * l * l), 0]])
    g_exact = [0.5 * np.sum(A * dK_dl), 0.5 * np.sum(A * dK_dv), 0.5 * np.trace(A)]
    f, g = oracle.nlml_grad(X, y, (l, v, s2))
    assert abs(f - f_exact) <= 1e-14 * abs(f_exact)
    np.testing.assert_allclose(g, g_exact, rtol=1e-13)


def test_nlml_logdet_vs_slogdet():
    X, y = nfir(100, 8)
    h = (1.0, 1.0, 0.1)
    f, _ = oracle.nlml_grad(X, y, h)
    K = oracle.assemble_K(X, h)
    sign, logdet = np.linalg.slogdet(K)
    assert sign > 0
    quad = y @ np.linalg.solve(K, y)
    np.testing.assert_allclose(f, 0.5 * quad + 0.5 * logdet + 50 * math.log(2 * math.pi),
                               rtol=1e-12)


@pytest.mark.parametrize("h", [(1.0, 1.0, 0.1), (0.3, 2.0, 0.5)])
def test_gradient_vs_finite_differences(h):
    X, y = nfir(60, 8)
    _, g = oracle.nlml_grad(X, y, h)
    step = 1e-5
    fd = []
    for i in range(3):
        hp = list(h); hm = list(h)
        hp[i] += step; hm[i] -= step
        fd.append((oracle.nlml_grad(X, y, tuple(hp))[0]
                   - oracle.nlml_grad(X, y, tuple(hm))[0]) / (2 * step))
    np.testing.assert_allclose(g, fd, rtol=1e-6)


def test_gradient_vs_torch_autograd():
    torch = pytest.importorskip("torch")
    X, y = nfir(70, 8)
    h = (0.3, 2.0, 0.5)
    Xt = torch.tensor(X, dtype=torch.float64)
    yt = torch.tensor(y, dtype=torch.float64)
    th = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    s = ((Xt[:, None, :] - Xt[None, :, :]) ** 2).sum(-1)
    K = th[1] * torch.exp(-s / (2 * th[0])) + th[2] * torch.eye(70, dtype=torch.float64)
    L = torch.linalg.cholesky(K)
    a = torch.cholesky_solve(yt[:, None], L)[:, 0]
    f = 0.5 * yt @ a + torch.log(torch.diagonal(L)).sum() + 35 * math.log(2 * math.pi)
    f.backward()
    fo, go = oracle.nlml_grad(X, y, h)
    assert abs(fo - f.item()) <= 1e-12 * abs(fo)
    np.testing.assert_allclose(go, th.grad.numpy(), rtol=1e-10)


def test_adam_replay_vs_torch_adam():
    torch = pytest.importorskip("torch")
    X, y = nfir(40, 8)
    theta0 = (0.3, 2.0, 0.5)
    trace, th_end = oracle.adam_fit(X, y, theta0, steps=20)
    z = torch.tensor(np.log(theta0), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([z], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    for t in range(20):
        th = torch.exp(z).detach().numpy()
        f, g = oracle.nlml_grad(X, y, tuple(th))
        assert abs(f - trace[t][1]) <= 1e-9 * abs(f)
        opt.zero_grad()
        z.grad = torch.tensor(g * th, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(th_end, torch.exp(z).detach().numpy(), rtol=1e-10)
    assert trace[-1][1] < trace[0][1]


# --------------------------------------------------------------------------
# Error metrics (the normwise reading of "relative error 1e-10"): values
# worked out by hand
# --------------------------------------------------------------------------

def test_rel_err_hand_values():
    # vectors: diff (1, 0, -2), ||diff|| = sqrt(5), ||B|| = sqrt(14)
    assert oracle.rel_err([2.0, 2.0, 1.0], [1.0, 2.0, 3.0]) == pytest.approx(math.sqrt(5 / 14),
                                                                           rel=1e-15)
    # matrices use the Frobenius norm: diff [[0, -2], [0, -2]], ||B||_F = sqrt(14)
    A = np.array([[1.0, 0.0], [0.0, 1.0]])
    B = np.array([[1.0, 2.0], [0.0, 3.0]])
    assert oracle.rel_err(A, B) == pytest.approx(math.sqrt(8 / 14), rel=1e-15)
    # not symmetric in its arguments: ||A - B|| / ||B||, not / ||A||
    assert oracle.rel_err(B, A) == pytest.approx(math.sqrt(8 / 2), rel=1e-15)
    # zero reference: the absolute norm of the difference
    assert oracle.rel_err([1.0, 2.0, 2.0], [0.0, 0.0, 0.0]) == 3.0
    assert oracle.rel_err([0.0], [0.0]) == 0.0


def test_rel_err_lower_hand_values():
    # only the lower triangles count: diff tril = [[0, 0], [2, 0]],
    # ||tril B||_F = sqrt(1 + 0 + 9) (the upper entries 9 and -5 are ignored)
    A = np.array([[1.0, 9.0], [2.0, 3.0]])
    B = np.array([[1.0, -5.0], [0.0, 3.0]])
    assert oracle.rel_err_lower(A, B) == pytest.approx(2 / math.sqrt(10), rel=1e-15)
    # the diagonal is part of the lower triangle
    C = np.array([[2.0, 0.0], [0.0, 3.0]])
    assert oracle.rel_err_lower(C, B) == pytest.approx(1 / math.sqrt(10), rel=1e-15)


def test_max_rel_hand_values():
    # max|A - B| = |4 - (-8)| = 12, max|B| = 8 (absolute values, not signed max)
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[1.0, 2.5], [2.0, -8.0]])
    assert oracle.max_rel(A, B) == 1.5
    assert oracle.max_rel(B, B) == 0.0
    assert oracle.max_rel([0.5], [0.0]) == 0.5
