"""CPU oracle for exact GP prediction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library does not import, link or call it, and it
imports nothing from the GPU library.

The arithmetic lives in ``gpr_oracle.c`` (plain loops, no BLAS/LAPACK),
compiled twice: in double (the oracle proper) and in long double (used only
to show how much of a disagreement is the double oracle's own rounding).
This module marshals numpy arrays into it and adds two pieces written here in
plain Python: the Adam replay of a hyperparameter fit and the error metrics.

Readings of the paper (Sec. 4.1, eq. (1)-(3)) are stated in ``gpr_oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIBS = {}
_f64p = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _lib(real: str = "double"):
    if real not in _build.LIBS:
        raise ValueError(f"unknown oracle precision {real!r}")
    if real not in _LIBS:
        path = _build.LIBS[real]
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        lib.orc_real_bytes.restype = ctypes.c_int
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_kernel_matrix.argtypes = [_f64p, _i64, _f64p, _i64, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, _f64p]
        lib.orc_assemble_K.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _f64p]
        lib.orc_cholesky.argtypes = [_f64p, _i64, _f64p]
        lib.orc_cholesky.restype = ctypes.c_int
        lib.orc_forward.argtypes = [_f64p, _i64, _f64p, _f64p]
        lib.orc_backward.argtypes = [_f64p, _i64, _f64p, _f64p]
        lib.orc_predict.argtypes = [_f64p, _f64p, _i64, _f64p, _i64, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _f64p, _f64p, _f64p, _f64p, _f64p]
        lib.orc_predict.restype = ctypes.c_int
        lib.orc_nlml_grad.argtypes = [_f64p, _f64p, _i64, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      _f64p, _f64p]
        lib.orc_nlml_grad.restype = ctypes.c_int
        lib.orc_gauss_jordan_inverse.argtypes = [_f64p, _i64, _f64p]
        lib.orc_gauss_jordan_inverse.restype = ctypes.c_int
        _LIBS[real] = lib
    return _LIBS[real]


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_f64p)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, info):
        super().__init__(f"oracle: matrix not positive definite (pivot column {info})")
        self.info = info


def num_threads(real="double"):
    """Threads the oracle's parallel loops run with (OpenMP)."""
    return int(_lib(real).orc_num_threads())


def kernel_matrix(A, B, hyper, real="double"):
    """``v exp(-|a_i - b_j|^2 / (2 l))`` for all rows (eq. (1) without its
    noise term: the cross and test covariances carry none)."""
    A, B = _c(A), _c(B)
    l, v, _ = hyper
    out = np.empty((A.shape[0], B.shape[0]))
    _lib(real).orc_kernel_matrix(_p(A), A.shape[0], _p(B), B.shape[0], A.shape[1],
                                 l, v, _p(out))
    return out


def assemble_K(X, hyper, real="double"):
    """Training covariance ``k(X, X) + sigma^2 I`` (eq. (1), noise by index)."""
    X = _c(X)
    l, v, s2 = hyper
    K = np.empty((X.shape[0], X.shape[0]))
    _lib(real).orc_assemble_K(_p(X), X.shape[0], X.shape[1], l, v, s2, _p(K))
    return K


def cholesky(K, real="double"):
    """Returns ``(L, info)``; ``info`` is 0 or the 1-based failing pivot column."""
    K = _c(K)
    L = np.empty_like(K)
    info = _lib(real).orc_cholesky(_p(K), K.shape[0], _p(L))
    return L, info


def forward(L, b, real="double"):
    L, b = _c(L), _c(b)
    x = np.empty_like(b)
    _lib(real).orc_forward(_p(L), L.shape[0], _p(b), _p(x))
    return x


def backward(L, b, real="double"):
    L, b = _c(L), _c(b)
    x = np.empty_like(b)
    _lib(real).orc_backward(_p(L), L.shape[0], _p(b), _p(x))
    return x


def predict(X, y, Xs, hyper, real="double", want=("L", "beta", "alpha", "mean", "cov")):
    """Exact GP prediction from the plain definitions (eqs. (1)-(3)).

    Returns a dict with the requested entries among L, beta, alpha, mean, cov.
    Raises :class:`OracleError` if the Cholesky pivot fails.
    """
    X, y, Xs = _c(X), _c(y), _c(Xs)
    n, D = X.shape
    ns = Xs.shape[0]
    l, v, s2 = hyper
    out = {}
    shapes = {"L": (n, n), "beta": (n,), "alpha": (n,), "mean": (ns,), "cov": (ns, ns)}
    for k in want:
        out[k] = np.empty(shapes[k])
    info = _lib(real).orc_predict(_p(X), _p(y), n, _p(Xs), ns, D, l, v, s2,
                                  _p(out.get("L")), _p(out.get("beta")),
                                  _p(out.get("alpha")), _p(out.get("mean")),
                                  _p(out.get("cov")))
    if info > 0:
        raise OracleError(info)
    if info < 0:
        raise MemoryError("oracle allocation failed")
    return out


def nlml_grad(X, y, hyper, real="double"):
    """``(nlml, grad)`` with ``grad = d/d(lengthscale, variance, noise variance)``."""
    X, y = _c(X), _c(y)
    l, v, s2 = hyper
    nl = np.zeros(1)
    g = np.zeros(3)
    info = _lib(real).orc_nlml_grad(_p(X), _p(y), X.shape[0], X.shape[1], l, v, s2,
                                    _p(nl), _p(g))
    if info > 0:
        raise OracleError(info)
    if info < 0:
        raise MemoryError("oracle allocation failed")
    return float(nl[0]), g


def gauss_jordan_inverse(A, real="double"):
    """Inverse by Gauss-Jordan elimination with partial pivoting (n <= 64)."""
    A = _c(A)
    out = np.empty_like(A)
    rc = _lib(real).orc_gauss_jordan_inverse(_p(A), A.shape[0], _p(out))
    if rc != 0:
        raise ZeroDivisionError("singular matrix in Gauss-Jordan")
    return out


def predict_gauss_jordan(X, y, Xs, hyper):
    """Independent route for eqs. (2)-(3) at small n: explicit K^{-1} by
    Gauss-Jordan, then alpha = K^{-1} y, mean = Ks alpha,
    cov = Kss - Ks K^{-1} Ks^T (matrix products written out with numpy)."""
    K = assemble_K(X, hyper)
    Kinv = gauss_jordan_inverse(K)
    Ks = kernel_matrix(Xs, X, hyper)
    Kss = kernel_matrix(Xs, Xs, hyper)
    alpha = Kinv @ _c(y)
    return {"Kinv": Kinv, "alpha": alpha, "mean": Ks @ alpha,
            "cov": Kss - Ks @ Kinv @ Ks.T}


# --------------------------------------------------------------------------
# Adam replay of a hyperparameter fit (log-parameterised, so theta stays > 0)
# --------------------------------------------------------------------------

def adam_fit(X, y, theta0, steps=20, lr=0.05, betas=(0.9, 0.999), eps=1e-8,
             grad_fn=None):
    """Adam on ``log theta`` for ``steps`` steps, the textbook update
    (bias-corrected first and second moments). ``grad_fn(theta) -> (nlml, g)``
    defaults to the oracle's :func:`nlml_grad`. Returns the list of
    ``(theta, nlml)`` before each step and the final theta."""
    if grad_fn is None:
        def grad_fn(th):
            return nlml_grad(X, y, th)
    z = np.log(np.asarray(theta0, dtype=np.float64))
    m = np.zeros(3)
    s = np.zeros(3)
    b1, b2 = betas
    trace = []
    for t in range(1, steps + 1):
        th = np.exp(z)
        f, g = grad_fn(tuple(th))
        trace.append((th.copy(), f))
        gz = g * th                      # chain rule d/dlog(theta) = theta * d/dtheta
        m = b1 * m + (1 - b1) * gz
        s = b2 * s + (1 - b2) * gz * gz
        mh = m / (1 - b1 ** t)
        sh = s / (1 - b2 ** t)
        z = z - lr * mh / (np.sqrt(sh) + eps)
    return trace, np.exp(z)


# --------------------------------------------------------------------------
# Error metrics
# --------------------------------------------------------------------------

def rel_err(A, B):
    """Normwise relative error ``||A - B|| / ||B||`` (Frobenius / 2-norm)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = float(np.linalg.norm(B))
    d = float(np.linalg.norm(A - B))
    return d / nb if nb > 0 else d


def rel_err_lower(A, B):
    """Normwise relative error over the lower triangles only."""
    return rel_err(np.tril(A), np.tril(B))


def max_rel(A, B):
    """``max|A - B| / max|B|``."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    mb = float(np.max(np.abs(B))) if B.size else 0.0
    md = float(np.max(np.abs(A - B))) if A.size else 0.0
    return md / mb if mb > 0 else md


def log2pi():
    return math.log(2 * math.pi)
