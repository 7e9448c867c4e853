"""Seeded synthetic NFIR-shaped inputs for exact GP regression.

This module is shared by the CPU oracle (tests) and the GPU path (tests,
bench, smoke). It holds no arithmetic of the method itself: it only draws
inputs.

Shape of the data (stand-in for the mass-spring-damper NFIR data of the
paper's Sec. 1 and Sec. 4.1, whose simulator and dataset are not available
here):

* forces ``u_t ~ U[-1, 1]``, ``t = 0 .. n + D - 2``, drawn with
  ``numpy.random.default_rng(seed)`` (PCG64);
* regressor row ``x_i`` holds the last ``D`` forces, newest first:
  ``X[i, d] = u[i + D - 1 - d]``;
* target ``y_i = tanh(sum_k 0.5**k * X[i, k]) + e_i`` with
  ``e_i ~ N(0, 0.01)`` read as a variance (standard deviation 0.1).

Training sets use seed 0 and test sets seed 1 unless stated otherwise.
"""
from __future__ import annotations

import numpy as np

TRAIN_SEED = 0
TEST_SEED = 1

# Hyperparameters fixed in the paper's experiments (Sec. 4.1):
# lengthscale 1, vertical variance 1, noise variance 0.1.
DEFAULT_HYPER = (1.0, 1.0, 0.1)


def nfir(n: int, D: int = 8, seed: int = TRAIN_SEED):
    """Return ``(X, y)``: ``X`` is ``n x D`` float64 C-contiguous, ``y`` has length ``n``."""
    if n < 0 or D <= 0:
        raise ValueError("need n >= 0 and D > 0")
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=n + D - 1)
    idx = np.arange(n)[:, None] + (D - 1) - np.arange(D)[None, :]
    X = np.ascontiguousarray(u[idx], dtype=np.float64)
    w = 0.5 ** np.arange(D)
    y = np.tanh(X @ w) + rng.normal(0.0, 0.1, size=n)
    return X, np.ascontiguousarray(y, dtype=np.float64)


def nfir_train_test(n: int, n_test: int, D: int = 8,
                    train_seed: int = TRAIN_SEED, test_seed: int = TEST_SEED):
    """Training set ``(X, y)`` and test features ``Xs`` (test targets are not used)."""
    X, y = nfir(n, D, train_seed)
    Xs, _ = nfir(n_test, D, test_seed)
    return X, y, Xs


def random_spd(n: int, seed: int = 0, shift: float = 1.0):
    """Random symmetric positive definite matrix ``A A^T / n + shift I`` (float64)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return np.ascontiguousarray(A @ A.T / max(n, 1) + shift * np.eye(n))
