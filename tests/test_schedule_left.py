"""The left-looking tile schedule (host logic, no GPU). In the left-looking
variant of the tiled Cholesky (Sec. 4.2 names it beside the right-looking
Fig. 1), tile column K receives the products L_IJ L_KJ^T of all earlier
columns J < K in one update task just before it is factored, instead of one
rank-m update per step J. Here a column's terms 0 .. K-2 come in one task
(issued one step early, beside the previous column's POTRF and TRSMs) and
its last term K-1 in a second one; the test block of the covariance solve
takes all its terms in one task at the end.

Checked: the update terms, expanded, are exactly the block Cholesky
equations' terms; every data dependency of those equations is ordered by
the launch order (race check); executed on the host in random orders allowed
by the streams and events, the sweep gives the oracle's factor and
covariance, bitwise equal across orders."""
import random

import numpy as np
import pytest
import scipy.linalg

import oracle
from gpr_inputs import nfir_train_test
from paper_2602_19683_amd import schedule_describe

from test_schedule import POTRF, TRSM, SYRK, GEMM, block_cholesky_tasks, happens_before

LEFT = 1


def expand(tasks):
    """(kind, I, K, J, nk, launch) records -> {(kind, I, K, j): launch} over the terms."""
    out = {}
    for kind, I, K, J, nk, li in (tuple(int(v) for v in t) for t in tasks):
        if kind in (SYRK, GEMM):
            for j in range(J, J + nk):
                out[(kind, I, K, j)] = li
        else:
            assert nk == 1
            out[(kind, I, K, J)] = li
    return out


CASES = [(1, 0, 0), (2, 0, 0), (3, 0, 0), (5, 0, 0), (9, 0, 0), (4, 3, 1), (7, 2, 1), (1, 2, 1),
         (5, 3, 2), (6, 1, 2), (2, 2, 2), (1, 3, 2), (3, 1, 2), (4, 3, 3), (1, 2, 3), (5, 3, 4),
         (2, 2, 4), (1, 3, 4), (6, 1, 4), (32, 8, 2)]


@pytest.mark.parametrize("M,Mhat,mode", CASES)
def test_left_schedule_terms_and_races(M, Mhat, mode):
    tasks, launches = schedule_describe(M, Mhat, mode, variant=LEFT)
    assert tasks.shape[1] == 6
    where = expand(tasks)
    n_terms = sum(int(t[4]) for t in tasks)
    want, edges = block_cholesky_tasks(M, Mhat, mode)
    assert len(where) == n_terms == len(want), "a term is repeated or missing"
    assert sorted(where) == sorted(want), "terms differ from the block equations"
    # a multi-term task holds consecutive terms of one tile
    reach, _ = happens_before([tuple(l) for l in launches])
    for i, (st, w0, w1, w2, _) in enumerate(launches):
        for w in (w0, w1, w2):
            assert w < i and (w < 0 or launches[w][0] != st)
    for a, b in edges:
        la, lb = where[a], where[b]
        if la == lb:
            # the same task (consecutive terms of one tile, accumulated in order)
            assert a[:3] == b[:3] and a[0] in (SYRK, GEMM), f"race {a} -> {b} inside a launch"
            continue
        assert (reach[lb] >> la) & 1, f"race {a} -> {b}"


def run_left_on_host(tiles, tinv, tasks, launches, rng):
    n = len(launches)
    _, pred = happens_before([tuple(l) for l in launches])
    by_launch = {}
    for t in tasks:
        by_launch.setdefault(int(t[5]), []).append(tuple(int(v) for v in t[:5]))
    done = set()
    while len(done) < n:
        ready = [i for i in range(n) if i not in done and pred[i] <= done]
        li = rng.choice(ready)
        todo = list(by_launch.get(li, []))
        rng.shuffle(todo)
        for kind, I, K, J, nk in todo:
            if kind == POTRF:
                A = tiles[(J, J)]
                L = np.linalg.cholesky(np.tril(A) + np.tril(A, -1).T)
                tiles[(J, J)] = L
                tinv[J] = scipy.linalg.solve_triangular(L, np.eye(L.shape[0]), lower=True)
            elif kind == TRSM:
                tiles[(I, J)] = tiles[(I, J)] @ tinv[J].T
            else:
                acc = np.zeros_like(tiles[(I, K)])
                for j in range(J, J + nk):
                    acc += tiles[(I, j)] @ tiles[(K, j)].T
                tiles[(I, K)] = tiles[(I, K)] - acc
        done.add(li)


@pytest.mark.parametrize("M,Mhat,mode,m", [(4, 0, 0, 8), (5, 3, 2, 6), (3, 2, 1, 7), (2, 2, 2, 5),
                                           (6, 1, 2, 4), (3, 2, 3, 7), (5, 3, 4, 6), (7, 2, 2, 3)])
def test_left_host_execution_matches_oracle(M, Mhat, mode, m):
    n, ns = M * m, Mhat * m
    h = (1.0, 1.0, 0.1)
    X, y, Xs = nfir_train_test(n, max(ns, 1))
    K = oracle.assemble_K(X, h)
    ref = oracle.predict(X, y, Xs, h) if ns else None
    Lref, _ = oracle.cholesky(K)
    results = []
    for seed in range(3):
        rng = random.Random(seed)
        tiles, tinv = {}, {}
        big = np.zeros((n + ns, n + ns))
        big[:n, :n] = K if mode not in (1, 3) else Lref
        if ns:
            big[n:, :n] = oracle.kernel_matrix(Xs, X, h)
            big[n:, n:] = oracle.kernel_matrix(Xs, Xs, h)
        T = M + (Mhat if mode else 0)
        for I in range(T):
            for J in range(I + 1):
                tiles[(I, J)] = big[I * m:(I + 1) * m, J * m:(J + 1) * m].copy()
        if mode in (1, 3):
            for J in range(M):
                tinv[J] = scipy.linalg.solve_triangular(tiles[(J, J)], np.eye(m), lower=True)
        tasks, launches = schedule_describe(M, Mhat, mode, variant=LEFT)
        run_left_on_host(tiles, tinv, tasks, launches, rng)
        out = np.zeros_like(big)
        for (I, J), t in tiles.items():
            out[I * m:(I + 1) * m, J * m:(J + 1) * m] = t
        results.append(out)
        if mode not in (1, 3):
            assert oracle.rel_err_lower(np.tril(out[:n, :n]), Lref) <= 1e-13
        if mode in (1, 2):
            S = np.tril(out[n:, n:])
            S = S + np.tril(S, -1).T
            assert oracle.rel_err(S, ref["cov"]) <= 1e-12
        if mode in (3, 4):
            var = h[1] - (out[n:, :n] ** 2).sum(axis=1)
            assert oracle.rel_err(var, np.diag(ref["cov"])) <= 1e-12
    for r in results[1:]:
        np.testing.assert_array_equal(r, results[0])


def test_left_dropped_wait_is_caught():
    """Removing any one wait of the left-looking launch list leaves some data
    dependency unordered, so the race check above would fail."""
    M, Mhat, mode = 6, 2, 2
    tasks, launches = schedule_describe(M, Mhat, mode, variant=LEFT)
    where = expand(tasks)
    _, edges = block_cholesky_tasks(M, Mhat, mode)
    for i in range(len(launches)):
        for k in (1, 2, 3):
            if launches[i][k] < 0:
                continue
            L = [list(map(int, l)) for l in launches]
            L[i][k] = -1
            reach, _ = happens_before([tuple(l) for l in L])
            broken = any(where[a] != where[b] and not (reach[where[b]] >> where[a]) & 1
                         for a, b in edges)
            assert broken, f"wait {k} of launch {i} is not needed"
