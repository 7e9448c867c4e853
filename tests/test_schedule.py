"""The tile schedule (host logic, no GPU): task counts of Fig. 1, the Fig. 2
example, a race check of the three-stream launch order against the data
dependencies of the block Cholesky equations (Sec. 4.2), and a host execution
of the schedule in random orders compared with the oracle."""
import os
import random

import numpy as np
import pytest
import scipy.linalg

import oracle
from gpr_inputs import nfir_train_test
from paper_2602_19683_amd import schedule_describe

POTRF, TRSM, SYRK, GEMM = 0, 1, 2, 3
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig2_first_iteration.txt")


def block_cholesky_tasks(M, Mhat, mode):
    """Tile tasks and their data dependencies, derived from the block form of
    K = L L^T on lower tiles (Sec. 4.2) rather than from a printed loop:
      L_KK = chol(A_KK - sum_{J<K} L_KJ L_KJ^T),
      L_IK = (A_IK - sum_{J<K} L_IJ L_KJ^T) L_KK^{-T}     (I > K),
    extended with the test rows M..M+Mhat-1 of the covariance solve
    (V^T = K_{X*,X} L^{-T} and K_{X*,X*} - V^T V; modes 1 to 4, modes 3 and 4
    without the test block). Each term L_IJ L_KJ^T is one update task
    (I, K, J) (SYRK when I == K, else GEMM) applied to tile (I, K) in
    increasing J; a tile becomes final by its POTRF or TRSM. Returns the task
    list and the edges (a, b): b reads what a writes, or both update the same
    tile in that order (so the accumulation order is fixed)."""
    factor = mode in (0, 2, 4)
    predict = mode in (1, 2, 3, 4)
    block = mode in (1, 2)
    T = M + (Mhat if predict else 0)

    def row_swept(I):
        return (I < M and factor) or (I >= M and predict)

    def producer(I, K):
        """The task that makes L tile (I, K) (K < M) final; None if given."""
        if not row_swept(I):
            return None
        return (POTRF, K, K, K) if I == K else (TRSM, I, K, K)

    tasks, edges = [], []
    for I in range(T):
        if not row_swept(I):
            continue
        for K in range(I + 1):
            if K >= M and not block:
                continue
            prev = None
            for J in range(min(K, M)):
                u = (SYRK if I == K else GEMM, I, K, J)
                tasks.append(u)
                for src in (producer(I, J), producer(K, J)):
                    if src is not None:
                        edges.append((src, u))
                if prev is not None:
                    edges.append((prev, u))
                prev = u
            if K < M:
                fin = producer(I, K)
                tasks.append(fin)
                if prev is not None:
                    edges.append((prev, fin))
                if I != K and producer(K, K) is not None:
                    edges.append((producer(K, K), fin))
    return tasks, edges


def happens_before(launches):
    n = len(launches)
    pred = [set() for _ in range(n)]
    last = {0: -1, 1: -1, 2: -1}
    launches = [tuple(int(v) for v in l) for l in launches]
    for i, (st, w0, w1, w2, _) in enumerate(launches):
        if last[st] >= 0:
            pred[i].add(last[st])
        for w in (w0, w1, w2):
            if w >= 0:
                pred[i].add(w)
        last[st] = i
    reach = [0] * n  # bitset of launches that happen before i
    for i in range(n):
        b = 0
        for p in pred[i]:
            b |= reach[p] | (1 << p)
        reach[i] = b
    return reach, pred


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8, 32])
def test_fig1_task_counts(M):
    tasks, launches = schedule_describe(M, 0, 0)
    kinds = tasks[:, 0]
    assert (kinds == POTRF).sum() == M
    assert (kinds == TRSM).sum() == M * (M - 1) // 2
    assert (kinds == SYRK).sum() == M * (M - 1) // 2
    assert (kinds == GEMM).sum() == M * (M - 1) * (M - 2) // 6


@pytest.mark.parametrize("M,Mhat", [(4, 4), (32, 8), (3, 1)])
def test_covariance_solve_task_counts(M, Mhat):
    tasks, _ = schedule_describe(M, Mhat, 1)
    kinds = tasks[:, 0]
    assert (kinds == POTRF).sum() == 0
    assert (kinds == TRSM).sum() == Mhat * M                         # V tiles, one per step
    # V updates: Mhat * M (M - 1) / 2; Sigma: Mhat (Mhat + 1) / 2 per step
    assert (kinds == GEMM).sum() + (kinds == SYRK).sum() == \
        Mhat * M * (M - 1) // 2 + M * Mhat * (Mhat + 1) // 2
    assert (kinds == SYRK).sum() == M * Mhat


def test_fig2_first_iteration_golden():
    grid = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    M = len(grid)
    tasks, _ = schedule_describe(M, 0, 0)
    sym = {POTRF: "P", TRSM: "T", SYRK: "S", GEMM: "G"}
    got = [["." for _ in range(M)] for _ in range(M)]
    for kind, I, K, J, _ in tasks:
        if J == 0:
            got[I][K] = sym[kind]
    assert got == grid


def test_memory_fraction_of_lower_tiles():
    # Sec. 4.2: lower tiles need 50 % to 75 % of the full matrix; the
    # assembled entries n^2 (M + 1) / (2 M) shrink as M grows (Sec. 5.1).
    for M in [2, 4, 8, 32, 64]:
        frac = (M * (M + 1) // 2) / (M * M)
        assert 0.5 < frac <= 0.75
        assert abs(frac - (M + 1) / (2 * M)) < 1e-15
    assert (32 * 33 // 2) * 512 * 512 * 8 == 1107296256  # bytes of K at n = 16384, m = 512


@pytest.mark.parametrize("M,Mhat,mode", [(1, 0, 0), (2, 0, 0), (3, 0, 0), (5, 0, 0), (9, 0, 0),
                                         (4, 3, 1), (7, 2, 1), (1, 2, 1), (5, 3, 2), (6, 1, 2),
                                         (2, 2, 2), (1, 3, 2), (3, 1, 2), (4, 3, 3), (1, 2, 3),
                                         (5, 3, 4), (2, 2, 4), (1, 3, 4), (6, 1, 4)])
def test_schedule_has_no_races(M, Mhat, mode):
    tasks, launches = schedule_describe(M, Mhat, mode)
    want, edges = block_cholesky_tasks(M, Mhat, mode)
    got = sorted(tuple(t[:4]) for t in tasks)
    assert got == sorted(want), "schedule task multiset differs from the block equations"
    where = {tuple(t[:4]): int(t[4]) for t in tasks}
    reach, _ = happens_before([tuple(l) for l in launches])
    # launches only wait on earlier launches of other streams
    for i, (st, w0, w1, w2, _) in enumerate(launches):
        for w in (w0, w1, w2):
            assert w < i and (w < 0 or launches[w][0] != st)
    # every data dependency is ordered by stream order or an event (two
    # tasks of one launch run concurrently, so a dependency between them is
    # a race)
    for a, b in edges:
        la, lb = where[a], where[b]
        assert la != lb and (reach[lb] >> la) & 1, f"race {a} -> {b}"
    # and every write of a tile is ordered with every other access to it
    # through those edges: the only writers of tile (I, K) are its updates
    # (chained) and its POTRF / TRSM (after the chain); its readers come
    # after its final writer
    writers = {}
    for t in want:
        writers.setdefault((t[1], t[2]), []).append(t)
    for tile, ws in writers.items():
        for x, y in zip(ws, ws[1:]):
            assert (reach[where[y]] >> where[x]) & 1, f"unordered writes of {tile}: {x}, {y}"


def run_schedule_on_host(tiles, tinv, tasks, launches, rng):
    """Executes the launches in a random order allowed by the stream / event
    semantics, tasks of one launch in random order, tile ops in numpy."""
    n = len(launches)
    reach, pred = happens_before([tuple(l) for l in launches])
    by_launch = {}
    for t in tasks:
        by_launch.setdefault(int(t[4]), []).append(tuple(t[:4]))
    done = set()
    while len(done) < n:
        ready = [i for i in range(n) if i not in done and pred[i] <= done]
        li = rng.choice(ready)
        todo = list(by_launch.get(li, []))
        rng.shuffle(todo)
        for kind, I, K, J in todo:
            if kind == POTRF:
                L = np.linalg.cholesky(np.tril(tiles[(J, J)]) + np.tril(tiles[(J, J)], -1).T)
                tiles[(J, J)] = L
                tinv[J] = scipy.linalg.solve_triangular(L, np.eye(L.shape[0]), lower=True)
            elif kind == TRSM:
                tiles[(I, J)] = tiles[(I, J)] @ tinv[J].T
            else:
                tiles[(I, K)] = tiles[(I, K)] - tiles[(I, J)] @ tiles[(K, J)].T
        done.add(li)


@pytest.mark.parametrize("M,Mhat,mode,m", [(4, 0, 0, 8), (5, 3, 2, 6), (3, 2, 1, 7), (2, 2, 2, 5),
                                           (6, 1, 2, 4), (3, 2, 3, 7), (5, 3, 4, 6)])
def test_host_execution_matches_oracle(M, Mhat, mode, m):
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
        tasks, launches = schedule_describe(M, Mhat, mode)
        run_schedule_on_host(tiles, tinv, tasks, launches, rng)
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
            # variances from the rows of V^T; the test block is left as assembled
            var = h[1] - (out[n:, :n] ** 2).sum(axis=1)
            assert oracle.rel_err(var, np.diag(ref["cov"])) <= 1e-12
            np.testing.assert_array_equal(np.tril(out[n:, n:]), np.tril(big[n:, n:]))
    for r in results[1:]:
        np.testing.assert_array_equal(r, results[0])   # order-independent, bitwise
