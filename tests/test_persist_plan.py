"""The ticket order of the persistent executor (host logic, no GPU).

* The work items are exactly the tile tasks of Fig. 1 (extended with the
  covariance rows) cut into POTRF row panels, TRSM strips of 32 rows and
  update blocks (SYRK: only the blocks on or below the diagonal).
* Every wait of every item is met by items with earlier tickets (so the
  executor cannot deadlock), and the panels of one POTRF come in increasing
  order.
* The waits are sufficient: the items are executed on the host in rounds of
  maximal concurrency -- every item whose waits are met runs in the same
  round against a snapshot of the matrix taken before the round -- so a
  missing dependency makes some item read a stale tile. The result must match
  the oracle's factor / covariance, and no two items of one round may write
  the same entries. A few random sequential orders must give the same bits.
"""
import random

import numpy as np
import pytest
import scipy.linalg

import oracle
from gpr_inputs import nfir_train_test
from paper_2602_19683_amd import persist_describe, schedule_describe

PI_POTRF, PI_TRSM, PI_UPDATE = 0, 1, 2
S_POTRF, S_TRSM, S_SYRK, S_GEMM = 0, 1, 2, 3


def tile_counter(I, K):
    return I * (I + 1) // 2 + K


def expected_items(M, Mhat, mode, m, bm):
    tasks, _ = schedule_describe(M, Mhat, mode)
    P, nb = m // 32, m // bm
    out = []
    for kind, I, K, J, _ in tasks:
        if kind == S_POTRF:
            out += [(PI_POTRF, w, J, J, J) for w in range(P)]
        elif kind == S_TRSM:
            out += [(PI_TRSM, s, I, J, J) for s in range(P)]
        else:
            nblk = nb * (nb + 1) // 2 if I == K else nb * nb
            out += [(PI_UPDATE, b, I, K, J) for b in range(nblk)]
    return sorted(out)


SHAPES = [(1, 0, 0, 64, 32), (3, 0, 0, 64, 32), (5, 0, 0, 96, 32), (4, 0, 0, 128, 64),
          (3, 2, 1, 64, 32), (2, 3, 1, 96, 32), (4, 2, 2, 64, 32), (3, 1, 2, 128, 64),
          (1, 2, 2, 64, 32), (6, 2, 2, 64, 64), (3, 2, 3, 64, 32), (4, 2, 4, 64, 32),
          (1, 2, 4, 64, 32)]


@pytest.mark.parametrize("M,Mhat,mode,m,bm", SHAPES)
@pytest.mark.parametrize("workers", [1, 7, 512])
def test_ticket_order_is_complete_and_deadlock_free(M, Mhat, mode, m, bm, workers):
    items, waits = persist_describe(M, Mhat, mode, m, bm, workers)
    assert sorted(tuple(int(v) for v in r) for r in items) == expected_items(M, Mhat, mode, m, bm)
    done = {}
    last_panel = {}
    for (kind, sub, I, K, J), w in zip(items.tolist(), waits.tolist()):
        n = w[0]
        for k in range(n):
            c, v = w[1 + 2 * k], w[2 + 2 * k]
            assert v > 0 and done.get(c, 0) >= v, "wait not met by earlier tickets"
        for k in range(n, 3):
            assert w[1 + 2 * k] == -1 and w[2 + 2 * k] == 0
        sig = w[7]
        assert sig == tile_counter(I, K if kind == PI_UPDATE else (J if kind == PI_TRSM else J))
        if kind == PI_POTRF:
            assert last_panel.get(J, -1) == sub - 1
            last_panel[J] = sub
        done[sig] = done.get(sig, 0) + 1


def test_describe_rejects_bad_arguments():
    from paper_2602_19683_amd import GPR_EINVAL
    from paper_2602_19683_amd import _lib
    import ctypes
    lib = _lib.load()
    n = ctypes.c_int64()
    assert lib.gpr_persist_describe(0, 0, 0, 64, 32, 1, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    assert lib.gpr_persist_describe(2, 0, 1, 64, 32, 1, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    assert lib.gpr_persist_describe(2, 0, 0, 64, 48, 1, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    assert lib.gpr_persist_describe(2, 0, 0, 48, 16, 1, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    assert lib.gpr_persist_describe(2, 0, 0, 64, 32, 0, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    # too small a capacity: the count is still written
    assert lib.gpr_persist_describe(2, 0, 0, 64, 32, 4, None, None, 0, ctypes.byref(n)) == GPR_EINVAL
    assert n.value == 2 * 2 + 2 + 3


class HostSweep:
    """The extended lower-tiled matrix and the item semantics in numpy."""

    def __init__(self, big, T, m, bm, M, mode):
        self.m, self.bm, self.M, self.mode = m, bm, M, mode
        self.t = {(I, J): big[I * m:(I + 1) * m, J * m:(J + 1) * m].copy()
                  for I in range(T) for J in range(I + 1)}
        self.dinv = {}
        self.step = {}
        if mode in (1, 3):
            for J in range(M):
                L = self.t[(J, J)]
                self.dinv[J] = scipy.linalg.solve_triangular(L, np.eye(m), lower=True)

    def run(self, item, src):
        """Runs one item reading from `src` (a HostSweep state); returns the
        writes as a list of (tile, rows, cols, value)."""
        kind, sub, I, K, J = item
        m, bm = self.m, self.bm
        if kind == PI_POTRF:
            A = src.t[(J, J)]
            r = slice(32 * sub, 32 * sub + 32)
            row = A[r].copy()
            for q in range(sub):
                rq = slice(32 * q, 32 * q + 32)
                acc = A[r, rq] - row[:, :32 * q] @ A[rq, :32 * q].T
                row[:, rq] = acc @ np.linalg.inv(A[rq, rq]).T
            d = A[r, r] - row[:, :32 * sub] @ row[:, :32 * sub].T
            row[:, r] = np.linalg.cholesky(np.tril(d) + np.tril(d, -1).T)
            row[:, 32 * sub + 32:] = 0.0
            return [((J, J), r, slice(0, m), row)]
        if kind == PI_TRSM:
            L = src.t[(J, J)]
            r = slice(32 * sub, 32 * sub + 32)
            return [((I, J), r, slice(0, m),
                     scipy.linalg.solve_triangular(L, src.t[(I, J)][r].T, lower=True).T)]
        nb = m // bm
        if I == K:
            bi = 0
            while (bi + 1) * (bi + 2) // 2 <= sub:
                bi += 1
            bj = sub - bi * (bi + 1) // 2
        else:
            bi, bj = divmod(sub, nb)
        ri, rj = slice(bi * bm, bi * bm + bm), slice(bj * bm, bj * bm + bm)
        # the updates of one block must come in step order (bitwise results)
        assert self.step.get((I, K, bi, bj), -1) == J - 1, "update out of step order"
        self.step[(I, K, bi, bj)] = J
        C = src.t[(I, K)][ri, rj] - src.t[(I, J)][ri] @ src.t[(K, J)][rj].T
        return [((I, K), ri, rj, C)]

    def apply(self, writes):
        for tile, r, c, v in writes:
            self.t[tile][r, c] = v


def run_rounds(state, items, waits, sequential_rng=None):
    """Rounds of maximal concurrency, or one runnable item at a time: a random
    one (sequential_rng a random.Random) or the one of the latest step, then
    the earliest ticket (sequential_rng == "latest": runs later steps as early
    as the waits allow and leaves bulk updates of earlier steps to the end)."""
    import copy
    n = len(items)
    cnt = {}
    panels_done = {}
    remaining = list(range(n))
    while remaining:
        runnable = []
        for i in remaining:
            kind, sub, I, K, J = items[i]
            w = waits[i]
            if any(cnt.get(w[1 + 2 * k], 0) < w[2 + 2 * k] for k in range(w[0])):
                continue
            if kind == PI_POTRF and panels_done.get(J, 0) < sub:
                continue
            runnable.append(i)
        assert runnable, "no runnable item: the waits deadlock"
        if sequential_rng == "latest":  # adversarial order
            runnable = [max(runnable, key=lambda i: (items[i][4], -i))]
        elif sequential_rng is not None:
            runnable = [sequential_rng.choice(runnable)]
        snap = copy.deepcopy(state) if len(runnable) > 1 else state
        written = {}
        all_writes = []
        for i in runnable:
            for tile, r, c, v in state.run(items[i], snap):
                mask = written.setdefault(tile, np.zeros((state.m, state.m), dtype=bool))
                assert not mask[r, c].any(), "two concurrent items write the same entries"
                mask[r, c] = True
                all_writes.append((tile, r, c, v))
        state.apply(all_writes)
        for i in runnable:
            kind, sub, I, K, J = items[i]
            sig = waits[i][7]
            cnt[sig] = cnt.get(sig, 0) + 1
            if kind == PI_POTRF:
                panels_done[J] = panels_done.get(J, 0) + 1
        done = set(runnable)
        remaining = [i for i in remaining if i not in done]


@pytest.mark.parametrize("M,Mhat,mode,m,bm", [(4, 0, 0, 64, 32), (3, 2, 2, 64, 32),
                                              (3, 2, 1, 64, 32), (2, 2, 2, 96, 32),
                                              (3, 1, 2, 128, 64), (3, 2, 3, 64, 32),
                                              (3, 2, 4, 64, 32)])
def test_host_execution_matches_oracle(M, Mhat, mode, m, bm):
    n, ns = M * m, Mhat * m
    h = (1.0, 1.0, 0.1)
    X, y, Xs = nfir_train_test(n, max(ns, 1))
    K = oracle.assemble_K(X, h)
    Lref, info = oracle.cholesky(K)
    assert info == 0
    ref = oracle.predict(X, y, Xs, h) if ns else None
    big = np.zeros((n + ns, n + ns))
    big[:n, :n] = K if mode not in (1, 3) else Lref
    if ns:
        big[n:, :n] = oracle.kernel_matrix(Xs, X, h)
        big[n:, n:] = oracle.kernel_matrix(Xs, Xs, h)
    T = M + (Mhat if mode else 0)
    items, waits = persist_describe(M, Mhat, mode, m, bm, 64)
    items = [tuple(int(v) for v in r) for r in items]
    waits = [tuple(int(v) for v in r) for r in waits]
    outs = []
    for order in [None, "latest", 0, 1]:
        st = HostSweep(big, T, m, bm, M, mode)
        run_rounds(st, items, waits, order if order in (None, "latest") else random.Random(order))
        out = np.zeros_like(big)
        for (I, J), t in st.t.items():
            out[I * m:(I + 1) * m, J * m:(J + 1) * m] = t
        if mode not in (1, 3):
            assert oracle.rel_err_lower(np.tril(out[:n, :n]), Lref) <= 1e-12
        if mode in (1, 2):
            S = np.tril(out[n:, n:])
            S = S + np.tril(S, -1).T
            assert oracle.rel_err(S, ref["cov"]) <= 1e-11
        if mode in (3, 4):   # variances only: V^T formed, the test block untouched
            var = h[1] - (out[n:, :n] ** 2).sum(axis=1)
            assert oracle.rel_err(var, np.diag(ref["cov"])) <= 1e-11
            np.testing.assert_array_equal(np.tril(out[n:, n:]), np.tril(big[n:, n:]))
        outs.append(out)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])   # the same bits in any valid order
