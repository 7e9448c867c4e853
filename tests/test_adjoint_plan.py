"""The reverse (adjoint) sweep of gpr_nlml_grad as a plan, checked on the host.

gpr_adjoint_describe exports the batched tile-product launches the library
runs for the NLML gradient. Here they are executed with numpy tile by tile
(every task of a launch reads the state before the launch, as on the GPU)
on a factor computed by the oracle, and the result is compared with the
closed form of the Cholesky adjoint for the NLML: the lower-convention
adjoint of K is tril(W) - diag(W) / 2 with W = K^{-1} - alpha alpha^T
(K^{-1} from the oracle's triangular solves on unit vectors). The gradient
reduced from it must equal the oracle's trace-formula gradient. A plan
whose launches let two tasks write one tile, or let a task read a tile that
another task of the same launch writes, fails the race check; so does a pair
of launches on the two streams that no wait orders and that touch the same
tile; and the plan executed in random orders the streams allow must give the
same bits.
"""
import random

import numpy as np
import pytest

import oracle
from gpr_inputs import nfir
from paper_2602_19683_amd import adjoint_describe

AM_NONE, AM_L, AM_LBAR, AM_ABAR, AM_TINV, AM_PART, AM_Q, AM_G, AM_X = range(-1, 8)
TRANS_A, TRANS_B, TRI_A, TRI_B = 1, 2, 4, 8


def _key(mat, I, J):
    if mat in (AM_L, AM_LBAR, AM_ABAR):
        return (mat, I, J)
    if mat in (AM_TINV, AM_PART):
        return (mat, I, 0)
    return (mat, 0, 0)


def launch_accesses(tasks, terms, launch):
    """(writes, reads) tile keys of one launch."""
    kind, step, first, count = launch[:4]
    writes, reads = set(), set()
    for t in range(first, first + count):
        (om, oI, oJ, cm, cI, cJ, part0, npart, ft, nterm, epi, _) = tasks[t]
        writes.add(_key(om, oI, oJ))
        if cm != AM_NONE and _key(cm, cI, cJ) != _key(om, oI, oJ):
            reads.add(_key(cm, cI, cJ))
        for p in range(part0, part0 + npart):
            reads.add(_key(AM_PART, p, 0))
        for q in range(ft, ft + nterm):
            am, aI, aJ, bm, bI, bJ, alpha, flags = terms[q]
            reads.add(_key(am, aI, aJ))
            reads.add(_key(bm, bI, bJ))
    return writes, reads


def happens_before(launches):
    """Bitsets of the launches that finish before each one starts: stream
    order plus the waits on the other stream."""
    n = len(launches)
    pred = [set() for _ in range(n)]
    last = {}
    for i, L in enumerate(launches):
        st, wait = int(L[4]), int(L[5])
        if st in last:
            pred[i].add(last[st])
        if wait >= 0:
            assert wait < i and int(launches[wait][4]) != st
            pred[i].add(wait)
        last[st] = i
    reach = [0] * n
    for i in range(n):
        r = 0
        for p in pred[i]:
            r |= reach[p] | (1 << p)
        reach[i] = r
    return reach, pred


def run_plan(M, G, m, L_t, Lbar_t, rng=None):
    """Executes the plan on dicts of m x m tiles in an order allowed by the
    streams and waits (list order, or a random one with rng); every task of a
    launch reads the state before the launch. Returns the Abar tiles."""
    tasks, terms, launches = adjoint_describe(M, G)
    st = {}
    for (I, J), T in L_t.items():
        st[(AM_L, I, J)] = T
    for (I, J), T in Lbar_t.items():
        st[(AM_LBAR, I, J)] = T.copy()
    for K in range(M):
        st[(AM_TINV, K, 0)] = np.linalg.inv(L_t[(K, K)])

    def get(mat, I, J):
        return st[_key(mat, I, J)]

    _, pred = happens_before(launches)
    order = list(range(len(launches)))
    if rng is not None:
        done, order = set(), []
        while len(order) < len(launches):
            ready = [i for i in range(len(launches)) if i not in done and pred[i] <= done]
            i = rng.choice(ready)
            order.append(i)
            done.add(i)
    for li in order:
        kind, step, first, count = launches[li][:4]
        writes, out = [], {}
        for t in range(first, first + count):
            (om, oI, oJ, cm, cI, cJ, part0, npart, ft, nterm, epi, _) = tasks[t]
            acc = np.zeros((m, m))
            if cm != AM_NONE:
                acc += get(cm, cI, cJ)
            for p in range(part0, part0 + npart):
                acc += get(AM_PART, p, 0)
            for q in range(ft, ft + nterm):
                am, aI, aJ, bm, bI, bJ, alpha, flags = terms[q]
                A, B = get(am, aI, aJ), get(bm, bI, bJ)
                assert _key(am, aI, aJ) != _key(om, oI, oJ)
                assert _key(bm, bI, bJ) != _key(om, oI, oJ)
                A = np.tril(A) if flags & TRI_A else A
                B = np.tril(B) if flags & TRI_B else B
                A = A.T if flags & TRANS_A else A
                B = B.T if flags & TRANS_B else B
                acc += alpha * (A @ B)
            if epi == 1:
                acc = np.tril(acc) - 0.5 * np.diag(np.diag(acc))
            elif epi == 2:
                acc = np.tril(acc) + np.tril(acc, -1).T
            k = _key(om, oI, oJ)
            writes.append(k)
            out[k] = acc
        w, r = launch_accesses(tasks, terms, launches[li])
        assert len(set(writes)) == len(writes), f"launch {kind}/{step}: two tasks write one tile"
        assert not (w & r), f"launch {kind}/{step}: a task reads another's output"
        st.update(out)
    return {(I, J): st[(AM_ABAR, I, J)] for I in range(M) for J in range(I + 1)}


def tiles(A, M, m):
    return {(I, J): A[I * m:(I + 1) * m, J * m:(J + 1) * m].copy()
            for I in range(M) for J in range(I + 1)}


def untile(T, M, m):
    A = np.zeros((M * m, M * m))
    for (I, J), t in T.items():
        A[I * m:(I + 1) * m, J * m:(J + 1) * m] = t
    return A


def reduce_grad(Ab, X, n, hyper):
    """sum_{i >= j} Abar_ij dK_ij/dtheta for the SE kernel (l, v, sigma^2)."""
    l, v, _ = hyper
    A = np.tril(Ab[:n, :n])
    s = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    e = np.exp(-s / (2 * l))
    return np.array([(A * v * e * s / (2 * l * l)).sum(), (A * e).sum(), np.trace(A)])


@pytest.mark.parametrize("n,m,G", [(8, 8, 2), (16, 8, 1), (40, 8, 2), (45, 8, 3),
                                   (64, 16, 2), (100, 16, 4), (7, 8, 1)])
def test_plan_matches_closed_form_adjoint(n, m, G):
    X, y = nfir(n, 3, seed=n + m)
    hyper = (0.8, 1.3, 0.2)
    K = oracle.assemble_K(X, hyper)
    L, info = oracle.cholesky(K)
    assert info == 0
    beta = oracle.forward(L, y)
    alpha = oracle.backward(L, beta)
    Kinv = np.column_stack([oracle.backward(L, oracle.forward(L, e)) for e in np.eye(n)])
    W = Kinv - np.outer(alpha, alpha)
    expect = np.tril(W) - 0.5 * np.diag(np.diag(W))

    # padded to M m with an identity block, as the library pads
    M = (n + m - 1) // m
    N = M * m
    Lp = np.eye(N)
    Lp[:n, :n] = L
    ap = np.zeros(N)
    bp = np.zeros(N)
    ap[:n], bp[:n] = alpha, beta
    seed = -np.tril(np.outer(ap, bp)) + np.diag(1.0 / np.diag(Lp))
    Ab = untile(run_plan(M, G, m, tiles(Lp, M, m), tiles(seed, M, m)), M, m)
    # any order the two streams allow gives the same bits
    for r in range(2):
        Ar = untile(run_plan(M, G, m, tiles(Lp, M, m), tiles(seed, M, m), random.Random(r)), M, m)
        np.testing.assert_array_equal(Ar, Ab)
    scale = np.abs(expect).max()
    assert np.abs(np.tril(Ab[:n, :n]) - expect).max() <= 1e-11 * scale
    # the padded block stays decoupled from the data block
    assert np.abs(Ab[n:, :n]).max(initial=0.0) <= 1e-12 * scale

    nl, g = oracle.nlml_grad(X, y, hyper)
    gp = reduce_grad(Ab, X, n, hyper)
    assert np.allclose(gp, g, rtol=1e-10, atol=1e-10 * np.abs(g).max())


@pytest.mark.parametrize("M,G", [(1, 1), (2, 2), (3, 1), (5, 2), (9, 3), (12, 5), (32, 2)])
def test_launches_on_two_streams_do_not_race(M, G):
    """Launches that the streams and waits leave unordered touch disjoint
    tiles (no read of another's output, no common output)."""
    tasks, terms, launches = adjoint_describe(M, G)
    reach, _ = happens_before(launches)
    acc = [launch_accesses(tasks, terms, L) for L in launches]
    n = len(launches)
    assert any(int(L[4]) == 1 for L in launches) or M < 4
    for i in range(n):
        for j in range(i + 1, n):
            if (reach[j] >> i) & 1:
                continue
            wi, ri = acc[i]
            wj, rj = acc[j]
            assert not (wi & wj), f"launches {i}, {j} write the same tile"
            assert not (wi & rj) and not (wj & ri), f"launches {i}, {j} race"


@pytest.mark.parametrize("M,G", [(1, 1), (2, 2), (5, 2), (9, 3), (12, 5)])
def test_plan_counts(M, G):
    tasks, terms, launches = adjoint_describe(M, G)
    # tile products: TRSM adjoint M(M-1)/2, POTRF adjoint 3 M, diagonal row
    # sums M(M-1)/2, pulls: M - J terms for each of the M - J - 1 tiles below
    # the diagonal of column J
    tprod = M * (M - 1) // 2 + 3 * M + M * (M - 1) // 2
    tprod += sum((M - J - 1) * (M - J) for J in range(M))
    assert len(terms) == tprod
    # no partial chunk holds more than G terms
    for kind, step, first, count, stream, wait in launches:
        if kind == 1:
            assert all(tasks[t][9] <= G for t in range(first, first + count))
    # on each stream the reverse steps run from M-1 down to 0
    for stream in (0, 1):
        steps = [int(L[1]) for L in launches if int(L[4]) == stream]
        assert steps == sorted(steps, reverse=True)
    chain = [int(L[1]) for L in launches if int(L[4]) == 0]
    assert chain[0] == M - 1 and chain[-1] == 0
