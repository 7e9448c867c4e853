"""The tile products that build the group inverses of the vector solves
(Sec. 4.1: beta = L^{-1} y and alpha = L^{-T} beta by block substitution over
groups of tile rows), checked on the host without a GPU: every task's terms
lie inside its launch's range (the kernel indexes them from there), every
operand is written by an earlier launch, and executing the plan with numpy
on a random factor gives the inverse of every group's block of tiles; then
the grouped substitution, in the order the solve kernels take it, solves
L x = b and L^T x = b."""
import numpy as np
import pytest

from paper_2602_19683_amd import solve_plan_describe

TR_L, TR_TINV, TR_W, TR_Y = 0, 1, 2, 3


def _plan(M, tile):
    G, tasks, terms = solve_plan_describe(M, tile)
    return G, tasks, terms


@pytest.mark.parametrize("tile", [32, 96, 256, 512, 1024])
@pytest.mark.parametrize("M", list(range(1, 12)) + [16, 32, 33])
def test_ranges_and_order(M, tile):
    G, tasks, terms = _plan(M, tile)
    assert G == (4 if tile <= 256 else 2)
    ng = -(-M // G)
    nslot = ng * G * (G - 1) // 2
    if M < 2:
        assert len(tasks) == 0 and len(terms) == 0
        return
    nlaunch = int(tasks[:, 0].max()) + 1
    assert nlaunch <= 2 * int(np.log2(G))   # a level with no task has no launch
    written = {}   # (kind, slot) -> launch
    term0 = 0
    for l in range(nlaunch):
        sel = tasks[tasks[:, 0] == l]
        nterm = int(sel[:, 5].sum())
        # launch-relative term ranges, contiguous and in task order
        pos = 0
        for t in sel:
            assert t[4] == pos and t[5] >= 1
            pos += int(t[5])
        assert pos == nterm
        lt = terms[term0:term0 + nterm]
        term0 += nterm
        for kind, a, b in lt[:, 0:3].tolist() + lt[:, 3:6].tolist():
            if kind == TR_L:
                assert 0 <= b < a < M        # strictly lower tiles of L
            elif kind == TR_TINV:
                assert 0 <= a < M
            else:
                assert kind in (TR_W, TR_Y) and 0 <= a < nslot
                assert written.get((kind, a), nlaunch) < l, "read before written"
        for t in sel:
            key = (int(t[1]), int(t[2]))
            assert t[1] in (TR_W, TR_Y) and 0 <= t[2] < nslot
            assert key not in written, "slot written twice"
            written[key] = l
    assert term0 == len(terms)
    # every off-diagonal tile of every group's inverse is produced
    for g in range(ng):
        ns = min(G, M - g * G)
        for i in range(ns):
            for j in range(i):
                assert (TR_W, g * G * (G - 1) // 2 + i * (i - 1) // 2 + j) in written


def _execute(M, tile, m, rng):
    """Runs the plan with numpy on an m x m tiling of a random factor."""
    G, tasks, terms = _plan(M, tile)
    n = M * m
    A = rng.standard_normal((n, n))
    L = np.linalg.cholesky(A @ A.T + n * np.eye(n))
    tl = lambda I, J: L[I * m:(I + 1) * m, J * m:(J + 1) * m]  # noqa: E731
    tinv = [np.linalg.inv(tl(J, J)) for J in range(M)]
    slots = {TR_W: {}, TR_Y: {}}

    def op(kind, a, b):
        if kind == TR_L:
            return tl(a, b)
        if kind == TR_TINV:
            return tinv[a]
        return slots[kind][a]

    if len(tasks):
        term0 = 0
        for l in range(int(tasks[:, 0].max()) + 1):
            sel = tasks[tasks[:, 0] == l]
            for t in sel:
                acc = np.zeros((m, m))
                for u in range(int(t[4]), int(t[4] + t[5])):
                    r = terms[term0 + u]
                    acc += r[6] * op(*r[0:3]) @ op(*r[3:6])
                slots[int(t[1])][int(t[2])] = acc
            term0 += int(sel[:, 5].sum())
    return G, L, tl, tinv, slots[TR_W]


@pytest.mark.parametrize("tile", [64, 512])
@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6, 7, 8, 9, 13])
def test_plan_builds_group_inverses_and_solves(M, tile):
    rng = np.random.default_rng(M * 1000 + tile)
    m = 3
    G, L, tl, tinv, W = _execute(M, tile, m, rng)
    S = G * (G - 1) // 2
    ng = -(-M // G)

    def inv(g, i, j):
        return tinv[g * G + i] if i == j else W[g * S + i * (i - 1) // 2 + j]

    for g in range(ng):
        J0, ns = g * G, min(G, M - g * G)
        Bi = np.linalg.inv(L[J0 * m:(J0 + ns) * m, J0 * m:(J0 + ns) * m])
        for i in range(ns):
            for j in range(i + 1):
                np.testing.assert_allclose(inv(g, i, j), Bi[i * m:(i + 1) * m, j * m:(j + 1) * m],
                                           rtol=0, atol=1e-12)
    b = rng.standard_normal(M * m)
    seg = lambda v, J: v[J * m:(J + 1) * m]  # noqa: E731
    for trans in (False, True):
        r, x = b.copy(), np.zeros_like(b)
        for step in range(ng):
            g = ng - 1 - step if trans else step
            J0, ns = g * G, min(G, M - g * G)
            if not trans:
                for i in range(ns):
                    x[(J0 + i) * m:(J0 + i + 1) * m] = sum(inv(g, i, j) @ seg(r, J0 + j)
                                                           for j in range(i + 1))
                for K in range(J0 + ns, M):
                    r[K * m:(K + 1) * m] -= sum(tl(K, J0 + j) @ seg(x, J0 + j) for j in range(ns))
            else:
                for j in range(ns):
                    x[(J0 + j) * m:(J0 + j + 1) * m] = sum(inv(g, i, j).T @ seg(r, J0 + i)
                                                           for i in range(j, ns))
                for K in range(J0):
                    r[K * m:(K + 1) * m] -= sum(tl(J0 + i, K).T @ seg(x, J0 + i)
                                                for i in range(ns))
        ref = np.linalg.solve(L.T if trans else L, b)
        np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-11)


def test_bad_arguments():
    from paper_2602_19683_amd.gpr import GPRError
    for M, tile in ((0, 256), (4, 16), (4, 100), (4, 2048)):
        with pytest.raises(GPRError):
            solve_plan_describe(M, tile)
