"""The persistent executor (one launch per sweep, device-side ticket order and
per-tile progress counters) against the stream executor and the oracle.

Both executors run the same device routines with the same per-element
operation order, so every FP64 result must agree BIT FOR BIT: factor,
mean, covariance, NLML and gradient. Small cases are also checked against
the oracle (FP64 bar 1e-10) at every size up to n = 4096; the full benchmark
shape (n = 16384, n_test = 4096, tile 512) is compared bitwise with the stream
executor here and with the oracle in test_gpu_c3_oracle.py.
"""
import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir, nfir_train_test

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


def factor(ctx, X, h, tile):
    K = ctx.assemble(dev(X), h, tile)
    ctx.cholesky(K)
    L = host(ctx.to_dense(K))
    assert ctx.sync()[0] == 0
    K.free()
    return L


@pytest.mark.parametrize("n,tile", [(32, 32), (100, 32), (256, 64), (777, 96), (1000, 128),
                                    (2048, 256), (4096, 512), (3000, 1024)])
def test_cholesky_bitwise_equal_to_streams(ctxs, n, tile):
    say(f"persistent cholesky n={n} tile={tile}")
    s, p = ctxs
    X, _ = nfir(n, seed=n + tile)
    Ls = factor(s, X, DEFAULT_HYPER, tile)
    Lp = factor(p, X, DEFAULT_HYPER, tile)
    np.testing.assert_array_equal(Lp, Ls)
    Lref, info = oracle.cholesky(oracle.assemble_K(X, DEFAULT_HYPER))
    assert info == 0
    e = oracle.rel_err_lower(np.tril(Lp), Lref)
    say(f"  rel(L) vs oracle {e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("n,ns,tile", [(128, 128, 32), (70, 5, 32), (1000, 300, 128),
                                       (4096, 1024, 256), (2048, 1000, 512)])
def test_fit_predict_bitwise_equal_to_streams(ctxs, n, ns, tile):
    say(f"persistent fit_predict n={n} n_test={ns} tile={tile}")
    s, p = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    out = []
    for c in (s, p):
        mean, cov, K = c.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile)
        out.append((host(mean), host(cov)))
        assert c.sync()[0] == 0
        # covariance solve with the factor now in the handle (given-factor sweep)
        m2, c2 = c.predict(K, Xd, yd, Xsd, DEFAULT_HYPER)
        np.testing.assert_array_equal(host(m2), out[-1][0])
        np.testing.assert_array_equal(host(c2), out[-1][1])
        K.free()
    np.testing.assert_array_equal(out[1][0], out[0][0])
    np.testing.assert_array_equal(out[1][1], out[0][1])
    ref = oracle.predict(X, y, Xs, DEFAULT_HYPER)
    em, ec = oracle.rel_err(out[1][0], ref["mean"]), oracle.rel_err(out[1][1], ref["cov"])
    say(f"  rel(mean) {em:.3e} rel(cov) {ec:.3e}")
    assert em <= TOL and ec <= TOL


@pytest.mark.parametrize("prec,n,ns,tile", [("fp32", 1000, 300, 128), ("fp32", 4096, 1024, 512),
                                           ("bf16", 1000, 300, 128)])
def test_mixed_precision_bitwise_equal_to_streams(ctxs, prec, n, ns, tile):
    """FP32 tile updates run as persistent items (BF16 sweeps of a persistent
    context run on the streams): factor, mean, covariance and the
    refinement statistics equal the stream executor's."""
    say(f"persistent mixed {prec} n={n} n_test={ns} tile={tile}")
    s, p = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    out = []
    for c in (s, p):
        mean, cov, K, st = c.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile, prec, ir_stats=True)
        L = host(c.to_dense(K))
        out.append((host(mean), host(cov), L, st))
        assert c.sync()[0] == 0
        K.free()
    for a, b in zip(out[0][:3], out[1][:3]):
        np.testing.assert_array_equal(b, a)
    assert out[0][3] == out[1][3]
    say(f"  refinement {out[1][3]}")


@pytest.mark.parametrize("n,ns,tile,persistent", [(128, 128, 32, True), (2048, 512, 64, True),
                                                   (1000, 300, 128, False), (4096, 1024, 64, False)])
def test_auto_executor_choice_and_bits(ctxs, n, ns, tile, persistent):
    """GPR_EXEC_AUTO runs a sweep of small tiles over a small matrix on the
    persistent executor and everything else on the streams (the profile's
    launch counts show which), with the stream executor's bits either way."""
    from paper_2602_19683_amd import GPR_EXEC_AUTO, Context
    say(f"auto executor n={n} n_test={ns} tile={tile} (persistent expected: {persistent})")
    s, _ = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    mean_s, cov_s, K = s.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile)
    ref = (host(mean_s), host(cov_s))
    K.free()
    with Context(0, executor=GPR_EXEC_AUTO) as a:
        a.profile(True)
        a.profile_read(reset=True)
        mean, cov, K = a.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile)
        got = (host(mean), host(cov))
        assert a.sync()[0] == 0
        prof = a.profile_read(reset=True)
        a.profile(False)
        K.free()
    ran_persistent = prof["persist"][0] > 0
    say(f"  persistent launches {prof['persist'][0]}, potrf launches {prof['potrf'][0]}")
    assert ran_persistent == persistent
    assert (prof["potrf"][0] == 0) == persistent
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])


def test_nlml_and_gradient_bitwise_equal_to_streams(ctxs):
    n, tile, h = 1024, 128, (0.3, 2.0, 0.5)
    say(f"persistent nlml_grad n={n} tile={tile}")
    s, p = ctxs
    X, y = nfir(n, seed=4)
    res = []
    for c in (s, p):
        nl, g, _ = c.nlml_grad(dev(X), dev(y), h, tile)
        assert c.sync()[0] == 0
        res.append((host(nl), host(g)))
    np.testing.assert_array_equal(res[1][0], res[0][0])
    np.testing.assert_array_equal(res[1][1], res[0][1])


def test_failed_pivot_reported_like_streams(ctxs):
    s, p = ctxs
    X, _ = nfir(300, seed=2)
    cols = []
    for c in (s, p):
        K = c.assemble(dev(X), (1.0, 1.0, -2.0), 64)   # diagonal v + s2 = -1
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        c.cholesky(K, info=info)
        st, col = c.sync(raise_on_error=False)
        cols.append((st, col, int(info.item())))
        K.free()
        assert c.sync()[0] == 0
    assert cols[0] == cols[1] and cols[0][0] == 1 and cols[0][2] == 1


def test_repeated_runs_and_profile(ctxs):
    """Several sweeps in a row reuse the cached ticket order and the cleared
    counters; shapes change in between (the order is rebuilt)."""
    s, p = ctxs
    p.profile(True)
    X, y, Xs = nfir_train_test(512, 128)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    first = None
    for tile in (128, 64, 128):
        for _ in range(2):
            mean, cov, K = p.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile)
            got = (host(mean), host(cov))
            assert p.sync()[0] == 0
            K.free()
            if tile == 128:
                if first is None:
                    first = got
                np.testing.assert_array_equal(got[0], first[0])
                np.testing.assert_array_equal(got[1], first[1])
    prof = p.profile_read()
    p.profile(False)
    assert prof["persist"][0] == 6
    assert prof["update"][0] == 0 and prof["potrf"][0] == 0


def test_full_size_bitwise_equal_to_streams(ctxs):
    """n = 16384, n_test = 4096, D = 8, tile 512: one fused sweep per executor."""
    n, ns, tile = 16384, 4096, 512
    say(f"persistent full size n={n} n_test={ns} tile={tile}")
    s, p = ctxs
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    out = []
    for c in (s, p):
        mean, cov, K = c.fit_predict(Xd, yd, Xsd, DEFAULT_HYPER, tile)
        out.append((host(mean), host(cov)))
        assert c.sync()[0] == 0
        K.free()
    np.testing.assert_array_equal(out[1][0], out[0][0])
    np.testing.assert_array_equal(out[1][1], out[0][1])
