"""Error paths of the C ABI that need a device: the device-memory cap
(GPR_MAX_DEVICE_BYTES -> GPR_ENOMEM) and the handle-state checks (a handle
that holds K, not a factor, is refused by the calls that need L, and a factor
is refused by the factorisation)."""
import numpy as np
import pytest

from gpr_inputs import DEFAULT_HYPER, nfir, nfir_train_test

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_device_cap_gives_enomem(monkeypatch):
    from paper_2602_19683_amd import Context, GPRError, _lib
    cap = 32 << 20
    monkeypatch.setenv("GPR_MAX_DEVICE_BYTES", str(cap))
    X, y, Xs = nfir_train_test(4096, 64)
    with Context(0) as ctx:          # the cap is read when the context is created
        # K of n = 4096 in tiles of 256: 136 tiles of 512 KiB = 68 MiB > 32 MiB
        say(f"cap {cap} bytes: assemble n=4096 tile 256 must fail")
        with pytest.raises(GPRError) as e:
            ctx.assemble(dev(X), DEFAULT_HYPER, 256)
        assert e.value.status == _lib.GPR_ENOMEM
        # a problem within the cap still runs, and exactly
        n = 1024
        Xd, yd, Xsd = dev(X[:n]), dev(y[:n]), dev(Xs)
        K = ctx.assemble(Xd, DEFAULT_HYPER, 128)
        ctx.cholesky(K)
        mean, cov = ctx.predict(K, Xd, yd, Xsd, DEFAULT_HYPER)
        assert ctx.sync()[0] == 0
        import oracle
        ref = oracle.predict(X[:n], y[:n], Xs, DEFAULT_HYPER, want=("mean", "cov"))
        assert oracle.rel_err(mean.cpu().numpy(), ref["mean"]) <= 1e-10
        # about 8 MiB held now (K, its inverses, the prediction workspace);
        # K of n = 2048 in tiles of 256 takes 18 MiB: one fits, a second is
        # refused, and freeing the first makes room again
        K2 = ctx.assemble(dev(X[:2048]), DEFAULT_HYPER, 256)
        with pytest.raises(GPRError) as e:
            ctx.assemble(dev(X[:2048]), DEFAULT_HYPER, 256)
        assert e.value.status == _lib.GPR_ENOMEM
        K2.free()
        K3 = ctx.assemble(dev(X[:2048]), DEFAULT_HYPER, 256)
        assert ctx.sync()[0] == 0
        K3.free()
        K.free()
    monkeypatch.delenv("GPR_MAX_DEVICE_BYTES")
    with Context(0) as ctx:          # no cap: the large case runs
        K = ctx.assemble(dev(X), DEFAULT_HYPER, 256)
        assert ctx.sync()[0] == 0
        K.free()


def test_handle_state_checks():
    from paper_2602_19683_amd import Context, GPRError, _lib
    n, ns, tile = 300, 40, 64
    X, y, Xs = nfir_train_test(n, ns)
    Xd, yd, Xsd = dev(X), dev(y), dev(Xs)
    with Context(0) as ctx:
        K = ctx.assemble(Xd, DEFAULT_HYPER, tile)      # holds K, not a factor
        say("predict / predict_var / solve on an unfactored handle must be refused")
        for call in (lambda: ctx.predict(K, Xd, yd, Xsd, DEFAULT_HYPER),
                     lambda: ctx.predict_var(K, Xd, yd, Xsd, DEFAULT_HYPER),
                     lambda: ctx.solve(K, yd)):
            with pytest.raises(GPRError) as e:
                call()
            assert e.value.status == _lib.GPR_EINVAL
        ctx.cholesky(K)
        say("cholesky of a handle that already holds a factor must be refused")
        with pytest.raises(GPRError) as e:
            ctx.cholesky(K)
        assert e.value.status == _lib.GPR_EINVAL
        # a factor for another n is refused by predict
        Xo, yo = nfir(n + 1)
        with pytest.raises(GPRError) as e:
            ctx.predict(K, dev(Xo), dev(yo), Xsd, DEFAULT_HYPER)
        assert e.value.status == _lib.GPR_EINVAL
        # the handle is still usable as a factor
        mean, _ = ctx.predict(K, Xd, yd, Xsd, DEFAULT_HYPER, full_cov=False)
        assert ctx.sync()[0] == 0
        assert np.all(np.isfinite(mean.cpu().numpy()))
        K.free()
