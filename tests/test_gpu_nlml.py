"""NLML and its gradient on the GPU (gpr_nlml_grad) against the oracle.

* NLML: relative error <= 1e-12 against the double oracle.
* Gradient in (l, v, sigma^2): normwise relative error <= 1e-9 against the
  oracle's trace formula (a different route: explicit L^{-1}, K^{-1} and
  1/2 tr((K^{-1} - alpha alpha^T) dK)), and <= 1e-6 against central finite
  differences of the GPU's own NLML with h = 1e-5 and h = 1e-6.
* The adjoint of K itself, 1/2 (K^{-1} - alpha alpha^T), element by element
  against the oracle's factor (K^{-1} from its triangular solves): max
  abs error <= 1e-10 of the largest entry.
* The 20-step Adam fit in log space from (0.3, 2.0, 0.5) through the
  torch.autograd.Function, step by step against the oracle's replay.
"""
import numpy as np
import pytest

import oracle
from gpr_inputs import DEFAULT_HYPER, nfir

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C4_HYPER = (0.3, 2.0, 0.5)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19683_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def nrel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_nlml(ctx, Xd, yd, h, tile, grad=True, kbar=False):
    nl, g, kb = ctx.nlml_grad(Xd, yd, h, tile, grad=grad, kbar=kbar)
    assert ctx.sync()[0] == 0
    out = [float(host(nl)[0])]
    out.append(host(g) if grad else None)
    out.append(host(kb) if kbar else None)
    return out


def fd_grad(ctx, Xd, yd, h, tile, step):
    g = np.zeros(3)
    for i in range(3):
        hp, hm = list(h), list(h)
        hp[i] += step
        hm[i] -= step
        fp = gpu_nlml(ctx, Xd, yd, hp, tile, grad=False)[0]
        fm = gpu_nlml(ctx, Xd, yd, hm, tile, grad=False)[0]
        g[i] = (fp - fm) / (2 * step)
    return g


@pytest.mark.parametrize("n,tile,h", [(32, 32, DEFAULT_HYPER), (128, 32, DEFAULT_HYPER),
                                      (150, 32, C4_HYPER), (100, 64, (2.0, 0.7, 0.01)),
                                      (512, 128, C4_HYPER), (1000, 256, DEFAULT_HYPER),
                                      (1024, 256, C4_HYPER), (777, 128, (0.5, 1.5, 0.05))])
def test_nlml_grad_matches_oracle(ctx, n, tile, h):
    say(f"nlml_grad n={n} tile={tile} h={h}")
    X, y = nfir(n, seed=3 * n + tile)
    nl, g, kb = gpu_nlml(ctx, dev(X), dev(y), h, tile, kbar=True)
    nl_ref, g_ref = oracle.nlml_grad(X, y, h)
    e_nl = abs(nl - nl_ref) / abs(nl_ref)
    e_g = nrel(g, g_ref)
    # adjoint of K, entry by entry
    K = oracle.assemble_K(X, h)
    L, info = oracle.cholesky(K)
    assert info == 0
    alpha = oracle.backward(L, oracle.forward(L, y))
    Kinv = np.column_stack([oracle.backward(L, oracle.forward(L, e)) for e in np.eye(n)])
    kb_ref = 0.5 * (Kinv - np.outer(alpha, alpha))
    e_kb = np.abs(kb - kb_ref).max() / np.abs(kb_ref).max()
    say(f"  nlml {nl:.12e} rel {e_nl:.2e}; grad {g} rel {e_g:.2e}; Kbar max rel {e_kb:.2e}")
    assert e_nl <= 1e-12
    assert e_g <= 1e-9
    assert e_kb <= 1e-10
    np.testing.assert_array_equal(kb, kb.T)


def test_nlml_only_and_determinism(ctx):
    n, tile = 700, 128
    X, y = nfir(n, seed=11)
    Xd, yd = dev(X), dev(y)
    a = gpu_nlml(ctx, Xd, yd, C4_HYPER, tile)
    b = gpu_nlml(ctx, Xd, yd, C4_HYPER, tile)
    c = gpu_nlml(ctx, Xd, yd, C4_HYPER, tile, grad=False)
    assert a[0] == b[0] == c[0]
    np.testing.assert_array_equal(a[1], b[1])


def test_not_positive_definite_gives_nan_and_enotpd(ctx):
    from paper_2602_19683_amd import GPR_ENOTPD
    n, tile = 96, 32
    X, y = nfir(n, seed=5)
    X[7] = X[3]  # two equal points and no noise: K is singular
    nl, g, _ = ctx.nlml_grad(dev(X), dev(y), (1.0, 1.0, -0.5), tile)
    st, col = ctx.sync(raise_on_error=False)
    assert st == GPR_ENOTPD and col >= 1
    assert np.isnan(host(nl)).all() and np.isnan(host(g)).all()
    # the context recovers
    nl2 = gpu_nlml(ctx, dev(X), dev(y), DEFAULT_HYPER, tile, grad=False)[0]
    assert np.isfinite(nl2)


@pytest.mark.parametrize("h", [C4_HYPER, DEFAULT_HYPER])
def test_gradient_matches_finite_differences(ctx, h):
    n, tile = 2048, 256
    say(f"finite differences n={n} tile={tile} h={h}")
    X, y = nfir(n, seed=17)
    Xd, yd = dev(X), dev(y)
    _, g, _ = gpu_nlml(ctx, Xd, yd, h, tile)
    for step in (1e-5, 1e-6):
        gfd = fd_grad(ctx, Xd, yd, h, tile, step)
        e = nrel(g, gfd)
        say(f"  step {step}: adjoint {g} fd {gfd} rel {e:.2e}")
        assert e <= 1e-6


@pytest.mark.slow
def test_full_size_c4(ctx):
    """n = 8192, D = 8, tile 256 at (0.3, 2.0, 0.5): oracle and finite differences."""
    n, tile, h = 8192, 256, C4_HYPER
    say(f"C4 n={n} tile={tile} h={h}")
    X, y = nfir(n)
    Xd, yd = dev(X), dev(y)
    nl, g, _ = gpu_nlml(ctx, Xd, yd, h, tile)
    say("  GPU done; oracle running")
    nl_ref, g_ref = oracle.nlml_grad(X, y, h)
    gfd = fd_grad(ctx, Xd, yd, h, tile, 1e-5)
    say(f"  nlml {nl!r} oracle {nl_ref!r}; grad {g} oracle {g_ref} fd {gfd}")
    assert abs(nl - nl_ref) / abs(nl_ref) <= 1e-12
    assert nrel(g, g_ref) <= 1e-9
    assert nrel(g, gfd) <= 1e-6


def test_adam_fit_through_autograd_matches_oracle(ctx):
    """20 Adam steps on log theta (lr 0.05) from (0.3, 2.0, 0.5): the GPU
    NLML and gradient behind torch.autograd and torch.optim.Adam, against the
    oracle's replay of the same optimiser."""
    from paper_2602_19683_amd import NLML
    n, tile = 1024, 256
    X, y = nfir(n)
    Xd, yd = dev(X), dev(y)
    z = torch.tensor(np.log(C4_HYPER), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([z], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    gpu_trace = []
    for _ in range(20):
        opt.zero_grad()
        theta = torch.exp(z)
        f = NLML.apply(theta, Xd, yd, ctx, tile)
        f.backward()
        gpu_trace.append((theta.detach().numpy().copy(), float(f.detach())))
        opt.step()
    ref_trace, ref_final = oracle.adam_fit(X, y, C4_HYPER, steps=20)
    worst = 0.0
    for (tg, fg), (tr, fr) in zip(gpu_trace, ref_trace):
        worst = max(worst, abs(fg - fr) / abs(fr))
        assert np.allclose(tg, tr, rtol=1e-9, atol=0)
    say(f"Adam: NLML {gpu_trace[0][1]:.6f} -> {gpu_trace[-1][1]:.6f}, worst step rel {worst:.2e}")
    assert worst <= 1e-8
    assert gpu_trace[-1][1] < gpu_trace[0][1]
    np.testing.assert_allclose(torch.exp(z).detach().numpy(), ref_final, rtol=1e-8)


def test_fit_hyper_matches_oracle_adam(ctx):
    """gpr_fit_hyper: 20 Adam steps on log theta from (0.3, 2.0, 0.5), each a
    GPU NLML-and-gradient evaluation, against the oracle's replay of the same
    optimiser (NLML before each step to 1e-8, final theta to 1e-8)."""
    n, tile = 1024, 256
    X, y = nfir(n)
    Xd, yd = dev(X), dev(y)
    theta, trace, steps = ctx.fit_hyper(Xd, yd, C4_HYPER, tile, max_steps=20)
    ref_trace, ref_final = oracle.adam_fit(X, y, C4_HYPER, steps=20)
    assert steps == 20 and len(trace) == 20
    worst = max(abs(f - fr) / abs(fr) for f, (_, fr) in zip(trace, ref_trace))
    say(f"fit_hyper: NLML {trace[0]:.6f} -> {trace[-1]:.6f}, worst step rel {worst:.2e}, "
        f"theta {theta}")
    assert worst <= 1e-8
    np.testing.assert_allclose(theta, ref_final, rtol=1e-8)
    assert trace[-1] < trace[0]


def test_fit_hyper_tolerance_and_restarts(ctx):
    """Stopping on the relative NLML change, and the best of several starts.
    The trajectory does not depend on the stopping rule, so the first 20
    NLMLs equal those of a 20-step run bit for bit."""
    n, tile = 1024, 256
    X, y = nfir(n)
    Xd, yd = dev(X), dev(y)
    _, tr20, _ = ctx.fit_hyper(Xd, yd, C4_HYPER, tile, max_steps=20)
    tol, cap = 1e-4, 200
    theta, trace, steps = ctx.fit_hyper(Xd, yd, C4_HYPER, tile, max_steps=cap, tol=tol)
    say(f"fit_hyper tol {tol}: {steps} steps, NLML {trace[0]:.6f} -> {trace[-1]:.6f}, "
        f"theta {theta}")
    k0 = min(steps, 20)
    np.testing.assert_array_equal(trace[:k0], tr20[:k0])
    assert 1 <= steps <= cap and len(trace) == steps
    # the rule: no earlier step met the tolerance; a stop before the cap met it
    assert all(abs(trace[k] - trace[k - 1]) > tol * abs(trace[k - 1]) for k in range(1, steps - 1))
    if steps < cap:
        assert abs(trace[-1] - trace[-2]) <= tol * abs(trace[-2])
    assert trace[-1] < trace[0]
    starts = [C4_HYPER, (1.0, 1.0, 0.1), (3.0, 0.5, 1.0)]
    (tb, trb, kb), ib = ctx.fit_hyper_restarts(Xd, yd, starts, tile, max_steps=30)
    finals = [ctx.fit_hyper(Xd, yd, s, tile, max_steps=30)[1][-1] for s in starts]
    say(f"restarts: final NLMLs {finals}, best start {ib}")
    assert ib == int(np.argmin(finals)) and trb[-1] == min(finals)
