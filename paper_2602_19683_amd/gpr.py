"""Python binding of libgpr: argument marshalling for torch tensors on a HIP
device. Every step of the computation runs in the library's HIP kernels;
torch only provides device memory and the current stream."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (GPR_EXEC_STREAMS, GPR_FP64, GPR_MIXED_BF16, GPR_MIXED_FP32, GPR_OK,
                   GPR_ENOTPD, GPR_STATE_K, GPR_STATE_L, Hyper, IRStats)

PRECISIONS = {"fp64": GPR_FP64, "fp32": GPR_MIXED_FP32, "bf16": GPR_MIXED_BF16}


class GPRError(RuntimeError):
    def __init__(self, status, where="", column=0):
        msg = _lib.load().gpr_strerror(status).decode()
        if column:
            msg += f" (column {column})"
        super().__init__(f"{where}: {msg} [status {status}]" if where else msg)
        self.status = status
        self.column = column


def _check(status, where):
    if status != GPR_OK:
        raise GPRError(status, where)

_VARIANTS = {"right": 0, "left": 1}


def _hyper(h):
    if isinstance(h, Hyper):
        return h
    l, v, s2 = (float(t) for t in h)
    return Hyper(l, v, s2)


def _dev_ptr(t, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _ir_dict(st):
    """Refinement statistics as a dict; method "ir" (plain refinement) or "pcg"
    (conjugate gradients preconditioned by the mixed factor took over)."""
    return {"iters": st.iters, "rel_residual": st.rel_residual,
            "precision": st.fallback_precision, "method": "pcg" if st.method == 1 else "ir"}


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _prec(p):
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


class Tiled:
    """Library-owned lower-tiled n x n matrix (K, then its factor L)."""

    def __init__(self, handle, ctx):
        self._h = handle
        self._ctx = ctx

    @property
    def handle(self):
        return self._h

    def info(self):
        n = ctypes.c_int64()
        tile = ctypes.c_int32()
        state = ctypes.c_int32()
        _check(_lib.load().gpr_tiled_info(self._h, ctypes.byref(n), ctypes.byref(tile),
                                          ctypes.byref(state)), "gpr_tiled_info")
        return n.value, tile.value, state.value

    @property
    def n(self):
        return self.info()[0]

    @property
    def tile(self):
        return self.info()[1]

    @property
    def state(self):
        return self.info()[2]

    def free(self):
        if self._h:
            _lib.load().gpr_tiled_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A libgpr context on one GPU (streams, events, workspace)."""

    def __init__(self, device=0, n_streams=3, executor=GPR_EXEC_STREAMS, variant="right"):
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        _check(self._lib.gpr_ctx_create(ctypes.byref(h), int(device), int(n_streams),
                                        int(executor)), "gpr_ctx_create")
        self._h = h
        self.device = device
        self.set_variant(variant)

    def set_variant(self, variant):
        """Task order of the factorisations: "right" (right-looking, Fig. 1)
        or "left" (left-looking)."""
        v = _VARIANTS[variant] if isinstance(variant, str) else int(variant)
        _check(self._lib.gpr_ctx_set_variant(self._h, v), "gpr_ctx_set_variant")
        self.variant = variant

    def close(self):
        if self._h:
            self._lib.gpr_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- hot path -------------------------------------------------------
    def assemble(self, X, hyper, tile, K=None, stream=None):
        n, D = X.shape
        h = ctypes.c_void_p(K.handle.value) if K is not None else ctypes.c_void_p()
        _check(self._lib.gpr_assemble(self._h, _dev_ptr(X, "X"), n, D, _hyper(hyper), int(tile),
                                      ctypes.byref(h), _stream(stream)), "gpr_assemble")
        return K if K is not None else Tiled(h, self)

    def cholesky(self, K, precision="fp64", info=None, stream=None):
        ip = _dev_ptr_int(info) if info is not None else None
        _check(self._lib.gpr_cholesky(self._h, K.handle, _prec(precision), ip, _stream(stream)),
               "gpr_cholesky")
        return K

    def cholesky_dense(self, A, tile, precision="fp64", info=None, stream=None):
        n = A.shape[0]
        ip = _dev_ptr_int(info) if info is not None else None
        _check(self._lib.gpr_cholesky_dense(self._h, _dev_ptr(A, "A", n * n), n, int(tile),
                                            _prec(precision), ip, _stream(stream)),
               "gpr_cholesky_dense")
        return A

    def predict(self, L, X, y, Xs, hyper, full_cov=True, mean=None, cov=None, stream=None,
                ir_stats=False):
        import torch
        n, D = X.shape
        ns = Xs.shape[0]
        if mean is None:
            mean = torch.empty(ns, dtype=torch.float64, device=X.device)
        if full_cov and cov is None:
            cov = torch.empty(ns, ns, dtype=torch.float64, device=X.device)
        st = IRStats()
        _check(self._lib.gpr_predict(self._h, L.handle, _dev_ptr(X, "X"), _dev_ptr(y, "y", n), n,
                                     _dev_ptr(Xs, "Xs"), ns, D, _hyper(hyper),
                                     _dev_ptr(mean, "mean", ns),
                                     _dev_ptr(cov, "cov", ns * ns) if full_cov else None,
                                     ctypes.byref(st), _stream(stream)), "gpr_predict")
        out = (mean, cov if full_cov else None)
        if ir_stats:
            return out + (_ir_dict(st),)
        return out

    def fit_predict(self, X, y, Xs, hyper, tile, precision="fp64", full_cov=True, K=None,
                    mean=None, cov=None, info=None, stream=None, ir_stats=False):
        """Assembly, Cholesky and prediction in one tile sweep. Returns
        (mean, cov, K) where K is the handle now holding the factor."""
        import torch
        n, D = X.shape
        ns = Xs.shape[0]
        if mean is None:
            mean = torch.empty(ns, dtype=torch.float64, device=X.device)
        if full_cov and cov is None:
            cov = torch.empty(ns, ns, dtype=torch.float64, device=X.device)
        h = ctypes.c_void_p(K.handle.value) if K is not None else ctypes.c_void_p()
        ip = _dev_ptr_int(info) if info is not None else None
        st = IRStats()
        _check(self._lib.gpr_fit_predict(self._h, _dev_ptr(X, "X"), _dev_ptr(y, "y", n), n,
                                         _dev_ptr(Xs, "Xs"), ns, D, _hyper(hyper), int(tile),
                                         _prec(precision), ctypes.byref(h),
                                         _dev_ptr(mean, "mean", ns),
                                         _dev_ptr(cov, "cov", ns * ns) if full_cov else None,
                                         ip, ctypes.byref(st), _stream(stream)),
               "gpr_fit_predict")
        K = K if K is not None else Tiled(h, self)
        out = (mean, cov if full_cov else None, K)
        if ir_stats:
            return out + (_ir_dict(st),)
        return out

    def predict_var(self, L, X, y, Xs, hyper, full_cov=False, mean=None, var=None, cov=None,
                    stream=None, ir_stats=False):
        """Mean and predictive variances (and the full covariance if asked)
        with the factor in L. Returns (mean, var, cov or None)."""
        import torch
        n, D = X.shape
        ns = Xs.shape[0]
        mean = mean if mean is not None else torch.empty(ns, dtype=torch.float64, device=X.device)
        var = var if var is not None else torch.empty(ns, dtype=torch.float64, device=X.device)
        if full_cov and cov is None:
            cov = torch.empty(ns, ns, dtype=torch.float64, device=X.device)
        st = IRStats()
        _check(self._lib.gpr_predict_var(self._h, L.handle, _dev_ptr(X, "X"), _dev_ptr(y, "y", n),
                                         n, _dev_ptr(Xs, "Xs"), ns, D, _hyper(hyper),
                                         _dev_ptr(mean, "mean", ns),
                                         _dev_ptr(cov, "cov", ns * ns) if full_cov else None,
                                         _dev_ptr(var, "var", ns), ctypes.byref(st),
                                         _stream(stream)), "gpr_predict_var")
        out = (mean, var, cov if full_cov else None)
        if ir_stats:
            return out + (_ir_dict(st),)
        return out

    def fit_predict_var(self, X, y, Xs, hyper, tile, precision="fp64", full_cov=False, K=None,
                        mean=None, var=None, cov=None, info=None, stream=None, ir_stats=False):
        """Assembly, Cholesky, mean and predictive variances (and the full
        covariance if asked) in one sweep. Returns (mean, var, cov or None, K)."""
        import torch
        n, D = X.shape
        ns = Xs.shape[0]
        mean = mean if mean is not None else torch.empty(ns, dtype=torch.float64, device=X.device)
        var = var if var is not None else torch.empty(ns, dtype=torch.float64, device=X.device)
        if full_cov and cov is None:
            cov = torch.empty(ns, ns, dtype=torch.float64, device=X.device)
        h = ctypes.c_void_p(K.handle.value) if K is not None else ctypes.c_void_p()
        ip = _dev_ptr_int(info) if info is not None else None
        st = IRStats()
        _check(self._lib.gpr_fit_predict_var(self._h, _dev_ptr(X, "X"), _dev_ptr(y, "y", n), n,
                                             _dev_ptr(Xs, "Xs"), ns, D, _hyper(hyper), int(tile),
                                             _prec(precision), ctypes.byref(h),
                                             _dev_ptr(mean, "mean", ns),
                                             _dev_ptr(cov, "cov", ns * ns) if full_cov else None,
                                             _dev_ptr(var, "var", ns), ip, ctypes.byref(st),
                                             _stream(stream)), "gpr_fit_predict_var")
        K = K if K is not None else Tiled(h, self)
        out = (mean, var, cov if full_cov else None, K)
        if ir_stats:
            return out + (_ir_dict(st),)
        return out

    def solve(self, L, b, x=None, stream=None):
        """x = K^{-1} b with the factor held by L."""
        import torch
        n = L.n
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=b.device)
        _check(self._lib.gpr_solve(self._h, L.handle, _dev_ptr(b, "b", n), _dev_ptr(x, "x", n),
                                   _stream(stream)), "gpr_solve")
        return x

    def solve_noalloc(self, L, b, x, stream=None):
        """x = K^{-1} b like solve(), into the caller's x, with no device
        allocation in the library (work vectors in its fixed per-GPU array;
        overlapping calls on one GPU race)."""
        n = L.n
        _check(self._lib.gpr_solve_noalloc(self._h, L.handle, _dev_ptr(b, "b", n),
                                           _dev_ptr(x, "x", n), _stream(stream)),
               "gpr_solve_noalloc")
        return x

    def nlml_grad(self, X, y, hyper, tile, precision="fp64", grad=True, kbar=False,
                  out_nlml=None, out_grad=None, out_kbar=None, stream=None):
        """NLML and (if grad) its gradient in the order (l, v, sigma^2), as
        device tensors; with kbar also the dense symmetric adjoint
        1/2 (K^{-1} - alpha alpha^T). Returns (nlml[1], grad[3] or None,
        kbar[n, n] or None)."""
        import torch
        n, D = X.shape
        if out_nlml is None:
            out_nlml = torch.empty(1, dtype=torch.float64, device=X.device)
        if grad and out_grad is None:
            out_grad = torch.empty(3, dtype=torch.float64, device=X.device)
        if kbar and out_kbar is None:
            out_kbar = torch.empty(n, n, dtype=torch.float64, device=X.device)
        _check(self._lib.gpr_nlml_grad(self._h, _dev_ptr(X, "X"), _dev_ptr(y, "y", n), n, D,
                                       _hyper(hyper), int(tile), _prec(precision),
                                       _dev_ptr(out_nlml, "out_nlml", 1),
                                       _dev_ptr(out_grad, "out_grad", 3) if grad else None,
                                       _dev_ptr(out_kbar, "out_kbar", n * n) if kbar else None,
                                       _stream(stream)),
               "gpr_nlml_grad")
        return out_nlml, (out_grad if grad else None), (out_kbar if kbar else None)

    def fit_hyper(self, X, y, theta0, tile, max_steps=20, lr=0.05, betas=(0.9, 0.999),
                  eps=1e-8, tol=0.0, stream=None):
        """Adam on log theta from theta0 = (l, v, sigma^2), each step one GPU
        NLML-and-gradient evaluation (gpr_fit_hyper). Returns (theta (numpy, 3),
        NLML before each step (numpy), steps taken)."""
        n, D = X.shape
        th0 = (ctypes.c_double * 3)(*[float(v) for v in theta0])
        out = (ctypes.c_double * 3)()
        trace = (ctypes.c_double * int(max_steps))()
        done = ctypes.c_int32(0)
        _check(self._lib.gpr_fit_hyper(self._h, _dev_ptr(X, "X"), _dev_ptr(y, "y", n), n, D,
                                       int(tile), th0, int(max_steps), float(lr),
                                       float(betas[0]), float(betas[1]), float(eps), float(tol),
                                       out, trace, ctypes.byref(done), _stream(stream)),
               "gpr_fit_hyper")
        k = done.value
        return np.array(out[:]), np.array(trace[:k]), k

    def fit_hyper_restarts(self, X, y, starts, tile, **kw):
        """fit_hyper from each theta0 in starts; returns the fit (theta, trace,
        steps) whose last NLML is lowest, and the index of its start."""
        best, best_i = None, -1
        for i, th0 in enumerate(starts):
            r = self.fit_hyper(X, y, th0, tile, **kw)
            if best is None or r[1][-1] < best[1][-1]:
                best, best_i = r, i
        return best, best_i

    # ---- instrumentation --------------------------------------------------
    PROFILE_KINDS = ("potrf", "trtri", "trsm", "update", "assemble", "trsv", "matvec", "export",
                     "adjoint", "reduce", "persist")

    def profile(self, on=True):
        _check(self._lib.gpr_profile_enable(self._h, int(bool(on))), "gpr_profile_enable")

    def profile_read(self, reset=True):
        """{kind: (launches, total_ms, flops, bytes)} since the last reset."""
        out = {}
        for k, name in enumerate(self.PROFILE_KINDS):
            nl = ctypes.c_int64()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            last = reset and k == len(self.PROFILE_KINDS) - 1
            _check(self._lib.gpr_profile_read(self._h, k, ctypes.byref(nl), ctypes.byref(ms),
                                              ctypes.byref(fl), ctypes.byref(by), int(last)),
                   "gpr_profile_read")
            out[name] = (nl.value, ms.value, fl.value, by.value)
        return out

    # ---- utilities ------------------------------------------------------
    def to_dense(self, T, out=None, stream=None):
        import torch
        n = T.n
        if out is None:
            out = torch.empty(n, n, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(self._lib.gpr_tiled_to_dense(self._h, T.handle, _dev_ptr(out, "out", n * n),
                                            _stream(stream)), "gpr_tiled_to_dense")
        return out

    def sync(self, stream=None, raise_on_error=True):
        col = ctypes.c_int64()
        st = self._lib.gpr_sync(self._h, _stream(stream), ctypes.byref(col))
        if st != GPR_OK and raise_on_error:
            raise GPRError(st, "gpr_sync", col.value)
        return st, col.value


def _dev_ptr_int(t):
    import torch
    if t.dtype != torch.int32 or not t.is_cuda or t.numel() < 1:
        raise ValueError("info must be an int32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def schedule_describe(M, Mhat, mode, variant=None):
    """Host-only: the batched launch list of the tile sweep (see gpr.h).

    Returns ``(tasks, launches)``: int32 arrays of shape (T, 5) = (kind, I, K,
    J, launch) and (L, 5) = (stream, wait0, wait1, wait2, launch kind). With
    a variant (0 / "right", 1 / "left"): tasks of shape (T, 6) = (kind, I, K,
    J, nk, launch), an update task holding the products of columns
    J .. J + nk - 1."""
    lib = _lib.load()
    if variant is not None:
        v = _VARIANTS[variant] if isinstance(variant, str) else int(variant)
        nt = ctypes.c_int64()
        nl = ctypes.c_int64()
        st = lib.gpr_schedule_describe_variant(M, Mhat, mode, v, None, 0, ctypes.byref(nt), None,
                                               0, ctypes.byref(nl))
        if st not in (GPR_OK, _lib.GPR_EINVAL) or nt.value < 0:
            raise GPRError(st, "gpr_schedule_describe_variant")
        tasks = np.zeros((nt.value, 6), dtype=np.int32)
        launches = np.zeros((nl.value, 5), dtype=np.int32)
        _check(lib.gpr_schedule_describe_variant(
            M, Mhat, mode, v, tasks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nt.value,
            ctypes.byref(nt), launches.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nl.value,
            ctypes.byref(nl)), "gpr_schedule_describe_variant")
        return tasks, launches
    nt = ctypes.c_int64()
    nl = ctypes.c_int64()
    st = lib.gpr_schedule_describe(M, Mhat, mode, None, 0, ctypes.byref(nt), None, 0,
                                   ctypes.byref(nl))
    if st not in (GPR_OK, _lib.GPR_EINVAL) or nt.value < 0:
        raise GPRError(st, "gpr_schedule_describe")
    tasks = np.zeros((nt.value, 5), dtype=np.int32)
    launches = np.zeros((nl.value, 5), dtype=np.int32)
    _check(lib.gpr_schedule_describe(M, Mhat, mode,
                                     tasks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     nt.value, ctypes.byref(nt),
                                     launches.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     nl.value, ctypes.byref(nl)), "gpr_schedule_describe")
    return tasks, launches


def solve_plan_describe(M, tile):
    """Host-only: the tile products that build the group inverses of the
    vector solves (see gpr.h). Returns ``(G, tasks, terms)``: the group size
    and int32 arrays of shape (T, 6) = (launch, out kind, out a, out b,
    first_term, nterm) and (R, 7) = (A kind, a, b, B kind, a, b, alpha)."""
    lib = _lib.load()
    g, nt, nr = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    st = lib.gpr_solve_plan_describe(M, tile, ctypes.byref(g), None, 0, ctypes.byref(nt), None, 0,
                                     ctypes.byref(nr))
    if st != GPR_OK:
        raise GPRError(st, "gpr_solve_plan_describe")
    tasks = np.zeros((nt.value, 6), dtype=np.int32)
    terms = np.zeros((nr.value, 7), dtype=np.int32)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    _check(lib.gpr_solve_plan_describe(M, tile, ctypes.byref(g), ip(tasks), nt.value,
                                       ctypes.byref(nt), ip(terms), nr.value, ctypes.byref(nr)),
           "gpr_solve_plan_describe")
    return g.value, tasks, terms


def adjoint_describe(M, G):
    """Host-only: the launch list of the reverse sweep of gpr_nlml_grad (see
    gpr.h). Returns ``(tasks, terms, launches)``: int32 arrays of shape
    (T, 12), (R, 8) and (L, 6)."""
    lib = _lib.load()
    nt, nr, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = lib.gpr_adjoint_describe(M, G, None, 0, ctypes.byref(nt), None, 0, ctypes.byref(nr),
                                  None, 0, ctypes.byref(nl))
    if st not in (GPR_OK, _lib.GPR_EINVAL) or nt.value < 0:
        raise GPRError(st, "gpr_adjoint_describe")
    tasks = np.zeros((nt.value, 12), dtype=np.int32)
    terms = np.zeros((nr.value, 8), dtype=np.int32)
    launches = np.zeros((nl.value, 6), dtype=np.int32)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    _check(lib.gpr_adjoint_describe(M, G, ip(tasks), nt.value, ctypes.byref(nt), ip(terms),
                                    nr.value, ctypes.byref(nr), ip(launches), nl.value,
                                    ctypes.byref(nl)), "gpr_adjoint_describe")
    return tasks, terms, launches


def persist_describe(M, Mhat, mode, tile, block, workers):
    """Host-only: the ticket order of the persistent executor (see gpr.h).
    Returns ``(items, waits)``: int32 (N, 5) = (kind, sub, I, K, J) and
    int64 (N, 8) = (number of waits, (counter, value) x 3, signalled counter)."""
    lib = _lib.load()
    n = ctypes.c_int64()
    st = lib.gpr_persist_describe(M, Mhat, mode, tile, block, workers, None, None, 0,
                                  ctypes.byref(n))
    if st not in (GPR_OK, _lib.GPR_EINVAL) or n.value <= 0 and st != GPR_OK:
        raise GPRError(st, "gpr_persist_describe")
    items = np.zeros((n.value, 5), dtype=np.int32)
    waits = np.zeros((n.value, 8), dtype=np.int64)
    _check(lib.gpr_persist_describe(M, Mhat, mode, tile, block, workers,
                                    items.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    waits.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    n.value, ctypes.byref(n)), "gpr_persist_describe")
    return items, waits


class NLML:
    """Differentiable NLML of the exact GP with the squared-exponential kernel:
    ``NLML.apply(theta, X, y, ctx, tile)`` with ``theta = (l, v, sigma^2)`` a
    float64 tensor of 3 entries. The forward pass runs gpr_nlml_grad on the
    GPU, with the reverse sweep when theta requires a gradient; the backward
    pass scales that gradient (no further device work). Returns a 0-d tensor
    on theta's device."""

    _fn = None

    @classmethod
    def apply(cls, theta, X, y, ctx, tile):
        if cls._fn is None:
            cls._fn = _make_nlml_function()
        return cls._fn.apply(theta, X, y, ctx, tile)


def _make_nlml_function():
    import torch

    class _NLMLFunction(torch.autograd.Function):
        @staticmethod
        def forward(fctx, theta, X, y, ctx, tile):
            th = [float(t) for t in theta.detach().cpu().tolist()]
            want = theta.requires_grad
            nl, g, _ = ctx.nlml_grad(X, y, th, tile, grad=want)
            ctx.sync()
            fctx.save_for_backward(g.to(theta.device) if want else theta.new_zeros(3))
            return nl.reshape(()).to(theta.device)

        @staticmethod
        def backward(fctx, gout):
            (g,) = fctx.saved_tensors
            return gout * g, None, None, None, None

    return _NLMLFunction
