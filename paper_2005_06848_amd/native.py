"""ctypes binding of libcfust.so (same names as the C ABI).

Tensors must be float64, contiguous, on the GPU.  The functions return torch
tensors on the same device; errors raise ``CfustError``.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import _build

LIB_PATH = _build.LIB_PATH

OK, EINVAL, ENOTPD, ENONFINITE, EHIP, ENOMEM = 0, 1, 2, 3, 4, 5
FP64, FP32 = 0, 1
NU_OSL, NU_EXACT, NU_FIXED = 0, 1, 2


class CfustError(RuntimeError):
    def __init__(self, code, where, bad=-1):
        msg = _lib().cfust_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code}, component {bad})")
        self.code = code
        self.bad = bad


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("nu_mode", ctypes.c_int),
        ("fix_delta_zero", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("nu_lo", ctypes.c_double),
        ("nu_hi", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("prof_ms", ctypes.c_void_p),
        ("graph", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("surrogate", ctypes.c_void_p),
        ("adapt_samples", ctypes.c_int),
        ("adapt_epochs", ctypes.c_int),
        ("reorder", ctypes.c_int),
        ("surrogate_check", ctypes.c_int),
        ("surrogate_switch", ctypes.c_double),
    ]


PROF_SLOTS = 4


def prof_buffer():
    """Host accumulator for the library's per-kernel HIP-event times (ms)."""
    return (ctypes.c_double * PROF_SLOTS)()


class EstepOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("tau", "logf", "e1", "e2", "e3", "e4", "stats", "loglik")] + [
        ("bad_component", ctypes.c_int)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2005_06848_amd._build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, i, i64, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        L.cfust_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.cfust_default_opts.restype = None
        L.cfust_stats_size.argtypes = [i, i]
        L.cfust_stats_size.restype = i
        L.cfust_workspace_size.argtypes = [i64, i, i, i, i, i, ctypes.POINTER(sz)]
        L.cfust_workspace_size.restype = i
        L.cfust_workspace_size_opts.argtypes = [i64, i, i, i, i, ctypes.POINTER(Opts),
                                                ctypes.POINTER(sz)]
        L.cfust_workspace_size_opts.restype = i
        L.cfust_estep.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, ctypes.POINTER(Opts),
                                  ctypes.POINTER(EstepOut)]
        L.cfust_estep.restype = i
        L.cfust_estep_noalloc.argtypes = L.cfust_estep.argtypes
        L.cfust_estep_noalloc.restype = i
        L.cfust_mstep.argtypes = [P, i64, i, i, i, P, P, P, ctypes.POINTER(Opts), P, P, P, P, P,
                                  ctypes.POINTER(i)]
        L.cfust_mstep.restype = i
        L.cfust_loglik.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, ctypes.POINTER(Opts), P, P]
        L.cfust_loglik.restype = i
        L.cfust_em_fit.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, ctypes.POINTER(Opts), P,
                                   ctypes.POINTER(i), ctypes.POINTER(i)]
        L.cfust_em_fit.restype = i
        L.cfust_aitken_linf.argtypes = [d, d, d]
        L.cfust_aitken_linf.restype = d
        L.cfust_eval_special.argtypes = [i, P, P, P, i64, P]
        L.cfust_eval_special.restype = i
        L.cfust_em_fit_batched.argtypes = [P, i, i, i, P, P, P, P, P, P, P, P, i,
                                           ctypes.POINTER(Opts), P, P, P]
        L.cfust_em_fit_batched.restype = i
        L.cfust_loglik_rqmc.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, i,
                                        ctypes.POINTER(Opts), P, ctypes.POINTER(d),
                                        ctypes.POINTER(d)]
        L.cfust_loglik_rqmc.restype = i
        L.cfust_em_fit_multistart.argtypes = [P, i64, i, i, i, i, P, P, P, P, P, P, i, i,
                                              ctypes.POINTER(Opts), P, P, P, P, P, P,
                                              ctypes.POINTER(i), P, ctypes.POINTER(i),
                                              ctypes.POINTER(i)]
        L.cfust_em_fit_multistart.restype = i
        L.cfust_batched_workspace_size.argtypes = [i, i, i, P, P, i, i, i, ctypes.POINTER(sz)]
        L.cfust_batched_workspace_size.restype = i
        ip = ctypes.POINTER(i)
        L.cfust_batched_config.argtypes = [ip, ip, ip, ip, ip, ctypes.POINTER(d)]
        L.cfust_batched_config.restype = i
        L.cfust_batched_shape.argtypes = [i, ip, ip, ip, ip]
        L.cfust_batched_shape.restype = i
        L.cfust_ghk_batch.argtypes = [i, i64, P, P, P, P, i, ctypes.POINTER(Opts), P]
        L.cfust_ghk_batch.restype = i
        f32p = ctypes.POINTER(ctypes.c_float)
        L.cfust_surrogate_create.argtypes = [i, ctypes.POINTER(d), ctypes.c_ulonglong,
                                             ctypes.POINTER(P)]
        L.cfust_surrogate_create.restype = i
        L.cfust_surrogate_destroy.argtypes = [P]
        L.cfust_surrogate_destroy.restype = None
        L.cfust_surrogate_train.argtypes = [P, P, P, i64, i, i, d, d, ctypes.c_ulonglong, f32p,
                                            ctypes.POINTER(Opts), ctypes.POINTER(d)]
        L.cfust_surrogate_train.restype = i
        L.cfust_surrogate_grad.argtypes = [P, P, P, i64, f32p, ctypes.POINTER(Opts), f32p,
                                           ctypes.POINTER(d)]
        L.cfust_surrogate_grad.restype = i
        L.cfust_surrogate_eval.argtypes = [P, P, i64, ctypes.POINTER(Opts), P]
        L.cfust_surrogate_eval.restype = i
        L.cfust_surrogate_get_state.argtypes = [P, f32p, f32p]
        L.cfust_surrogate_get_state.restype = i
        L.cfust_surrogate_set_state.argtypes = [P, f32p, f32p]
        L.cfust_surrogate_set_state.restype = i
        L.cfust_surrogate_save.argtypes = [P, ctypes.c_char_p]
        L.cfust_surrogate_save.restype = i
        L.cfust_surrogate_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(P)]
        L.cfust_surrogate_load.restype = i
        L.cfust_surrogate_fallback_count.argtypes = [P]
        L.cfust_surrogate_fallback_count.restype = i64
        L.cfust_surrogate_adapt.argtypes = [P, P, i64, i, i, i, P, P, P, P, P, P, i, i64, i,
                                            ctypes.c_ulonglong, ctypes.POINTER(Opts),
                                            ctypes.POINTER(d), ctypes.POINTER(i64)]
        L.cfust_surrogate_adapt.restype = i
        L.cfust_surrogate_em_switch.argtypes = [P]
        L.cfust_surrogate_em_switch.restype = i
        L.cfust_pair_features.argtypes = [P, i64, i, i, i, P, P, P, P, P, ctypes.POINTER(Opts), P]
        L.cfust_pair_features.restype = i
        L.cfust_mlp_gemm.argtypes = [i, i, i, i, i, P, P, P, P]
        L.cfust_mlp_gemm.restype = i
        L.cfust_strerror.argtypes = [i]
        L.cfust_strerror.restype = ctypes.c_char_p
        L.cfust_opts_size.argtypes = []
        L.cfust_opts_size.restype = sz
        if L.cfust_opts_size() != ctypes.sizeof(Opts):
            raise ImportError(f"{LIB_PATH}: cfust_opts is {L.cfust_opts_size()} bytes in the "
                              f"library but {ctypes.sizeof(Opts)} in this binding (stale build?)")
        _LIB = L
    return _LIB


def lib():
    return _lib()


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_opts(precision="fp64", nu_mode="osl", fix_delta_zero=False, max_iter=100, tol=1e-6,
              nu_lo=1.0, nu_hi=200.0, stream=None, workspace=None, prof=None, graph=True, tile=0,
              surrogate=None, adapt_samples=0, adapt_epochs=0, reorder=False,
              surrogate_check=0, surrogate_switch=0.0):
    o = Opts()
    _lib().cfust_default_opts(ctypes.byref(o))
    o.precision = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
    o.nu_mode = ({"osl": NU_OSL, "exact": NU_EXACT, "fixed": NU_FIXED}[nu_mode]
                 if isinstance(nu_mode, str) else int(nu_mode))
    o.fix_delta_zero = int(bool(fix_delta_zero))
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.nu_lo = float(nu_lo)
    o.nu_hi = float(nu_hi)
    if stream is None:
        stream = torch.cuda.current_stream()
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if prof is not None:
        o.prof_ms = ctypes.cast(prof, ctypes.c_void_p)
    o.graph = int(bool(graph))
    o.tile = int(tile)
    if surrogate is not None:
        o.surrogate = surrogate.handle
    o.adapt_samples = int(adapt_samples)
    o.adapt_epochs = int(adapt_epochs)
    o.reorder = int(bool(reorder))
    o.surrogate_check = int(surrogate_check)
    o.surrogate_switch = float(surrogate_switch)
    return o


def stats_size(p, q):
    return _lib().cfust_stats_size(p, q)


def workspace_size_opts(n, p, q, g, n_qmc, **opt):
    """Workspace bytes under these options (precision, surrogate check)."""
    b = ctypes.c_size_t(0)
    o = make_opts(**opt)
    rc = _lib().cfust_workspace_size_opts(n, p, q, g, n_qmc, ctypes.byref(o), ctypes.byref(b))
    if rc:
        raise CfustError(rc, "cfust_workspace_size_opts")
    return b.value


def workspace_size(n, p, q, g, n_qmc, precision="fp64"):
    b = ctypes.c_size_t(0)
    prec = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
    rc = _lib().cfust_workspace_size(n, p, q, g, n_qmc, prec, ctypes.byref(b))
    if rc:
        raise CfustError(rc, "cfust_workspace_size")
    return b.value


def alloc_workspace(n, p, q, g, n_qmc, precision="fp64", device="cuda"):
    nbytes = workspace_size(n, p, q, g, n_qmc, precision)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _params(params):
    names = ("pi", "mu", "Sigma", "Delta", "nu")
    ts = [_dev(params[k], k) for k in names]
    g, p = ts[1].shape
    q = ts[3].shape[2]
    return ts, g, p, q


def cfust_estep(y, params, u, want=("tau", "logf", "e1", "e2", "e3", "e4"), **opt):
    """One E-step (section 3.2, Algorithm 2) on the GPU."""
    return _estep("cfust_estep", y, params, u, want, opt)


def cfust_estep_noalloc(y, params, u, want=("tau", "logf", "e1", "e2", "e3", "e4"), **opt):
    """The same E-step in the library's static device scratch (no allocation
    inside the call; the output tensors are allocated here, by the caller)."""
    return _estep("cfust_estep_noalloc", y, params, u, want, opt)


def _estep(fn, y, params, u, want, opt):
    y = _dev(y, "y")
    u = _dev(u, "u")
    (pi, mu, Sigma, Delta, nu), g, p, q = _params(params)
    n = y.shape[0]
    dev = y.device
    out = {}
    shapes = dict(tau=(n, g), logf=(n, g), e1=(n, g), e2=(n, g), e3=(n, g, q), e4=(n, g, q, q))
    for k, shp in shapes.items():
        out[k] = torch.empty(shp, dtype=torch.float64, device=dev) if k in want else None
    stats = torch.empty((g, stats_size(p, q)), dtype=torch.float64, device=dev)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    eo = EstepOut(*[_ptr(out[k]) for k in shapes], _ptr(stats), _ptr(ll), -1)
    o = make_opts(**opt)
    rc = getattr(_lib(), fn)(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                             _ptr(nu), _ptr(u), u.shape[0], ctypes.byref(o), ctypes.byref(eo))
    if rc:
        raise CfustError(rc, fn, eo.bad_component)
    res = {k: v for k, v in out.items() if v is not None}
    res["stats"] = stats
    res["loglik"] = ll
    return res


def cfust_mstep(stats, n, params_old, out=None, **opt):
    """One M-step (section 3.3, Algorithm 3) on the GPU; returns new parameters."""
    stats = _dev(stats, "stats")
    (pi0, mu0, Sg0, D0, nu0), g, p, q = _params(params_old)
    if out is None:
        out = {k: torch.empty_like(v) for k, v in
               dict(pi=pi0, mu=mu0, Sigma=Sg0, Delta=D0, nu=nu0).items()}
    bad = ctypes.c_int(-1)
    o = make_opts(**opt)
    rc = _lib().cfust_mstep(_ptr(stats), int(n), p, q, g, _ptr(mu0), _ptr(D0), _ptr(nu0),
                            ctypes.byref(o), _ptr(out["pi"]), _ptr(out["mu"]), _ptr(out["Sigma"]),
                            _ptr(out["Delta"]), _ptr(out["nu"]), ctypes.byref(bad))
    if rc:
        raise CfustError(rc, "cfust_mstep", bad.value)
    return out


def cfust_loglik(y, params, u, want_logf=False, **opt):
    """Log-likelihood eq. (3) on the GPU."""
    y = _dev(y, "y")
    u = _dev(u, "u")
    (pi, mu, Sigma, Delta, nu), g, p, q = _params(params)
    n = y.shape[0]
    ll = torch.empty(1, dtype=torch.float64, device=y.device)
    lf = torch.empty((n, g), dtype=torch.float64, device=y.device) if want_logf else None
    o = make_opts(**opt)
    rc = _lib().cfust_loglik(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                             _ptr(nu), _ptr(u), u.shape[0], ctypes.byref(o), _ptr(ll), _ptr(lf))
    if rc:
        raise CfustError(rc, "cfust_loglik")
    return (ll, lf) if want_logf else ll


def cfust_em_fit(y, params0, u, max_iter=100, tol=1e-6, **opt):
    """EM fit (Algorithms 2-4) on the GPU.  Returns the fitted parameters (new
    tensors), the log-likelihood trace and the number of M-steps."""
    y = _dev(y, "y")
    u = _dev(u, "u")
    par = {k: _dev(v, k).clone() for k, v in params0.items()}
    (pi, mu, Sigma, Delta, nu), g, p, q = _params(par)
    n = y.shape[0]
    trace = (ctypes.c_double * (max_iter + 1))()
    n_iter = ctypes.c_int(0)
    bad = ctypes.c_int(-1)
    o = make_opts(max_iter=max_iter, tol=tol, **opt)
    rc = _lib().cfust_em_fit(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                             _ptr(nu), _ptr(u), u.shape[0], ctypes.byref(o), trace,
                             ctypes.byref(n_iter), ctypes.byref(bad))
    k = n_iter.value
    par["trace"] = [trace[t] for t in range(k + 1)]
    par["n_iter"] = k
    if rc:
        # the fit up to the last completed E-step: l^(0..n_iter) and the
        # parameters the failing iteration started from
        err = CfustError(rc, "cfust_em_fit", bad.value)
        err.partial = par
        raise err
    return par


def cfust_aitken_linf(l0, l1, l2):
    return _lib().cfust_aitken_linf(float(l0), float(l1), float(l2))


def cfust_eval_special(fn, x, x2=None):
    x = _dev(x, "x")
    out = torch.empty_like(x)
    rc = _lib().cfust_eval_special(int(fn), _ptr(x), _ptr(x2), _ptr(out), x.numel(),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc:
        raise CfustError(rc, "cfust_eval_special")
    return out


def cfust_em_fit_batched(y, n_obs, g, params0, u, max_iter=50, tol=1e-6, **opt):
    """Batched EM fit of independent problems (rows of y and components of the
    parameter arrays concatenated problem by problem).  Returns the fitted
    parameters (new tensors, concatenated), traces [P][max_iter+1] (NaN past
    n_iter), n_iter [P] and status [P] (numpy arrays)."""
    import numpy as np
    y = _dev(y, "y")
    u = _dev(u, "u")
    par = {k: _dev(v, k).clone() for k, v in params0.items()}
    P = len(n_obs)
    p = y.shape[1]
    q = par["Delta"].shape[2]
    n_arr = (ctypes.c_int64 * P)(*[int(v) for v in n_obs])
    g_arr = (ctypes.c_int * P)(*[int(v) for v in g])
    trace = np.zeros((P, max_iter + 1))
    n_iter = np.zeros(P, dtype=np.int32)
    status = np.zeros(P, dtype=np.int32)
    o = make_opts(max_iter=max_iter, tol=tol, **opt)
    rc = _lib().cfust_em_fit_batched(_ptr(y), p, q, P, n_arr, g_arr, _ptr(par["pi"]), _ptr(par["mu"]),
                                     _ptr(par["Sigma"]), _ptr(par["Delta"]), _ptr(par["nu"]), _ptr(u),
                                     u.shape[0], ctypes.byref(o), trace.ctypes.data,
                                     n_iter.ctypes.data, status.ctypes.data)
    if rc:
        raise CfustError(rc, "cfust_em_fit_batched")
    return par, trace, n_iter, status


def cfust_loglik_rqmc(y, params, us, **opt):
    """l under each of K point sets us [K][N][q+1]: (values, mean, std_err)."""
    import numpy as np
    y = _dev(y, "y")
    us = _dev(us, "us")
    (pi, mu, Sigma, Delta, nu), g, p, q = _params(params)
    K, N = us.shape[0], us.shape[1]
    ll = np.zeros(K)
    mean, se = ctypes.c_double(0), ctypes.c_double(0)
    o = make_opts(**opt)
    rc = _lib().cfust_loglik_rqmc(_ptr(y), y.shape[0], p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma),
                                  _ptr(Delta), _ptr(nu), _ptr(us), N, K, ctypes.byref(o),
                                  ll.ctypes.data, ctypes.byref(mean), ctypes.byref(se))
    if rc:
        raise CfustError(rc, "cfust_loglik_rqmc")
    return ll, mean.value, se.value


def cfust_em_fit_multistart(y, starts, u, burn_in=0, max_iter=100, tol=1e-6, **opt):
    """Algorithm 1 (largest l selected) then the EM fit.  starts: list of m
    parameter dicts.  Returns the fitted parameters with trace, n_iter,
    best (selected start) and start_loglik (l of each start after burn-in)."""
    import numpy as np
    y = _dev(y, "y")
    u = _dev(u, "u")
    m = len(starts)
    cat = {k: torch.cat([_dev(s_[k], k).reshape(1, *s_[k].shape) for s_ in starts]).contiguous()
           for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    g, p = starts[0]["mu"].shape
    q = starts[0]["Delta"].shape[2]
    n = y.shape[0]
    out = {k: torch.empty_like(v[0]) for k, v in cat.items()}
    ll0 = np.zeros(m)
    best = ctypes.c_int(-1)
    trace = (ctypes.c_double * (max_iter + 1))()
    n_iter = ctypes.c_int(0)
    bad = ctypes.c_int(-1)
    o = make_opts(max_iter=max_iter, tol=tol, **opt)
    rc = _lib().cfust_em_fit_multistart(
        _ptr(y), n, p, q, g, m, _ptr(cat["pi"]), _ptr(cat["mu"]), _ptr(cat["Sigma"]),
        _ptr(cat["Delta"]), _ptr(cat["nu"]), _ptr(u), u.shape[0], int(burn_in), ctypes.byref(o),
        _ptr(out["pi"]), _ptr(out["mu"]), _ptr(out["Sigma"]), _ptr(out["Delta"]), _ptr(out["nu"]),
        ll0.ctypes.data, ctypes.byref(best), trace, ctypes.byref(n_iter), ctypes.byref(bad))
    if rc:
        raise CfustError(rc, "cfust_em_fit_multistart", bad.value)
    k = n_iter.value
    out["trace"] = [trace[t] for t in range(k + 1)]
    out["n_iter"] = k
    out["best"] = best.value
    out["start_loglik"] = ll0
    return out


def cfust_batched_config():
    w, c, s, k, ppw = (ctypes.c_int(0) for _ in range(5))
    ms = ctypes.c_double(0)
    n = _lib().cfust_batched_config(ctypes.byref(w), ctypes.byref(c), ctypes.byref(s),
                                    ctypes.byref(k), ctypes.byref(ppw), ctypes.byref(ms))
    return dict(waves_per_block=w.value, chunk=c.value, waves_per_simd=s.value,
                waves_per_pair=k.value, points_per_wave=ppw.value, tuned_ms=ms.value,
                n_candidates=n)


def cfust_batched_shape(index):
    """Candidate launch shape `index` of the batched form (tile = index + 1),
    or None outside the table."""
    w, c, s, k = (ctypes.c_int(0) for _ in range(4))
    rc = _lib().cfust_batched_shape(int(index), ctypes.byref(w), ctypes.byref(c), ctypes.byref(s),
                                    ctypes.byref(k))
    if rc != OK:
        return None
    return dict(waves_per_block=w.value, chunk=c.value, waves_per_simd=s.value,
                waves_per_pair=k.value)


def cfust_ghk_batch(h, R, dof, u, **opt):
    """GHK estimates for standardised problems V ~ t_q(0, R, dof) truncated to
    V <= h: returns [M][1+q+q(q+1)/2] (log P(V<=h), E[V|V<=h], upper triangle
    of E[VV^T|V<=h]); R: correlation matrices [M][q][q]."""
    h = _dev(h, "h")
    R = _dev(R, "R")
    dof = _dev(dof, "dof")
    u = _dev(u, "u")
    M, q = h.shape
    if R.shape != (M, q, q) or dof.shape != (M,):
        raise ValueError("R must be [M][q][q] and dof [M]")
    out = torch.empty((M, 1 + q + q * (q + 1) // 2), dtype=torch.float64, device=h.device)
    o = make_opts(**opt)
    rc = _lib().cfust_ghk_batch(q, M, _ptr(h), _ptr(R), _ptr(dof), _ptr(u), u.shape[0],
                                ctypes.byref(o), _ptr(out))
    if rc:
        raise CfustError(rc, "cfust_ghk_batch")
    return out


SURR_PARAMS = 164672
SURR_STD = 256


def feat_width(q):
    return q + q * (q - 1) // 2 + 1


def targ_width(q):
    return 1 + q + q * (q + 1) // 2


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Surrogate:
    """Handle of the surrogate network (cfust_surrogate_*)."""

    def __init__(self, handle, q):
        self.handle = handle
        self.q = q

    @classmethod
    def create(cls, q, range_, seed=0):
        import numpy as np
        r = np.ascontiguousarray(range_, dtype=np.float64)
        if r.shape != (6,):
            raise ValueError("range is h_lo, h_hi, dof_lo, dof_hi, r_max, eig_min")
        h = ctypes.c_void_p()
        rc = _lib().cfust_surrogate_create(q, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           int(seed), ctypes.byref(h))
        if rc:
            raise CfustError(rc, "cfust_surrogate_create")
        return cls(h, q)

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        rc = _lib().cfust_surrogate_load(os.fsencode(path), ctypes.byref(h))
        if rc:
            raise CfustError(rc, "cfust_surrogate_load")
        with open(path, "rb") as fh:
            q = int.from_bytes(fh.read(16)[12:16], "little", signed=True)
        return cls(h, q)

    def save(self, path):
        rc = _lib().cfust_surrogate_save(self.handle, os.fsencode(path))
        if rc:
            raise CfustError(rc, "cfust_surrogate_save")

    def close(self):
        if self.handle is not None and _LIB is not None:
            _LIB.cfust_surrogate_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, feat, targ, epochs, batch=4096, lr0=1e-3, lr1=1e-5, seed=0, wo=None, **opt):
        import numpy as np
        feat = _dev(feat, "feat")
        targ = _dev(targ, "targ")
        trace = (ctypes.c_double * max(epochs, 1))()
        w = None if wo is None else np.ascontiguousarray(wo, dtype=np.float32)
        o = make_opts(**opt)
        rc = _lib().cfust_surrogate_train(self.handle, _ptr(feat), _ptr(targ), feat.shape[0],
                                          int(epochs), int(batch), float(lr0), float(lr1),
                                          int(seed), None if w is None else _f32p(w),
                                          ctypes.byref(o), trace)
        if rc:
            raise CfustError(rc, "cfust_surrogate_train")
        return list(trace)[:epochs]

    def grad(self, feat, targ, wo=None, **opt):
        import numpy as np
        feat = _dev(feat, "feat")
        targ = _dev(targ, "targ")
        g = np.empty(SURR_PARAMS, dtype=np.float32)
        loss = ctypes.c_double(0)
        w = None if wo is None else np.ascontiguousarray(wo, dtype=np.float32)
        o = make_opts(**opt)
        rc = _lib().cfust_surrogate_grad(self.handle, _ptr(feat), _ptr(targ), feat.shape[0],
                                         None if w is None else _f32p(w), ctypes.byref(o),
                                         _f32p(g), ctypes.byref(loss))
        if rc:
            raise CfustError(rc, "cfust_surrogate_grad")
        return g, loss.value

    def eval(self, feat, **opt):
        feat = _dev(feat, "feat")
        M, F = feat.shape
        q = {feat_width(k): k for k in range(1, 9)}[F]
        out = torch.empty((M, targ_width(q)), dtype=torch.float64, device=feat.device)
        o = make_opts(**opt)
        rc = _lib().cfust_surrogate_eval(self.handle, _ptr(feat), M, ctypes.byref(o), _ptr(out))
        if rc:
            raise CfustError(rc, "cfust_surrogate_eval")
        return out

    def get_state(self):
        import numpy as np
        p = np.empty(SURR_PARAMS, dtype=np.float32)
        s = np.empty(SURR_STD, dtype=np.float32)
        rc = _lib().cfust_surrogate_get_state(self.handle, _f32p(p), _f32p(s))
        if rc:
            raise CfustError(rc, "cfust_surrogate_get_state")
        return p, s

    def set_state(self, params=None, stdv=None):
        import numpy as np
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        s = None if stdv is None else np.ascontiguousarray(stdv, dtype=np.float32)
        rc = _lib().cfust_surrogate_set_state(self.handle, None if p is None else _f32p(p),
                                              None if s is None else _f32p(s))
        if rc:
            raise CfustError(rc, "cfust_surrogate_set_state")

    def fallback_count(self):
        return int(_lib().cfust_surrogate_fallback_count(self.handle))

    def adapt(self, y, params, u, samples=16384, epochs=100, seed=1, **opt):
        """Fine-tune on GHK labels of `samples` random pairs at params; returns
        (last-epoch loss, rows trained on)."""
        y = _dev(y, "y")
        u = _dev(u, "u")
        (pi, mu, Sigma, Delta, nu), g, p, q = _params(params)
        loss = ctypes.c_double(0)
        rows = ctypes.c_int64(0)
        o = make_opts(**opt)
        rc = _lib().cfust_surrogate_adapt(self.handle, _ptr(y), y.shape[0], p, q, g, _ptr(pi),
                                          _ptr(mu), _ptr(Sigma), _ptr(Delta), _ptr(nu), _ptr(u),
                                          u.shape[0], int(samples), int(epochs), int(seed),
                                          ctypes.byref(o), ctypes.byref(loss), ctypes.byref(rows))
        if rc:
            raise CfustError(rc, "cfust_surrogate_adapt")
        return loss.value, rows.value

    def em_switch(self):
        """First GHK E-step of the last two-phase cfust_em_fit (-1: none)."""
        return int(_lib().cfust_surrogate_em_switch(self.handle))


def cfust_pair_features(y, params, **opt):
    """Raw feature rows (h | correlations | dof) of both integrals of every
    pair: [n*g*2][q + q(q-1)/2 + 1]."""
    y = _dev(y, "y")
    (pi, mu, Sigma, Delta, nu), g, p, q = _params(params)
    n = y.shape[0]
    out = torch.empty((2 * n * g, feat_width(q)), dtype=torch.float64, device=y.device)
    o = make_opts(**opt)
    rc = _lib().cfust_pair_features(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma),
                                    _ptr(Delta), _ptr(nu), ctypes.byref(o), _ptr(out))
    if rc:
        raise CfustError(rc, "cfust_pair_features")
    return out


def cfust_mlp_gemm(ta, tb, A, B, M, N, K):
    """Matrix-core product of bf16 operands (int16 tensors holding the bit
    patterns): C[M][N] fp32 = op(A) op(B)."""
    for t, nm in ((A, "A"), (B, "B")):
        if not t.is_cuda or t.dtype != torch.int16 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous int16 CUDA tensor")
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    rc = _lib().cfust_mlp_gemm(int(ta), int(tb), M, N, K, _ptr(A), _ptr(B), _ptr(C),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc:
        raise CfustError(rc, "cfust_mlp_gemm")
    return C
