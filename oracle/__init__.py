"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU product path (``paper_2005_06848_amd``) never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_cfust.so")
SOURCES = [os.path.join(_HERE, "cfust_oracle.c")]

OK, EINVAL, ENOTPD, ENONFINITE, ENOMEM = 0, 1, 2, 3, 5
NU_OSL, NU_EXACT_FD, NU_FIXED, NU_EXACT = 0, 1, 2, 3
FD_REL = 1e-3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fno-fast-math",
               "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i, i64, P = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        for name in ("orc_norm_cdf", "orc_log_norm_cdf", "orc_norm_quantile",
                     "orc_norm_quantile_log", "orc_digamma"):
            f = getattr(L, name)
            f.restype, f.argtypes = d, [d]
        for name in ("orc_gamma_p", "orc_gamma_q", "orc_chi2_quantile", "orc_chi2_quantile_ddof"):
            f = getattr(L, name)
            f.restype, f.argtypes = d, [d, d]
        L.orc_stats_size.restype, L.orc_stats_size.argtypes = i, [i, i]
        L.orc_aitken_linf.restype, L.orc_aitken_linf.argtypes = d, [d, d, d]
        L.orc_ghk.restype = i
        L.orc_ghk.argtypes = [i, P, P, d, P, i, i, P, P, P]
        L.orc_ghk_tangent.restype = i
        L.orc_ghk_tangent.argtypes = [i, P, P, d, P, i, P, P]
        L.orc_estep.restype = i
        L.orc_estep.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, i, i,
                                P, P, P, P, P, P, P, P, P]
        L.orc_mstep.restype = i
        L.orc_mstep.argtypes = [P, i64, i, i, i, P, P, P, i, i, d, d, P, P, P, P, P, P]
        L.orc_loglik.restype = i
        L.orc_loglik.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, i, P, P]
        L.orc_em_fit.restype = i
        L.orc_em_fit.argtypes = [P, i64, i, i, i, P, P, P, P, P, P, i, i, i, i, i, d, d, d,
                                 P, P, P]
        L.orc_genz_order.restype = i
        L.orc_genz_order.argtypes = [i, P, P, P, P]
        L.orc_ghk_ordered.restype = i
        L.orc_ghk_ordered.argtypes = [i, P, P, d, P, i, i, P, P, P, P]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, bad=-1):
        super().__init__(f"oracle returned {code} (bad component {bad})")
        self.code = code
        self.bad = bad


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data


def stats_size(p, q):
    return 3 + p + q + p * q + p * (p + 1) // 2 + q * (q + 1) // 2


def norm_cdf(x):
    return lib().orc_norm_cdf(float(x))


def log_norm_cdf(x):
    return lib().orc_log_norm_cdf(float(x))


def norm_quantile(p):
    return lib().orc_norm_quantile(float(p))


def norm_quantile_log(lp):
    return lib().orc_norm_quantile_log(float(lp))


def digamma(x):
    return lib().orc_digamma(float(x))


def gamma_p(a, x):
    return lib().orc_gamma_p(float(a), float(x))


def gamma_q(a, x):
    return lib().orc_gamma_q(float(a), float(x))


def aitken_linf(l0, l1, l2):
    return lib().orc_aitken_linf(float(l0), float(l1), float(l2))


def chi2_quantile(u, dof):
    return lib().orc_chi2_quantile(float(u), float(dof))


def chi2_quantile_ddof(u, dof):
    """d/d(dof) of the chi-square quantile at probability u."""
    return lib().orc_chi2_quantile_ddof(float(u), float(dof))


def ghk(h, C, dof, u, moments=True):
    """GHK estimate: returns (logT, EV, EVV) for V ~ t_q(0, C C^T, dof), V <= h."""
    h = _f64(h)
    C = _f64(C)
    u = _f64(u)
    q = h.size
    logT = np.zeros(1)
    EV = np.zeros(q)
    EVV = np.zeros((q, q))
    rc = lib().orc_ghk(q, _ptr(h), _ptr(C), float(dof), _ptr(u), u.shape[0], int(moments),
                       _ptr(logT), _ptr(EV), _ptr(EVV))
    if rc:
        raise OracleError(rc)
    return float(logT[0]), EV, EVV


def ghk_tangent(h, C, a, u):
    """log P(V <= h), V ~ t_q(0, C C^T, 2a) (GHK, no moments) and the
    derivative in a' at a' = a of the same estimate with bound h sqrt(a'/a)
    and dof 2a'."""
    h, C, u = _f64(h), _f64(C), _f64(u)
    q = h.shape[0]
    lt, dl = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_ghk_tangent(q, _ptr(h), _ptr(C), float(a), _ptr(u), u.shape[0],
                               ctypes.byref(lt), ctypes.byref(dl))
    if rc:
        raise OracleError(rc)
    return lt.value, dl.value


def genz_order(h, R):
    """Genz-Bretz variable order of P(Z <= h), Z ~ N(0, R): (perm, chol(R[perm][perm]))."""
    h = _f64(h)
    R = _f64(R)
    q = h.size
    perm = np.zeros(q, dtype=np.int32)
    Cp = np.zeros((q, q))
    rc = lib().orc_genz_order(q, _ptr(h), _ptr(R), perm.ctypes.data, _ptr(Cp))
    if rc:
        raise OracleError(rc)
    return perm, Cp


def ghk_ordered(h, R, dof, u, moments=True):
    """GHK with the Genz-Bretz order: (logT, EV, EVV, perm), moments in the
    original labelling; R is a correlation matrix."""
    h = _f64(h)
    R = _f64(R)
    u = _f64(u)
    q = h.size
    logT = np.zeros(1)
    EV = np.zeros(q)
    EVV = np.zeros((q, q))
    perm = np.zeros(q, dtype=np.int32)
    rc = lib().orc_ghk_ordered(q, _ptr(h), _ptr(R), float(dof), _ptr(u), u.shape[0],
                               int(moments), _ptr(logT), _ptr(EV), _ptr(EVV), perm.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(logT[0]), EV, EVV, perm


def _model(params):
    return (_f64(params["pi"]), _f64(params["mu"]), _f64(params["Sigma"]),
            _f64(params["Delta"]), _f64(params["nu"]))


def estep(y, params, u, nu_mode=NU_OSL, want=("tau", "logf", "e1", "e2", "e3", "e4"),
          reorder=False):
    y = _f64(y)
    u = _f64(u)
    n, p = y.shape
    pi, mu, Sigma, Delta, nu = _model(params)
    g, q = Delta.shape[0], Delta.shape[2]
    out = {}
    shapes = dict(tau=(n, g), logf=(n, g), e1=(n, g), e2=(n, g), e3=(n, g, q), e4=(n, g, q, q))
    for k in shapes:
        out[k] = np.zeros(shapes[k]) if k in want else None
    stats = np.zeros((g, stats_size(p, q)))
    ll = np.zeros(1)
    bad = ctypes.c_int(-1)
    rc = lib().orc_estep(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                         _ptr(nu), _ptr(u), u.shape[0], nu_mode, int(reorder),
                         _ptr(out["tau"]), _ptr(out["logf"]), _ptr(out["e1"]), _ptr(out["e2"]),
                         _ptr(out["e3"]), _ptr(out["e4"]), _ptr(stats), _ptr(ll),
                         ctypes.addressof(bad))
    if rc:
        raise OracleError(rc, bad.value)
    out = {k: v for k, v in out.items() if v is not None}
    out["stats"] = stats
    out["loglik"] = float(ll[0])
    return out


def mstep(stats, n, params_old, nu_mode=NU_OSL, fix_delta_zero=False, nu_lo=1.0, nu_hi=200.0):
    stats = _f64(stats)
    pi0, mu0, Sg0, D0, nu0 = _model(params_old)
    g, p = mu0.shape
    q = D0.shape[2]
    pi = np.zeros(g)
    mu = np.zeros((g, p))
    Sigma = np.zeros((g, p, p))
    Delta = np.zeros((g, p, q))
    nu = np.zeros(g)
    bad = ctypes.c_int(-1)
    rc = lib().orc_mstep(_ptr(stats), int(n), p, q, g, _ptr(mu0), _ptr(D0), _ptr(nu0), nu_mode,
                         int(fix_delta_zero), nu_lo, nu_hi, _ptr(pi), _ptr(mu), _ptr(Sigma),
                         _ptr(Delta), _ptr(nu), ctypes.addressof(bad))
    if rc:
        raise OracleError(rc, bad.value)
    return dict(pi=pi, mu=mu, Sigma=Sigma, Delta=Delta, nu=nu)


def loglik(y, params, u, want_logf=False, reorder=False):
    y = _f64(y)
    u = _f64(u)
    n, p = y.shape
    pi, mu, Sigma, Delta, nu = _model(params)
    g, q = Delta.shape[0], Delta.shape[2]
    ll = np.zeros(1)
    lf = np.zeros((n, g)) if want_logf else None
    rc = lib().orc_loglik(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                          _ptr(nu), _ptr(u), u.shape[0], int(reorder), _ptr(ll), _ptr(lf))
    if rc:
        raise OracleError(rc)
    return (float(ll[0]), lf) if want_logf else float(ll[0])


def em_fit(y, params0, u, max_iter=10, tol=1e-6, nu_mode=NU_OSL, fix_delta_zero=False,
           nu_lo=1.0, nu_hi=200.0, reorder=False):
    y = _f64(y)
    u = _f64(u)
    n, p = y.shape
    pi, mu, Sigma, Delta, nu = [a.copy() for a in _model(params0)]
    g, q = Delta.shape[0], Delta.shape[2]
    trace = np.zeros(max_iter + 1)
    n_iter = ctypes.c_int(0)
    bad = ctypes.c_int(-1)
    rc = lib().orc_em_fit(_ptr(y), n, p, q, g, _ptr(pi), _ptr(mu), _ptr(Sigma), _ptr(Delta),
                          _ptr(nu), _ptr(u), u.shape[0], nu_mode, int(reorder),
                          int(fix_delta_zero), max_iter,
                          tol, nu_lo, nu_hi, _ptr(trace), ctypes.addressof(n_iter),
                          ctypes.addressof(bad))
    if rc:
        raise OracleError(rc, bad.value)
    k = n_iter.value
    return dict(pi=pi, mu=mu, Sigma=Sigma, Delta=Delta, nu=nu, trace=trace[:k + 1], n_iter=k)


def em_fit_multistart(y, starts, u, burn_in=0, max_iter=10, tol=1e-6, nu_mode=NU_OSL,
                      reorder=False, **kw):
    """Algorithm 1 (section 3.1) composed from the oracle's own EM: every
    start runs burn_in EM iterations (its l^(0) when burn_in = 0), the start
    with the largest l after them is kept (the paper's "smallest" read as the
    largest, i.e. maximum likelihood), and the fit continues from it.  The
    burn-in uses nu_mode in the natural variable order; the continuation uses
    nu_mode and reorder."""
    runs = [em_fit(y, s, u, max_iter=burn_in, tol=0.0, nu_mode=nu_mode, **kw) for s in starts]
    ll = np.array([r["trace"][-1] for r in runs])
    best = int(np.argmax(ll))
    fit = em_fit(y, runs[best], u, max_iter=max_iter, tol=tol, nu_mode=nu_mode, reorder=reorder,
                 **kw)
    fit["best"] = best
    fit["start_loglik"] = ll
    return fit
