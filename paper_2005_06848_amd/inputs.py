"""Seeded synthetic inputs for the CFUST mixture E-step.

This module is shared by the GPU path's tests and benchmark and by the
oracle's tests.  It holds none of the E-step / M-step arithmetic: only
seeded random draws (numpy PCG64), the quasi-Monte Carlo point set and the
starting parameters that both implementations receive as *inputs*.

* ``qmc_points`` -- unscrambled 30-bit Sobol integers in dimension q+1, XOR'ed
  with a seeded random digital shift, mapped to the open unit interval by
  u = (x + 1/2) / 2^30, so that no coordinate is ever 0 or 1.  Column 0 drives
  the chi-square scale of the multivariate-t integrals, columns 1..q drive the
  sequential truncated-normal draws.
* ``sample_cfust`` -- draws from a finite mixture of canonical fundamental
  skew-t distributions through the hidden-variable form of the model
  (section 2: latent gamma and truncated-normal variables):
  y = mu + (Delta |U0| + U1) / sqrt(w), w ~ Gamma(nu/2, rate nu/2),
  U0 ~ N(0, I_q), U1 ~ N(0, Sigma).
* ``init_from_partition`` -- a starting value Psi^(0) computed from a hard
  partition (section 3.1: initial partitions from k-means or random).
* ``config(k)`` -- the five synthetic workloads (sizes below) that stand in for
  the paper's AIS data, which is not available.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.stats import qmc as _qmc
from scipy.special import gammaln as _gammaln

SEED_BASE = 200506848
QMC_SHIFT_SEED = 0x2005


# ----------------------------------------------------------------------------
# quasi-Monte Carlo points
# ----------------------------------------------------------------------------
def qmc_points(n_qmc: int, q: int, seed: int = QMC_SHIFT_SEED) -> np.ndarray:
    """Return u[n_qmc][q+1] (float64, C order) in (0, 1)."""
    if n_qmc < 1 or q < 1:
        raise ValueError("n_qmc and q must be >= 1")
    eng = _qmc.Sobol(d=q + 1, scramble=False, bits=30)
    m = int(math.ceil(math.log2(n_qmc)))
    raw = eng.random_base2(m)[:n_qmc]
    x = np.rint(raw * 2.0 ** 30).astype(np.int64)
    rng = np.random.default_rng(seed)
    shift = rng.integers(0, 2 ** 30, size=q + 1, dtype=np.int64)
    u = ((x ^ shift[None, :]).astype(np.float64) + 0.5) / 2.0 ** 30
    return np.ascontiguousarray(u)


# ----------------------------------------------------------------------------
# model draws
# ----------------------------------------------------------------------------
def wishart_sigma(rng: np.random.Generator, p: int) -> np.ndarray:
    """Sigma = sum_{k=1}^{p+2} x_k x_k^T / (p+2), x_k ~ N(0, I_p)."""
    x = rng.standard_normal((p + 2, p))
    return x.T @ x / (p + 2)


def korobov_generator(n: int, d: int) -> np.ndarray:
    """Generating vector z = (1, a, a^2, ...) mod n of a rank-1 Korobov lattice
    rule, a chosen among the odd a < n/2 by the P_2 criterion of the rule
    (the worst-case error in the Korobov space of smoothness 2):
        P_2 = -1 + (1/n) sum_k prod_j (1 + 2 pi^2 B_2({k z_j / n})),
    B_2(x) = x^2 - x + 1/6."""
    k = np.arange(n)
    best, best_a = np.inf, 1
    for a in range(1, n // 2, 2):
        z = np.array([pow(a, j, n) for j in range(d)])
        x = (np.outer(k, z) % n) / n
        b2 = x * x - x + 1.0 / 6.0
        p2 = -1.0 + np.mean(np.prod(1.0 + 2.0 * np.pi ** 2 * b2, axis=1))
        if p2 < best:
            best, best_a = p2, a
    return np.array([pow(best_a, j, n) for j in range(d)])


def lattice_points(n_qmc: int, q: int, seed: int = QMC_SHIFT_SEED, z=None,
                   tent: bool = True) -> np.ndarray:
    """u[n_qmc][q+1] from a randomly shifted rank-1 lattice rule, with the
    tent (baker's) transform x -> 1 - |2x - 1| unless tent is False, kept
    inside (0, 1)."""
    d = q + 1
    if z is None:
        z = korobov_generator(n_qmc, d)
    rng = np.random.default_rng(seed)
    shift = rng.random(d)
    x = (np.outer(np.arange(n_qmc), z) % n_qmc) / n_qmc + shift[None, :]
    x -= np.floor(x)
    if tent:
        x = 1.0 - np.abs(2.0 * x - 1.0)
    eps = 2.0 ** -53
    return np.ascontiguousarray(np.clip(x, eps, 1.0 - eps))


def sample_cfust(rng: np.random.Generator, n: int, pi, mu, Sigma, Delta, nu):
    """Draw n observations and their labels from the CFUST mixture."""
    pi = np.asarray(pi, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    Sigma = np.asarray(Sigma, dtype=np.float64)
    Delta = np.asarray(Delta, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    g, p = mu.shape
    q = Delta.shape[2]
    z = rng.choice(g, size=n, p=pi / pi.sum())
    y = np.empty((n, p))
    for i in range(g):
        idx = np.nonzero(z == i)[0]
        m = idx.size
        if m == 0:
            continue
        w = rng.gamma(shape=nu[i] / 2.0, scale=2.0 / nu[i], size=m)
        u0 = np.abs(rng.standard_normal((m, q)))
        L = np.linalg.cholesky(Sigma[i])
        u1 = rng.standard_normal((m, p)) @ L.T
        y[idx] = mu[i] + (u0 @ Delta[i].T + u1) / np.sqrt(w)[:, None]
    return np.ascontiguousarray(y), z


def kappa_nu(nu: float) -> float:
    """E[|U0| / sqrt(W)] per coordinate: sqrt(nu/pi) Gamma((nu-1)/2) / Gamma(nu/2)."""
    return math.sqrt(nu / math.pi) * math.exp(_gammaln((nu - 1) / 2.0) - _gammaln(nu / 2.0))


def lkj_corr_batch(rng: np.random.Generator, m: int, d: int, eta: float) -> np.ndarray:
    """m random correlation matrices from LKJ(eta) by the onion method
    (Lewandowski, Kurowicka & Joe 2009): grow each matrix one row at a time,
    the new row's squared length drawn from a Beta and its direction uniform,
    mapped through the current Cholesky factor.  Returns [m][d][d]."""
    R = np.zeros((m, d, d))
    idx = np.arange(d)
    R[:, idx, idx] = 1.0
    if d == 1:
        return R
    beta = eta + (d - 2) / 2.0
    r = 2.0 * rng.beta(beta, beta, size=m) - 1.0
    R[:, 0, 1] = r
    R[:, 1, 0] = r
    for k in range(2, d):
        beta -= 0.5
        yk = rng.beta(k / 2.0, beta, size=m)
        z = rng.standard_normal((m, k))
        w = np.sqrt(yk)[:, None] * z / np.linalg.norm(z, axis=1, keepdims=True)
        L = np.linalg.cholesky(R[:, :k, :k])
        qv = np.einsum("mab,mb->ma", L, w)
        R[:, :k, k] = qv
        R[:, k, :k] = qv
    return R


def lkj_corr(rng: np.random.Generator, d: int, eta: float) -> np.ndarray:
    """One random correlation matrix from LKJ(eta) (see lkj_corr_batch)."""
    return lkj_corr_batch(rng, 1, d, eta)[0]


def surrogate_samples(rng: np.random.Generator, m: int, q: int, h_lo: float = -4.0,
                      h_hi: float = 6.0, dof_lo: float = 5.0, dof_hi: float = 20.0,
                      dof_step: float = 0.25, eta: float = 2.0, h_extra=None):
    """Inputs of the surrogate's training set: correlation matrices R ~ LKJ(eta),
    degrees of freedom uniform on a grid of step dof_step in [dof_lo, dof_hi],
    truncation points h uniform on [h_lo, h_hi]^q (or, for the first rows,
    the points given in h_extra).  Returns h [m][q], R [m][q][q], dof [m]."""
    R = lkj_corr_batch(rng, m, q, eta)
    grid = np.arange(dof_lo, dof_hi + 1e-9, dof_step)
    dof = rng.choice(grid, size=m)
    h = rng.uniform(h_lo, h_hi, size=(m, q))
    if h_extra is not None:
        k = min(len(h_extra), m)
        h[:k] = h_extra[:k]
    return np.ascontiguousarray(h), np.ascontiguousarray(R), np.ascontiguousarray(dof)


# ----------------------------------------------------------------------------
# starting values
# ----------------------------------------------------------------------------
def _kmeans_once(rng, y, g, n_lloyd):
    n = y.shape[0]
    centres = [y[rng.integers(n)]]
    d2 = np.sum((y - centres[0]) ** 2, axis=1)
    for _ in range(1, g):
        prob = d2 / d2.sum()
        c = y[rng.choice(n, p=prob)]
        centres.append(c)
        d2 = np.minimum(d2, np.sum((y - c) ** 2, axis=1))
    C = np.array(centres)
    lab = np.zeros(n, dtype=np.int64)
    for _ in range(n_lloyd):
        dist = ((y[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        lab = np.argmin(dist, axis=1)
        for i in range(g):
            sel = y[lab == i]
            if sel.shape[0] > 0:
                C[i] = sel.mean(0)
    inertia = float(((y - C[lab]) ** 2).sum())
    return lab, inertia


def kmeans_pp(rng: np.random.Generator, y: np.ndarray, g: int, n_lloyd: int = 25,
              n_init: int = 8) -> np.ndarray:
    """Seeded k-means++ seeding plus a fixed number of Lloyd steps, restarted
    ``n_init`` times; the partition with the lowest within-cluster sum of
    squares among those whose smallest cluster holds at least
    max(p + 2, 2% of n) points is kept (heavy tails otherwise let single
    outliers take a centre)."""
    n, p = y.shape
    min_size = max(p + 2, int(0.02 * n))
    best, best_ok = None, None
    for _ in range(n_init):
        lab, inertia = _kmeans_once(rng, y, g, n_lloyd)
        ok = np.bincount(lab, minlength=g).min() >= min_size
        if best is None or inertia < best[1]:
            best = (lab, inertia)
        if ok and (best_ok is None or inertia < best_ok[1]):
            best_ok = (lab, inertia)
    return (best_ok or best)[0]


def init_from_partition(y: np.ndarray, lab: np.ndarray, g: int, q: int, nu0: float = 10.0):
    """Psi^(0) from a hard partition.

    Per cluster with sample covariance S and per-coordinate sample skewness:
    delta_k = sign(skew_k) sqrt(c S_kk), Delta^(0) = the first q columns of
    diag(delta) (zero-padded when q > p), Sigma^(0) = S - Delta Delta^T with c
    halved from 1/2 until Sigma^(0) is positive definite,
    mu^(0) = ybar - kappa_nu Delta 1_q, nu^(0) = nu0, pi = cluster fractions.
    """
    n, p = y.shape
    pi = np.zeros(g)
    mu = np.zeros((g, p))
    Sigma = np.zeros((g, p, p))
    Delta = np.zeros((g, p, q))
    nu = np.full(g, float(nu0))
    kap = kappa_nu(nu0)
    for i in range(g):
        sel = y[lab == i]
        if sel.shape[0] < p + 2:
            sel = y
        pi[i] = max(np.mean(lab == i), 1.0 / n)
        ybar = sel.mean(0)
        S = np.cov(sel, rowvar=False).reshape(p, p)
        sd = np.sqrt(np.diag(S))
        skew = ((sel - ybar) ** 3).mean(0) / sd ** 3
        sgn = np.where(skew >= 0, 1.0, -1.0)
        c = 0.5
        for _ in range(60):
            dvec = sgn * np.sqrt(c * np.diag(S))
            D = np.zeros((p, q))
            for k in range(min(p, q)):
                D[k, k] = dvec[k]
            Sg = S - D @ D.T
            try:
                np.linalg.cholesky(Sg)
                break
            except np.linalg.LinAlgError:
                c *= 0.5
        Delta[i] = D
        Sigma[i] = 0.5 * (Sg + Sg.T)
        mu[i] = ybar - kap * D.sum(1)
    pi /= pi.sum()
    return dict(pi=pi, mu=mu, Sigma=Sigma, Delta=Delta, nu=nu)


def multistart_inits(y: np.ndarray, g: int, q: int, m: int, seed: int = 7):
    """m starting values Psi^(0) from m initial partitions (k-means++ with one
    restart each, seeds seed, seed+1, ...), as the parallel initialisation of
    section 3.1 takes them."""
    out = []
    for k in range(m):
        rng = np.random.default_rng(seed + k)
        out.append(init_from_partition(y, kmeans_pp(rng, y, g, n_init=1), g, q))
    return out


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
CONFIG_DOC = {
    1: "plain FP64 EM: n=500 p=2 q=2 g=2 nu=(4,8) N=1024, 10 iterations",
    2: "FP64 E-step + M-step: n=20000 p=4 q=4 g=3 nu~U(3,15) N=4096",
    3: "FP32 precision form: n=200000 p=6 q=6 g=4 nu~U(3,10) N=8192",
    4: "batched: 64 starts, n~U{5000..50000} g~U{2..6} p=q=5 N=4096",
    5: "surrogate use: n=1000000 p=6 q=6 g=4 nu~U(3,10)",
    6: "high-q stress: n=202 p=q=11 g=2 nu~U(4,12) N=8192, whole fit",
}


def _true_params_basic(rng, p, q, g, nu, delta_half, pi):
    mu = 3.0 * rng.standard_normal((g, p))
    Sigma = np.stack([wishart_sigma(rng, p) for _ in range(g)])
    Delta = rng.uniform(-delta_half, delta_half, size=(g, p, q))
    return dict(pi=np.asarray(pi, float), mu=mu, Sigma=Sigma, Delta=Delta,
                nu=np.asarray(nu, float))


def _true_params_separated(rng, p, q, g, nu, delta_half):
    Sigma = np.stack([wishart_sigma(rng, p) for _ in range(g)])
    Delta = rng.uniform(-delta_half, delta_half, size=(g, p, q))
    sig = max(math.sqrt(np.linalg.eigvalsh(Sigma[i] + Delta[i] @ Delta[i].T)[-1]) for i in range(g))
    v = rng.standard_normal(p)
    v /= np.linalg.norm(v)
    mu = np.stack([6.0 * sig * i * v for i in range(g)])
    return dict(pi=np.full(g, 1.0 / g), mu=mu, Sigma=Sigma, Delta=Delta,
                nu=np.asarray(nu, float))


def config(k: int, n: int | None = None, seed: int | None = None, kmeans_restarts: int = 8):
    """Return a dict with y, the true parameters, Psi^(0), u and sizes for workload k.

    ``n`` overrides the number of observations (the draws for the first
    observations do not depend on it for workloads 1-3 and 5 only through the
    label draw, so tests use it for reduced copies of the same recipe).
    ``seed`` replaces the workload's own seed: another draw of the same recipe.
    ``kmeans_restarts`` sets the restarts of the k-means++ start (Psi^(0)).
    """
    rng = np.random.default_rng(SEED_BASE + k if seed is None else seed)
    if k == 1:
        p, q, g, N = 2, 2, 2, 1024
        true = _true_params_basic(rng, p, q, g, [4.0, 8.0], 2.0, [0.4, 0.6])
        n = 500 if n is None else n
        iters = 10
    elif k == 2:
        p, q, g, N = 4, 4, 3, 4096
        true = _true_params_separated(rng, p, q, g, rng.uniform(3, 15, size=g), 3.0)
        n = 20000 if n is None else n
        iters = 50
    elif k == 3:
        p, q, g, N = 6, 6, 4, 8192
        true = _true_params_basic(rng, p, q, g, rng.uniform(3, 10, size=g), 2.0, np.full(g, 0.25))
        n = 200000 if n is None else n
        iters = 1
    elif k == 5:
        p, q, g, N = 6, 6, 4, 8192
        true = _true_params_basic(rng, p, q, g, rng.uniform(3, 10, size=g), 2.0, np.full(g, 0.25))
        n = 1000000 if n is None else n
        iters = 1
    elif k == 6:
        # the shape of the paper's data set (202 observations of 11 variables,
        # two groups of 102 and 100) with q = p: a stress case for large q
        p, q, g, N = 11, 11, 2, 8192
        true = _true_params_basic(rng, p, q, g, rng.uniform(4, 12, size=g), 1.0,
                                  [102 / 202, 100 / 202])
        n = 202 if n is None else n
        iters = 1000
    else:
        raise ValueError("workload 4 is built by batched_problems()")
    y, z = sample_cfust(rng, n, **true)
    lab = kmeans_pp(rng, y, g, n_init=kmeans_restarts)
    init = init_from_partition(y, lab, g, q)
    u = qmc_points(N, q)
    return dict(k=k, n=n, p=p, q=q, g=g, n_qmc=N, iters=iters, y=y, labels=z,
                true=true, init=init, u=u)


def batched_problems(n_problems: int = 64, n_lo: int = 5000, n_hi: int = 50000,
                     seed_offset: int = 4):
    """Workload 4: independent EM starts with uneven n and g (p = q = 5)."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    p = q = 5
    probs = []
    for _ in range(n_problems):
        g = int(rng.integers(2, 7))
        n = int(rng.integers(n_lo, n_hi + 1))
        true = _true_params_basic(rng, p, q, g, rng.uniform(3, 15, size=g), 2.0,
                                  rng.dirichlet(np.full(g, 5.0)))
        y, z = sample_cfust(rng, n, **true)
        lab = kmeans_pp(rng, y, g, n_lloyd=10, n_init=2)
        init = init_from_partition(y, lab, g, q)
        probs.append(dict(n=n, p=p, q=q, g=g, y=y, labels=z, true=true, init=init))
    return probs


def random_case(seed: int, n: int, p: int, q: int, g: int, n_qmc: int,
                nu_lo: float = 3.0, nu_hi: float = 15.0):
    """Small random problem for shape sweeps: parameters, data and points."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    true = _true_params_basic(rng, p, q, g, rng.uniform(nu_lo, nu_hi, size=g), 2.0,
                              rng.dirichlet(np.full(g, 4.0)))
    y, z = sample_cfust(rng, max(n, 1), **true)
    y = y[:n]
    # the evaluation point is the true parameter set perturbed (not a fit)
    par = {k: np.array(v, copy=True) for k, v in true.items()}
    par["mu"] = par["mu"] + 0.3 * rng.standard_normal(par["mu"].shape)
    par["nu"] = par["nu"] * rng.uniform(0.8, 1.25, size=g)
    return dict(n=n, p=p, q=q, g=g, n_qmc=n_qmc, y=np.ascontiguousarray(y),
                params=par, u=qmc_points(n_qmc, q))
