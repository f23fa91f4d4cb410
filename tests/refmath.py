"""Independent reference mathematics for pinning the oracle (tests only).

Nothing here calls the oracle or the GPU library.  Each function is a
textbook or closed-form result, evaluated with scipy/numpy primitives:
  * the univariate Student-t CDF and its truncated first/second moments;
  * the bivariate normal CDF through Owen's T function (Owen 1956), integrated
    over the chi scale to give the bivariate Student-t CDF;
  * the skew-t density of the p = q = 1 case of the CFUST family;
  * the EM algorithm for a multivariate-t mixture (the Delta = 0 case);
  * brute-force Monte Carlo of truncated multivariate-t moments and of the
    CFUST hidden-variable posterior expectations.
"""
import numpy as np
from scipy import integrate, optimize, special as sp, stats


def t_trunc_moments_upper(h, nu):
    """E[V | V <= h], E[V^2 | V <= h] for V ~ t_nu (via T = -V > -h)."""
    a = -h
    pdf = stats.t.pdf(a, nu)
    sf = sp.stdtr(nu, -a)
    m1 = pdf * (nu + a * a) / ((nu - 1) * sf)
    m2 = (a * pdf * (nu + a * a) + nu * sf) / ((nu - 2) * sf)
    return -m1, m2


def phi2(x, y, rho):
    """Bivariate standard normal CDF, x, y != 0 (Owen 1956)."""
    r = np.sqrt(1.0 - rho * rho)
    ax = (y - rho * x) / (x * r)
    ay = (x - rho * y) / (y * r)
    beta = 0.0 if x * y > 0 else 0.5
    return 0.5 * sp.ndtr(x) + 0.5 * sp.ndtr(y) - sp.owens_t(x, ax) - sp.owens_t(y, ay) - beta


def t2_cdf(h1, h2, rho, nu):
    """Bivariate Student-t CDF P(V1 <= h1, V2 <= h2), correlation rho, dof nu:
    V = Z / S with S = sqrt(chi2_nu / nu); integrate Phi2(s h1, s h2) over S."""
    def dens_s(s):
        return stats.chi2.pdf(nu * s * s, nu) * 2.0 * nu * s

    def f(s):
        return phi2(s * h1, s * h2, rho) * dens_s(s)

    val, err = integrate.quad(f, 0.0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)
    return val


def skew_t_pq1_logpdf(y, mu, sigma2, delta, nu):
    """CFUST density for p = q = 1 written with univariate t functions:
    2 t_1(y; mu, omega2, nu) T_1(delta (y-mu)/omega2 sqrt((nu+1)/(nu+d)) / sqrt(lam); nu+1),
    omega2 = sigma2 + delta^2, lam = 1 - delta^2/omega2, d = (y-mu)^2/omega2."""
    om2 = sigma2 + delta * delta
    lam = 1.0 - delta * delta / om2
    d = (y - mu) ** 2 / om2
    z = (y - mu) / np.sqrt(om2)
    arg = delta * (y - mu) / om2 * np.sqrt((nu + 1) / (nu + d)) / np.sqrt(lam)
    return np.log(2.0) + stats.t.logpdf(z, nu) - 0.5 * np.log(om2) + np.log(sp.stdtr(nu + 1, arg))


def t_mixture_em(y, pi, mu, Sigma, nu, iters):
    """Textbook EM for a mixture of multivariate t distributions
    (McLachlan & Peel 2000, section 7.5), with the exact nu equation."""
    y = np.asarray(y, float)
    n, p = y.shape
    pi = np.array(pi, float)
    mu = np.array(mu, float)
    Sigma = np.array(Sigma, float)
    nu = np.array(nu, float)
    g = pi.size
    trace = []
    for it in range(iters + 1):
        logf = np.zeros((n, g))
        dist = np.zeros((n, g))
        for i in range(g):
            logf[:, i] = np.log(pi[i]) + stats.multivariate_t(mu[i], Sigma[i], df=nu[i]).logpdf(y)
            r = y - mu[i]
            dist[:, i] = np.einsum("nj,jk,nk->n", r, np.linalg.inv(Sigma[i]), r)
        lse = sp.logsumexp(logf, axis=1)
        trace.append(lse.sum())
        if it == iters:
            break
        tau = np.exp(logf - lse[:, None])
        for i in range(g):
            u = (nu[i] + p) / (nu[i] + dist[:, i])
            t = tau[:, i]
            ni = t.sum()
            pi[i] = ni / n
            mu[i] = (t * u) @ y / (t * u).sum()
            r = y - mu[i]
            Sigma[i] = (r * (t * u)[:, None]).T @ r / ni
            c = (t * (np.log(u) - u)).sum() / ni + sp.digamma((nu[i] + p) / 2) - np.log((nu[i] + p) / 2)
            fn = lambda v: -sp.digamma(v / 2) + np.log(v / 2) + 1 + c
            if fn(200.0) >= 0:
                nu[i] = 200.0
            elif fn(1.0) <= 0:
                nu[i] = 1.0
            else:
                nu[i] = optimize.brentq(fn, 1.0, 200.0, xtol=1e-14, rtol=1e-15, maxiter=500)
        pi /= pi.sum()
    return dict(pi=pi, mu=mu, Sigma=Sigma, nu=nu, trace=np.array(trace))


def mc_truncated_t(h, R, dof, n_draws, seed, chunk=1_000_000):
    """Brute-force Monte Carlo of P(V <= h), E[V | V <= h], E[V V^T | V <= h]
    for V ~ t_q(0, R, dof).  Returns estimates and their standard errors."""
    rng = np.random.default_rng(seed)
    q = len(h)
    L = np.linalg.cholesky(np.asarray(R, float))
    h = np.asarray(h, float)
    cnt = 0
    s1 = np.zeros(q)
    s2 = np.zeros((q, q))
    s1sq = np.zeros(q)
    s2sq = np.zeros((q, q))
    done = 0
    while done < n_draws:
        m = min(chunk, n_draws - done)
        z = rng.standard_normal((m, q)) @ L.T
        s = np.sqrt(rng.chisquare(dof, size=m) / dof)
        v = z / s[:, None]
        keep = np.all(v <= h, axis=1)
        vk = v[keep]
        cnt += vk.shape[0]
        s1 += vk.sum(0)
        s1sq += (vk ** 2).sum(0)
        outer = vk[:, :, None] * vk[:, None, :]
        s2 += outer.sum(0)
        s2sq += (outer ** 2).sum(0)
        done += m
    P = cnt / n_draws
    m1 = s1 / cnt
    m2 = s2 / cnt
    se1 = np.sqrt(np.maximum(s1sq / cnt - m1 ** 2, 0) / cnt)
    se2 = np.sqrt(np.maximum(s2sq / cnt - m2 ** 2, 0) / cnt)
    seP = np.sqrt(P * (1 - P) / n_draws)
    return P, m1, m2, seP, se1, se2


def mc_cfust_posterior(y, mu, Sigma, Delta, nu, n_draws, seed, chunk=500_000):
    """Importance sampling over the hidden-variable prior of one CFUST
    component (W ~ Gamma(nu/2, rate nu/2), U = |U0|/sqrt(W)), weighted by
    N_p(y; mu + Delta U, Sigma / W):
      f(y) = E[weight],  E[g(W,U) | y] = E[g weight] / E[weight].
    Returns f, E[W], E[W U], E[W U U^T] and standard errors (batch means)."""
    rng = np.random.default_rng(seed)
    p = len(y)
    q = Delta.shape[1]
    Sinv = np.linalg.inv(Sigma)
    logdetS = np.linalg.slogdet(Sigma)[1]
    batches = []
    done = 0
    while done < n_draws:
        m = min(chunk, n_draws - done)
        w = rng.gamma(nu / 2.0, 2.0 / nu, size=m)
        u = np.abs(rng.standard_normal((m, q))) / np.sqrt(w)[:, None]
        r = y[None, :] - mu[None, :] - u @ Delta.T
        quad = np.einsum("nj,jk,nk->n", r, Sinv, r)
        logwt = -0.5 * p * np.log(2 * np.pi) - 0.5 * logdetS + 0.5 * p * np.log(w) - 0.5 * w * quad
        wt = np.exp(logwt)
        batches.append(np.concatenate([
            [wt.mean()],
            [(wt * w).mean()],
            (wt[:, None] * w[:, None] * u).mean(0),
            (wt[:, None, None] * w[:, None, None] * u[:, :, None] * u[:, None, :]).reshape(m, -1).mean(0),
        ]))
        done += m
    B = np.array(batches)
    nb = B.shape[0]

    def ratio(k):
        return B[:, k] / B[:, 0]

    f = B[:, 0].mean()
    fse = B[:, 0].std(ddof=1) / np.sqrt(nb)
    vals = B.mean(0)
    out = vals[1:] / vals[0]
    # delta-method SE from batch means of the ratio
    rb = B[:, 1:] / B[:, :1]
    se = rb.std(0, ddof=1) / np.sqrt(nb)
    e2 = out[0]
    e3 = out[1:1 + q]
    e4 = out[1 + q:].reshape(q, q)
    return dict(f=f, f_se=fse, e2=e2, e2_se=se[0], e3=e3, e3_se=se[1:1 + q],
                e4=e4, e4_se=se[1 + q:].reshape(q, q))
