"""Pins of the oracle's exact e1 = E[log W | y] (nu_mode EXACT: the derivative
of the GHK estimate itself; nu_mode EXACT_FD: a central difference).

The hidden-variable model gives W | y a density proportional to
w^{a-1} e^{-b w} Phi_q(sqrt(w) c; Lambda) (a = (nu+p)/2, b = (nu+d)/2,
c = Delta^T Omega^{-1} (y - mu), Lambda = I - Delta^T Omega^{-1} Delta).  The
pins compute E[log W | y] straight from that density by one-dimensional
quadrature over w, with the normal CDF from scipy (q = 1) or the bivariate
normal CDF as a one-dimensional integral on generalised Gauss-Laguerre nodes
(q = 2), and check
the oracle's values against it.  Delta = 0 reduces all modes to
psi(a) - log b exactly.  The derivative of the estimate is pinned on its own
by a fourth-order difference quotient of the oracle's plain GHK estimate
(which it differentiates), and its chi-square quantile derivative by mpmath.
"""
import mpmath
import numpy as np
from scipy import integrate, special, stats

import oracle as orc
from paper_2005_06848_amd import inputs


def _pair_quantities(y, mu, Sigma, Delta, nu):
    p = len(y)
    Om = Sigma + Delta @ Delta.T
    r = y - mu
    d = float(r @ np.linalg.solve(Om, r))
    c = Delta.T @ np.linalg.solve(Om, r)
    Lam = np.eye(Delta.shape[1]) - Delta.T @ np.linalg.solve(Om, Delta)
    return 0.5 * (nu + p), 0.5 * (nu + d), c, Lam


def _oracle_e1(y, mu, Sigma, Delta, nu, u, mode):
    par = dict(pi=np.array([1.0]), mu=mu[None], Sigma=Sigma[None], Delta=Delta[None],
               nu=np.array([nu]))
    out = orc.estep(y[None], par, u, nu_mode=mode, want=("e1",))
    return float(out["e1"][0, 0])


def test_delta_zero_modes_agree():
    rng = np.random.default_rng(1)
    p, q = 3, 2
    y, mu = rng.standard_normal(p), rng.standard_normal(p)
    Sigma = inputs.wishart_sigma(rng, p)
    Delta = np.zeros((p, q))
    u = inputs.qmc_points(512, q)
    e_osl = _oracle_e1(y, mu, Sigma, Delta, 6.0, u, orc.NU_OSL)
    e_fd = _oracle_e1(y, mu, Sigma, Delta, 6.0, u, orc.NU_EXACT_FD)
    e_ex = _oracle_e1(y, mu, Sigma, Delta, 6.0, u, orc.NU_EXACT)
    a, b, _, _ = _pair_quantities(y, mu, Sigma, Delta, 6.0)
    assert e_fd == e_osl
    assert e_ex == e_osl
    assert abs(e_fd - (special.digamma(a) - np.log(b))) < 1e-14


def test_q1_matches_quadrature_of_the_definition():
    rng = np.random.default_rng(2)
    p, q = 2, 1
    u = inputs.qmc_points(1 << 15, q)
    for case in range(4):
        y, mu = rng.standard_normal(p) * 2, rng.standard_normal(p)
        Sigma = inputs.wishart_sigma(rng, p)
        Delta = rng.uniform(-2, 2, size=(p, q))
        nu = rng.uniform(3, 12)
        a, b, c, Lam = _pair_quantities(y, mu, Sigma, Delta, nu)
        sl = np.sqrt(Lam[0, 0])

        def dens(w, k):
            return (np.log(w) ** k) * np.exp((a - 1) * np.log(w) - b * w
                                             + special.log_ndtr(np.sqrt(w) * c[0] / sl))

        num = integrate.quad(lambda w: dens(w, 1), 0, np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
        den = integrate.quad(lambda w: dens(w, 0), 0, np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
        ref = num / den
        e_fd = _oracle_e1(y, mu, Sigma, Delta, nu, u, orc.NU_EXACT_FD)
        e_ex = _oracle_e1(y, mu, Sigma, Delta, nu, u, orc.NU_EXACT)
        e_osl = _oracle_e1(y, mu, Sigma, Delta, nu, u, orc.NU_OSL)
        assert abs(e_fd - ref) < 2e-5 * max(1.0, abs(ref)), (case, e_fd, ref, e_osl)
        assert abs(e_ex - ref) < 2e-5 * max(1.0, abs(ref)), (case, e_ex, ref, e_osl)


def test_q2_matches_quadrature_of_the_definition():
    """Cases where GHK with 2^15 points has converged: E[W | y] from the same
    quadrature is checked first (it does not involve the difference), then
    E[log W | y].  (For deep truncations with strong correlation the GHK
    estimate itself still moves by percents at this N.)"""
    rng = np.random.default_rng(3)
    p, q = 3, 2
    u = inputs.qmc_points(1 << 15, q)
    for case in range(3):
        mu = rng.standard_normal(p)
        y = mu + 0.7 * rng.standard_normal(p)
        Sigma = inputs.wishart_sigma(rng, p)
        Delta = rng.uniform(-1, 1, size=(p, q))
        nu = rng.uniform(3, 12)
        a, b, c, Lam = _pair_quantities(y, mu, Sigma, Delta, nu)
        s1, s2 = np.sqrt(Lam[0, 0]), np.sqrt(Lam[1, 1])
        rho = Lam[0, 1] / (s1 * s2)

        def phi2(x1, x2):
            # P(Z1 <= x1, Z2 <= x2), unit variances, correlation rho, as a
            # one-dimensional integral over Z1
            f = lambda t: np.exp(-0.5 * t * t) / np.sqrt(2 * np.pi) * special.ndtr(
                (x2 - rho * t) / np.sqrt(1 - rho * rho))
            return integrate.quad(f, -np.inf, x1, epsabs=1e-14, epsrel=1e-12, limit=200)[0]

        # w = x / b, x with weight x^{a-1} e^{-x}
        x, wt = special.roots_genlaguerre(80, a - 1)
        w = x / b
        ph = np.array([phi2(np.sqrt(wk) * c[0] / s1, np.sqrt(wk) * c[1] / s2) for wk in w])
        ref_e1 = float(np.sum(wt * ph * np.log(w)) / np.sum(wt * ph))
        ref_e2 = float(np.sum(wt * ph * w) / np.sum(wt * ph))
        par = dict(pi=np.array([1.0]), mu=mu[None], Sigma=Sigma[None], Delta=Delta[None],
                   nu=np.array([nu]))
        for mode in (orc.NU_EXACT_FD, orc.NU_EXACT):
            out = orc.estep(y[None], par, u, nu_mode=mode, want=("e1", "e2"))
            e1, e2 = float(out["e1"][0, 0]), float(out["e2"][0, 0])
            assert abs(e2 - ref_e2) < 1e-5 * ref_e2, (case, mode, e2, ref_e2)
            assert abs(e1 - ref_e1) < 1e-4 * max(1.0, abs(ref_e1)), (case, mode, e1, ref_e1)


def test_chi2_quantile_derivative_matches_mpmath():
    """d/d(dof) of the chi-square quantile: implicit differentiation of the
    regularised incomplete gamma at 40 digits (mpmath) against the oracle's
    series.  In the far upper tail the series for dP/da cancels to about
    1/Q, hence the looser bar there."""
    mpmath.mp.dps = 40

    def quantile(u, dof):
        f = lambda x: mpmath.gammainc(dof / 2, 0, x / 2, regularized=True) - u
        return mpmath.findroot(f, orc.chi2_quantile(float(u), float(dof)))

    for u, dof, tol in [(0.3, 7.0, 1e-13), (1e-6, 5.5, 1e-13), (0.5, 30.0, 1e-13),
                        (0.01, 3.2, 1e-13), (0.9, 140.0, 1e-12), (0.97, 4.1, 1e-12),
                        (0.999999, 12.3, 1e-9)]:
        ref = float(mpmath.diff(lambda d: quantile(mpmath.mpf(u), d), mpmath.mpf(dof)))
        got = orc.chi2_quantile_ddof(u, dof)
        assert abs(got - ref) <= tol * abs(ref), (u, dof, got, ref)


def test_tangent_is_the_derivative_of_the_estimate():
    """The oracle's tangent of log J(a') (bound h sqrt(a'/a), dof 2a', the
    same points) against a fourth-order central difference of the plain GHK
    estimate over a': a dropped term or a wrong sign in the chain rule
    through the sequential bounds and draws, or in the chi-scale tangent,
    fails this."""
    rng = np.random.default_rng(11)
    for case, q in enumerate((1, 2, 3, 5, 6)):
        u = inputs.qmc_points(1024, q)
        A = rng.standard_normal((q, q))
        R = A @ A.T + q * np.eye(q)
        dg = np.sqrt(np.diag(R))
        R = R / np.outer(dg, dg)
        C = np.linalg.cholesky(R)
        h = rng.uniform(-1.0, 2.0, size=q)
        a = rng.uniform(2.5, 9.0)
        lt, dl = orc.ghk_tangent(h, C, a, u)
        lt0 = orc.ghk(h, C, 2 * a, u, moments=False)[0]
        assert lt == lt0
        f = lambda ap: orc.ghk(h * np.sqrt(ap / a), C, 2 * ap, u, moments=False)[0]
        dlt = 1e-3 * a
        fd = (8 * (f(a + dlt) - f(a - dlt)) - (f(a + 2 * dlt) - f(a - 2 * dlt))) / (12 * dlt)
        assert abs(dl - fd) < 1e-8 * max(abs(fd), 1e-2), (case, q, dl, fd)
