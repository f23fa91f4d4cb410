"""Oracle special functions pinned against scipy.special and mpmath."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special as sp


def test_norm_cdf_and_log(orc):
    """Against 50-digit mpmath.  Forming x/sqrt(2) in double costs a relative
    error of about x^2 ulp in the lower tail, so the bound grows with x^2."""
    mp.mp.dps = 50
    xs = np.concatenate([np.linspace(-8, 8, 161), [-12.5, -20, -29.99, -30.01, -37.3, -45, -80, 9, 15]])
    for x in xs:
        tol = 4e-16 * (4.0 + x * x)
        ref = mp.ncdf(mp.mpf(float(x)))
        if x > -37.5:
            assert orc.norm_cdf(x) == pytest.approx(float(ref), rel=tol)
            assert sp.ndtr(x) == pytest.approx(float(ref), rel=tol)  # the bound is realistic
        assert orc.log_norm_cdf(x) == pytest.approx(float(mp.log(ref)), rel=2e-15, abs=tol)


def test_log_norm_cdf_deep_tail_mpmath(orc):
    mp.mp.dps = 50
    for x in [-30.5, -38.0, -60.0, -200.0]:
        ref = float(mp.log(mp.ncdf(x)))
        assert orc.log_norm_cdf(x) == pytest.approx(ref, rel=1e-14)


def test_norm_quantile(orc):
    ps = np.concatenate([np.logspace(-300, -1, 60), np.linspace(0.02, 0.98, 49), 1 - np.logspace(-15, -2, 14)])
    for p in ps:
        w = orc.norm_quantile(p)
        ref = sp.ndtri(p)
        assert w == pytest.approx(ref, rel=5e-14, abs=1e-15)
        # round trip against the library CDF (a different implementation)
        if 1e-300 < p < 0.5:
            assert sp.ndtr(w) == pytest.approx(p, rel=2e-13)


def test_norm_quantile_log_below_double_range(orc):
    mp.mp.dps = 60
    for lp in [-800.0, -2000.0, -1e5]:
        w = orc.norm_quantile_log(lp)
        # log Phi(w) = lp checked in high precision
        assert float(mp.log(mp.ncdf(w))) == pytest.approx(lp, rel=1e-13)


def test_digamma(orc):
    for x in [1e-3, 0.1, 0.5, 1.0, 2.5, 3.7, 9.99, 10.0, 17.3, 150.0, 1e4]:
        assert orc.digamma(x) == pytest.approx(sp.digamma(x), rel=2e-14, abs=2e-14)


def test_incomplete_gamma(orc):
    for a in [0.5, 1.0, 3.0, 6.7, 12.5, 40.0]:
        for x in [1e-3, 0.3, 1.0, a, a + 1.0, 2 * a + 3, 60.0]:
            assert orc.gamma_p(a, x) == pytest.approx(sp.gammainc(a, x), rel=1e-13, abs=1e-300)
            assert orc.gamma_q(a, x) == pytest.approx(sp.gammaincc(a, x), rel=1e-12, abs=1e-300)


def test_chi2_quantile_against_mpmath(orc):
    mp.mp.dps = 40
    lo = 0.5 / 2 ** 30
    for dof in [5.0, 6.5, 10.0, 12.0, 19.3, 30.0]:
        for u in [lo, 1e-6, 0.01, 0.3, 0.5, 0.77, 0.999, 1 - lo]:
            x = orc.chi2_quantile(u, dof)
            a = mp.mpf(dof) / 2
            # P(a, x/2) = u in high precision, checked through the relative
            # sensitivity dP/dx * x / P (so the pin is on x, not on P)
            P = mp.gammainc(a, 0, mp.mpf(x) / 2, regularized=True)
            Q = 1 - P
            if u <= 0.5:
                err = abs(float(P) - u) / u
            else:
                err = abs(float(Q) - (1 - u)) / (1 - u)
            dens = float(mp.exp((a - 1) * mp.log(mp.mpf(x) / 2) - mp.mpf(x) / 2 - mp.loggamma(a))) / 2
            sens = dens * x / (u if u <= 0.5 else 1 - u)
            assert err / max(sens, 1e-30) < 1e-13, (dof, u, x)
            ref = 2 * sp.gammaincinv(dof / 2, u) if u <= 0.5 else 2 * sp.gammainccinv(dof / 2, 1 - u)
            assert x == pytest.approx(ref, rel=1e-12)
