"""Pins of the oracle's Genz-Bretz variable ordering (orc_genz_order) and of
the integrals taken in that order.

The ordering is the prioritisation of Genz & Bretz (2009, section 4.1.3):
step i places the unplaced variable with the smallest standardised
conditional bound given the truncated means of the variables already
placed.  The pins check it against
  - two cases worked by hand (independent variables: ascending h; a strongly
    correlated pair that moves a larger bound ahead of a smaller one);
  - the regression form of the same conditional bound, E[Z_j | Z_P = z_P] =
    R_jP R_PP^-1 z_P and Var = 1 - R_jP R_PP^-1 R_Pj, evaluated with numpy
    solves (a different route from the oracle's Cholesky recurrence);
  - the Cholesky identity Cp Cp^T = R[perm][perm];
and the ordered GHK estimate against
  - the same integral in the natural order (both estimate one quantity);
  - relabelling: permuting h and R relabels the moments and nothing else;
  - the E-step and log-likelihood with and without ordering.
"""
import numpy as np
from scipy import stats

import oracle as orc
from paper_2005_06848_amd import inputs


def _trunc_mean(b):
    """E[Z | Z <= b] for Z ~ N(0,1), by scipy."""
    return -stats.norm.pdf(b) / stats.norm.cdf(b)


def test_independent_variables_go_in_ascending_order():
    perm, Cp = orc.genz_order([3.0, -1.0, 0.5], np.eye(3))
    assert list(perm) == [1, 2, 0]
    assert np.array_equal(Cp, np.eye(3))


def test_correlated_pair_worked_by_hand():
    # h = (0, 0.5, 1), corr(Z0, Z1) = 0.95, Z2 independent.
    # step 0: bounds (0, 0.5, 1) -> Z0; y0 = -phi(0)/Phi(0) = -0.79788.
    # step 1: Z1: (0.5 + 0.95 * 0.79788) / sqrt(1 - 0.95^2) = 4.029;
    #         Z2: 1.0 -> Z2 goes second although h1 < h2.
    R = np.array([[1.0, 0.95, 0.0], [0.95, 1.0, 0.0], [0.0, 0.0, 1.0]])
    perm, Cp = orc.genz_order([0.0, 0.5, 1.0], R)
    assert list(perm) == [0, 2, 1]
    want = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.95, 0.0, np.sqrt(1 - 0.95 ** 2)]])
    assert np.allclose(Cp, want, atol=1e-15)


def test_order_matches_regression_form_of_the_conditional_bound():
    rng = np.random.default_rng(11)
    for case in range(40):
        q = int(rng.integers(2, 9))
        R = inputs.lkj_corr(rng, q, 1.0)
        h = rng.uniform(-2.5, 3.0, size=q)
        perm, Cp = orc.genz_order(h, R)
        assert sorted(perm) == list(range(q))
        # Cholesky identity of the permuted matrix
        Rp = R[np.ix_(perm, perm)]
        assert np.allclose(Cp @ Cp.T, Rp, atol=1e-13)
        assert np.allclose(np.triu(Cp, 1), 0.0)
        # at every step the placed variable minimises the conditional bound
        ys = []
        for i in range(q):
            P = list(perm[:i])
            zP = Cp[:i, :i] @ np.array(ys) if i else np.zeros(0)
            bounds = {}
            for j in range(q):
                if j in P:
                    continue
                if i:
                    w = np.linalg.solve(R[np.ix_(P, P)], R[P, j])
                    m, v = w @ zP, 1.0 - R[j, P] @ w
                else:
                    m, v = 0.0, 1.0
                bounds[j] = (h[j] - m) / np.sqrt(v)
            best = min(bounds.values())
            assert bounds[perm[i]] <= best + 1e-12 * max(1.0, abs(best))
            ys.append(_trunc_mean(bounds[perm[i]]))


def _cases(rng, m, q):
    for _ in range(m):
        R = inputs.lkj_corr(rng, q, 1.0)
        h = rng.uniform(-1.0, 2.0, size=q)
        dof = float(rng.uniform(4.0, 15.0))
        yield h, R, dof


def test_ordered_and_natural_estimates_agree():
    rng = np.random.default_rng(12)
    u = inputs.qmc_points(1 << 16, 5)
    for h, R, dof in _cases(rng, 6, 5):
        C = np.linalg.cholesky(R)
        l0, m0, s0 = orc.ghk(h, C, dof, u)
        l1, m1, s1, perm = orc.ghk_ordered(h, R, dof, u)
        assert abs(l1 - l0) < 2e-4 * max(1.0, abs(l0))
        assert np.allclose(m1, m0, atol=3e-3)
        assert np.allclose(s1, s0, atol=6e-3)
        assert np.allclose(s1, s1.T, atol=1e-12)


def test_relabelling_only_relabels_the_moments():
    rng = np.random.default_rng(13)
    u = inputs.qmc_points(2048, 4)
    # weak correlations: the order is the ascending order of h, here the
    # 4-cycle (1, 3, 0, 2), which is not its own inverse
    R = np.eye(4) + 0.05 * (np.ones((4, 4)) - np.eye(4))
    h = np.array([0.5, -1.0, 1.5, 0.0])
    l0, m0, s0, perm = orc.ghk_ordered(h, R, 7.0, u)
    assert list(perm) == [1, 3, 0, 2]
    for _ in range(5):
        R = inputs.lkj_corr(rng, 4, 1.0)
        h = rng.uniform(-1.0, 2.0, size=4)
        l0, m0, s0, p0 = orc.ghk_ordered(h, R, 7.0, u)
        sig = rng.permutation(4)
        l1, m1, s1, p1 = orc.ghk_ordered(h[sig], R[np.ix_(sig, sig)], 7.0, u)
        assert list(sig[p1]) == list(p0)
        assert abs(l1 - l0) <= 1e-13 * max(1.0, abs(l0))
        assert np.allclose(m1, m0[sig], rtol=1e-12, atol=1e-14)
        assert np.allclose(s1, s0[np.ix_(sig, sig)], rtol=1e-12, atol=1e-14)


def test_estep_and_loglik_with_ordering_agree_with_natural_order():
    c = inputs.random_case(31, n=12, p=4, q=3, g=2, n_qmc=1 << 14)
    y, par, u = c["y"], c["params"], c["u"]
    a = orc.estep(y, par, u)
    b = orc.estep(y, par, u, reorder=True)
    # pairs that carry weight; far-tail pairs (responsibility ~1e-8, log f
    # ~ -30) are dominated by the chi-square column of the points in either
    # order and stay unconverged at 2^20 points
    w = a["tau"] > 1e-3
    assert w.sum() >= 12
    assert np.allclose(b["logf"][w], a["logf"][w], atol=2e-4)
    assert np.allclose(b["e2"][w], a["e2"][w], rtol=2e-3)
    assert np.allclose(b["e3"][w], a["e3"][w], rtol=5e-3, atol=5e-3)
    assert np.allclose(b["e4"][w], a["e4"][w], rtol=5e-3, atol=1e-2)
    assert np.allclose(b["stats"], a["stats"], rtol=2e-3, atol=2e-3)
    ll = orc.loglik(y, par, u, reorder=True)
    assert abs(ll - b["loglik"]) < 1e-9 * abs(ll)
    fit = orc.em_fit(y, par, u, max_iter=2, tol=0.0, reorder=True)
    assert abs(fit["trace"][0] - b["loglik"]) < 1e-9 * abs(ll)


def test_ordering_reduces_the_randomised_qmc_error_on_a_hard_case():
    # an equicorrelated q = 6 orthant with one very restrictive bound placed
    # last: the natural order wastes most points on the first five variables
    q, K = 6, 16
    R = 0.6 * np.ones((q, q)) + 0.4 * np.eye(q)
    h = np.array([1.5, 1.2, 1.0, 0.8, 0.6, -2.0])
    C = np.linalg.cholesky(R)
    nat, ordd = [], []
    for k in range(K):
        u = inputs.qmc_points(1024, q, seed=1000 + k)
        nat.append(orc.ghk(h, C, 8.0, u, moments=False)[0])
        ordd.append(orc.ghk_ordered(h, R, 8.0, u, moments=False)[0])
    se_nat = np.std(nat, ddof=1) / np.sqrt(K)
    se_ord = np.std(ordd, ddof=1) / np.sqrt(K)
    assert abs(np.mean(nat) - np.mean(ordd)) < 5 * np.hypot(se_nat, se_ord)
    assert se_ord < 0.5 * se_nat
