"""Pins of the seeded input generators (no method arithmetic lives there)."""
import math

import numpy as np
import torch
from scipy import stats

from paper_2005_06848_amd import inputs


def test_qmc_points_are_shifted_sobol():
    u = inputs.qmc_points(1024, 3)
    assert u.shape == (1024, 4) and np.all(u > 0) and np.all(u < 1)
    eng = torch.quasirandom.SobolEngine(4, scramble=False)
    raw = eng.draw(1024, dtype=torch.float64).numpy()
    x = np.rint(raw * 2 ** 30).astype(np.int64)
    back = np.rint(u * 2 ** 30 - 0.5).astype(np.int64)
    shift = back[0] ^ x[0]
    np.testing.assert_array_equal(back ^ shift[None, :], x)


def test_cfust_sampler_mean():
    """E[Y] = mu + kappa_nu Delta 1_q for the hidden-variable draw."""
    rng = np.random.default_rng(0)
    mu = np.array([[1.0, -2.0]])
    Sigma = np.array([[[1.0, 0.2], [0.2, 0.5]]])
    Delta = np.array([[[1.0, -0.5], [0.3, 0.8]]])
    nu = np.array([7.0])
    y, _ = inputs.sample_cfust(rng, 400000, [1.0], mu, Sigma, Delta, nu)
    expect = mu[0] + inputs.kappa_nu(7.0) * Delta[0].sum(1)
    se = y.std(0) / math.sqrt(y.shape[0])
    assert np.all(np.abs(y.mean(0) - expect) < 5 * se)


def test_lkj_marginal_is_beta():
    """LKJ(eta) in dimension d: (r + 1)/2 ~ Beta(eta - 1 + d/2, eta - 1 + d/2),
    Beta(4, 4) for d = 6, eta = 2."""
    rng = np.random.default_rng(1)
    rs = []
    for _ in range(4000):
        R = inputs.lkj_corr(rng, 6, 2.0)
        assert np.allclose(np.diag(R), 1.0) and np.linalg.eigvalsh(R).min() > 0
        rs.append(R[0, 1])
        rs.append(R[2, 5])
    ks = stats.kstest((np.array(rs) + 1) / 2, stats.beta(4, 4).cdf)
    assert ks.pvalue > 1e-3


def test_lattice_rule_structure():
    """A rank-1 lattice rule with generator z integrates exp(2 pi i h.x) to
    zero unless h.z = 0 mod n: every one-dimensional projection is a shifted
    full grid, and low-order Fourier modes integrate to zero."""
    n, q = 1024, 3
    z = inputs.korobov_generator(n, q + 1)
    assert z[0] == 1 and np.all(z % 2 == 1)
    x = inputs.lattice_points(n, q, seed=5, z=z, tent=False)
    for j in range(q + 1):
        grid = np.sort(np.round((x[:, j] - x[0, j]) * n) % n)
        np.testing.assert_array_equal(grid, np.arange(n))
    for h in ([1, 0, 0, 0], [0, 2, 0, 0], [1, 1, 0, 0], [0, 1, -1, 1], [3, 0, 0, -2]):
        h = np.array(h)
        assert (h @ z) % n != 0
        assert abs(np.mean(np.exp(2j * np.pi * (x @ h)))) < 1e-12
    u = inputs.lattice_points(n, q, seed=5, z=z)
    assert np.all(u > 0) and np.all(u < 1)
