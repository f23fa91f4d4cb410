"""Randomised QMC error bars of the log-likelihood (cfust_loglik_rqmc) and
rank-1 lattice points as an alternative point set.

Every shifted estimate equals the oracle's with the same points (1e-10);
the RQMC means of Sobol and lattice points agree with each other and with a
2^14-point randomised lattice estimate within five combined standard
errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_06848_amd import native
    native.lib()
    return torch.device("cuda:0")


def T(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def test_rqmc_error_bars(dev, orc):
    from paper_2005_06848_amd import inputs, native
    c = inputs.config(1)
    y, par = c["y"], c["init"]
    q, N, K = c["q"], 1024, 16
    par_d = {k: T(v, dev) for k, v in par.items()}
    sob = np.stack([inputs.qmc_points(N, q, seed=100 + k) for k in range(K)])
    z = inputs.korobov_generator(N, q + 1)
    lat = np.stack([inputs.lattice_points(N, q, seed=200 + k, z=z) for k in range(K)])
    print("[gpu] rqmc config 1, K=16, N=1024", flush=True)
    ll_s, m_s, se_s = native.cfust_loglik_rqmc(T(y, dev), par_d, T(sob, dev))
    ll_l, m_l, se_l = native.cfust_loglik_rqmc(T(y, dev), par_d, T(lat, dev))
    for k in range(2):
        np.testing.assert_allclose(ll_s[k], orc.loglik(y, par, sob[k]), rtol=1e-10)
        np.testing.assert_allclose(ll_l[k], orc.loglik(y, par, lat[k]), rtol=1e-10)
    assert se_s > 0 and se_l > 0
    # reference: randomised lattice with 2^14 points and K shifts (every
    # estimate here is unbiased; the comparisons use combined errors)
    zb = inputs.korobov_generator(1 << 14, q + 1)
    big = np.stack([inputs.lattice_points(1 << 14, q, seed=300 + k, z=zb) for k in range(K)])
    _, m_b, se_b = native.cfust_loglik_rqmc(T(y, dev), par_d, T(big, dev))
    print(f"  sobol {m_s:.6f} +- {se_s:.2e}; lattice {m_l:.6f} +- {se_l:.2e}; "
          f"lattice 2^14 {m_b:.6f} +- {se_b:.2e}")
    # five combined standard errors: the error of a shifted rule is not
    # Gaussian and K shifts estimate its spread only roughly
    assert abs(m_s - m_l) < 5 * np.hypot(se_s, se_l)
    assert abs(m_s - m_b) < 5 * np.hypot(se_s, se_b)
    assert abs(m_l - m_b) < 5 * np.hypot(se_l, se_b)
    assert se_b < se_l  # more points, smaller error bar
