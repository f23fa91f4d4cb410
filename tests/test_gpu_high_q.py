"""q above 8 (up to 12) on the GPU against the FP64 oracle.

At q >= 10 a pair's record (3 + q + q(q+1)/2 doubles) is wider than a
wave, so lanes carry a second entry; these cases check every entry.  Bar as
in tests/parity.py: FP64 1e-10 per quantity; FP32 1e-4 on moments and
statistics, 1e-7 on the log-likelihood; EM traces and parameters 1e-9.
Workload 6 is the high-q stress case (n = 202, p = q = 11, g = 2, N = 8192).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_06848_amd import native
    native.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def T(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def P(par, dev):
    return {k: T(v, dev) for k, v in par.items() if k in ("pi", "mu", "Sigma", "Delta", "nu")}


def gpu_estep(dev, y, par, u, **opt):
    from paper_2005_06848_amd import native
    print(f"[gpu] high-q estep n={y.shape[0]} p={y.shape[1]} q={par['Delta'].shape[2]} "
          f"g={len(par['pi'])} N={u.shape[0]} {opt}", flush=True)
    g = native.cfust_estep(T(y, dev), P(par, dev), T(u, dev), **opt)
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["loglik"] = float(out["loglik"][0])
    return out


@pytest.mark.parametrize("shape", [(21, 9, 9, 2, 129), (15, 6, 10, 3, 100), (19, 11, 11, 2, 257),
                                   (13, 12, 12, 2, 65), (7, 3, 12, 1, 64)])
def test_high_q_estep_parity(dev, orc, shape):
    from paper_2005_06848_amd import inputs
    import parity
    n, p, q, g, N = shape
    c = inputs.random_case(131 + n, n, p, q, g, N)
    ref = orc.estep(c["y"], c["params"], c["u"])
    got = gpu_estep(dev, c["y"], c["params"], c["u"])
    err = parity.estep_errors(got, ref, p, q)
    bad = {k: v for k, v in err.items() if not v <= TOL}
    assert not bad, err
    # the entries past the first 64 of each record are the last e4 entries
    assert np.max(np.abs(got["e4"][..., q - 1, q - 1])) > 0


def test_high_q_loglik_and_fp32(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.random_case(151, 40, 11, 11, 2, 1024)
    y, par, u = c["y"], c["params"], c["u"]
    ll_ref, lf_ref = orc.loglik(y, par, u, want_logf=True)
    print("[gpu] high-q loglik n=40 q=11", flush=True)
    ll, lf = native.cfust_loglik(T(y, dev), P(par, dev), T(u, dev), want_logf=True)
    assert abs(float(ll) - ll_ref) <= TOL * abs(ll_ref)
    assert np.max(np.abs(lf.cpu().numpy() - lf_ref)) <= TOL
    ref = orc.estep(y, par, u)
    got = gpu_estep(dev, y, par, u, precision="fp32")
    err = parity.estep_errors(got, ref, 11, 11)
    assert err["e3"] < 1e-4 and err["e4"] < 1e-4 and err["stats"] < 1e-4, err
    assert err["loglik"] < 1e-7, err


def test_high_q_em_fit_matches_oracle(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.config(6, n=60)
    u = c["u"][:1024]
    ref = orc.em_fit(c["y"], c["init"], u, max_iter=4, tol=0.0)
    print("[gpu] high-q em_fit workload 6 n=60 N=1024", flush=True)
    fit = native.cfust_em_fit(T(c["y"], dev), P(c["init"], dev), T(u, dev), max_iter=4, tol=0.0)
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=1e-9)
    err = parity.params_rel_err({k: fit[k].cpu().numpy() for k in ("pi", "mu", "Sigma", "Delta", "nu")},
                                ref)
    assert max(err.values()) < 1e-9, err


def test_workload6_full_size_vs_oracle(dev):
    """Workload 6 at full size (n = 202, N = 8192) in one launch against the
    oracle over all observations: every per-pair output, the partial sums
    and the log-likelihood."""
    from paper_2005_06848_amd import inputs
    import oracle_pool
    import parity
    c = inputs.config(6)
    y, par, u = c["y"], c["init"], c["u"]
    got = gpu_estep(dev, y, par, u)
    print("[cpu] oracle E-step, workload 6, all observations", flush=True)
    ref = oracle_pool.estep_parallel(y, par, u)
    err = parity.estep_errors(got, ref, 11, 11)
    print(err, flush=True)
    assert max(err.values()) <= TOL, err


def test_workload6_exact_fit_ends_cleanly(dev):
    """The whole fit of the stress workload (n = 202, p = q = 11, g = 2,
    N = 8192) with the exact nu step, from the k-means start, for up to 600
    iterations.  With about 200 free parameters per component and 202
    observations one component degenerates (its Sigma turns singular, where
    the likelihood is unbounded); the fit must end either by Aitken's rule or
    with ENOTPD naming that component (the new Sigma's pivot guard), never
    with a non-finite value.  l rises monotonically (up to 1e-9 relative)
    over the first 60 iterations."""
    from paper_2005_06848_amd import inputs, native
    c = inputs.config(6)
    print("[gpu] high-q whole fit workload 6, exact nu (max 600 iterations)", flush=True)
    try:
        fit = native.cfust_em_fit(T(c["y"], dev), P(c["init"], dev), T(c["u"], dev),
                                  max_iter=600, tol=1e-6, nu_mode="exact")
        end = "converged" if fit["n_iter"] < 600 else "iteration cap"
    except native.CfustError as e:
        assert e.code == native.ENOTPD and e.bad in (0, 1), str(e)
        fit, end = e.partial, f"ENOTPD, component {e.bad}"
    tr = np.array(fit["trace"])
    print(f"  {end} after {fit['n_iter']} iterations; l {tr[0]:.4f} -> max {tr.max():.4f} "
          f"at {tr.argmax()} -> {tr[-1]:.4f}")
    assert np.all(np.isfinite(tr))
    d = np.diff(tr[:61])
    assert np.all(d > -1e-9 * np.abs(tr[1:61])), d.min()


def test_high_q_forms_rejected(dev):
    from paper_2005_06848_amd import inputs, native
    c = inputs.random_case(161, 10, 11, 11, 2, 64)
    y, par, u = T(c["y"], dev), P(c["params"], dev), T(c["u"], dev)
    with pytest.raises(native.CfustError):
        native.cfust_estep(y, par, u, reorder=True)
    with pytest.raises(native.CfustError):
        native.cfust_em_fit_batched(y, [10], [2], par, u, max_iter=2)
    with pytest.raises(native.CfustError):
        native.cfust_em_fit_multistart(y, [par, par], u, burn_in=1, max_iter=2)
    with pytest.raises(native.CfustError):
        native.cfust_ghk_batch(T(np.zeros((2, 11)), dev), T(np.broadcast_to(np.eye(11), (2, 11, 11)), dev),
                               T(np.full(2, 8.0), dev), u)
