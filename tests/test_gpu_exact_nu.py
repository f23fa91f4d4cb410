"""Exact E[log W | y] (nu_mode "exact": the derivative of the GHK estimate
itself, carried as a tangent through integral A) on the GPU against the
FP64 oracle's own tangent (nu_mode EXACT).

Bars: FP64 1e-10 per quantity as in tests/parity.py, e1 included, EM traces
and parameters to 1e-9; FP32 1e-4 on e1 and the moments, 1e-7 on l.  The
exact nu step makes the ECM monotone up to the QMC estimates' small
inconsistency, which the monotonicity test checks."""
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
    print(f"[gpu] exact estep n={y.shape[0]} p={y.shape[1]} q={par['Delta'].shape[2]} "
          f"g={len(par['pi'])} N={u.shape[0]} {opt}", flush=True)
    g = native.cfust_estep(T(y, dev), P(par, dev), T(u, dev), nu_mode="exact", **opt)
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["loglik"] = float(out["loglik"][0])
    return out


@pytest.mark.parametrize("shape", [(1, None), (0, (90, 3, 2, 3, 300)), (0, (65, 2, 4, 2, 1000)),
                                   (0, (33, 5, 1, 2, 129))])
def test_exact_estep_parity(dev, orc, shape):
    from paper_2005_06848_amd import inputs
    import parity
    if shape[0] == 1:
        c = inputs.config(1)
        y, par, u = c["y"], c["init"], c["u"]
    else:
        n, p, q, g, N = shape[1]
        c = inputs.random_case(31 + n, n, p, q, g, N)
        y, par, u = c["y"], c["params"], c["u"]
    ref = orc.estep(y, par, u, nu_mode=orc.NU_EXACT)
    got = gpu_estep(dev, y, par, u)
    err = parity.estep_errors(got, ref, y.shape[1], par["Delta"].shape[2])
    bad = {k: v for k, v in err.items() if not v <= TOL}
    assert not bad, err
    # the exact and one-step-late e1 differ on this data (the test is not vacuous)
    osl = orc.estep(y, par, u, nu_mode=orc.NU_OSL, want=("e1",))["e1"]
    assert np.max(np.abs(osl - ref["e1"])) > 1e-6


def test_exact_em_fit_matches_oracle(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.config(1)
    ref = orc.em_fit(c["y"], c["init"], c["u"], max_iter=10, tol=0.0, nu_mode=orc.NU_EXACT)
    print("[gpu] exact em_fit config 1", flush=True)
    fit = native.cfust_em_fit(T(c["y"], dev), P(c["init"], dev), T(c["u"], dev), max_iter=10,
                              tol=0.0, nu_mode="exact")
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=1e-9)
    err = parity.params_rel_err({k: fit[k].cpu().numpy() for k in ("pi", "mu", "Sigma", "Delta", "nu")},
                                ref)
    assert max(err.values()) < 1e-9, err


def test_exact_fp32_form(dev, orc):
    """FP32 integrand: e1 through the FP32 tangent (its weighted sum in
    FP64), to 1e-4 relative like the other moments, at q = 3, 5 and 6:
    (200, 4, 3, 2, 2048) spreads 400 pairs over 8 waves each,
    (100, 5, 5, 2, 1024) uses the q = 5 four-wave split kernel, and
    (2100, 6, 6, 2, 1024) the one-wave kernel."""
    from paper_2005_06848_amd import inputs
    import parity
    for seed, (n, p, q, g, N) in ((41, (200, 4, 3, 2, 2048)), (43, (100, 5, 5, 2, 1024)),
                                  (47, (2100, 6, 6, 2, 1024))):
        c = inputs.random_case(seed, n, p, q, g, N)
        ref = orc.estep(c["y"], c["params"], c["u"], nu_mode=orc.NU_EXACT)
        got = gpu_estep(dev, c["y"], c["params"], c["u"], precision="fp32")
        err = parity.estep_errors(got, ref, p, q)
        print(f"  fp32 exact q={q}:", err, flush=True)
        assert err["e1"] < 1e-4 and err["stats"] < 1e-4 and err["loglik"] < 1e-7, (q, err)
        assert max(err["e2"], err["e3"], err["e4"]) < 1e-4, (q, err)


def test_exact_fp32_config3_subsample(dev):
    """FP32 exact E-step on the seeded 2000-observation subsample of the
    precision workload (n = 200000, p = q = 6, g = 4, N = 8192) against the
    oracle over the same observations: e1 and the moments to 1e-4, l to
    1e-7."""
    from paper_2005_06848_amd import inputs
    import oracle
    import oracle_pool
    import parity
    c = inputs.config(3)
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(c["n"], size=2000, replace=False))
    y = c["y"][idx]
    got = gpu_estep(dev, y, c["init"], c["u"], precision="fp32")
    print("[cpu] oracle exact E-step on the 2000-observation subsample", flush=True)
    ref = oracle_pool.estep_parallel(y, c["init"], c["u"], nu_mode=oracle.NU_EXACT)
    err = parity.estep_errors(got, ref, c["p"], c["q"])
    print("  fp32 exact config-3 subsample:", err, flush=True)
    assert err["e1"] < 1e-4 and err["stats"] < 1e-4 and err["loglik"] < 1e-7, err
    assert max(err["e2"], err["e3"], err["e4"]) < 1e-4, err


def test_exact_high_q_workload6(dev, orc):
    """FP64 exact E-step at q = 11 on the stress workload (n = 202,
    p = q = 11, g = 2, N = 8192; 404 pairs split over several waves each)
    against the oracle at the FP64 bar."""
    from paper_2005_06848_amd import inputs
    import parity
    c = inputs.config(6)
    ref = orc.estep(c["y"], c["init"], c["u"], nu_mode=orc.NU_EXACT)
    got = gpu_estep(dev, c["y"], c["init"], c["u"])
    err = parity.estep_errors(got, ref, 11, 11)
    print("  fp64 exact q=11:", err, flush=True)
    bad = {k: v for k, v in err.items() if not v <= TOL}
    assert not bad, err


def test_exact_batched_matches_oracle(dev, orc):
    """The batched form with the exact nu step: three problems of uneven n
    and g, 3 EM iterations in one batched launch sequence (FP64), against
    the oracle's exact EM per problem."""
    from paper_2005_06848_amd import inputs, native
    import parity
    cases = [inputs.random_case(301 + k, n, 3, 2, g, 512) for k, (n, g) in
             enumerate(((150, 2), (90, 3), (210, 1)))]
    u = cases[0]["u"]
    keys = ("pi", "mu", "Sigma", "Delta", "nu")
    y = np.concatenate([c["y"] for c in cases])
    par = {k: np.concatenate([c["params"][k] for c in cases]) for k in keys}
    ns, gs = [c["n"] for c in cases], [c["g"] for c in cases]
    print(f"[gpu] batched exact n={ns} g={gs}", flush=True)
    fit, trace, n_iter, status = native.cfust_em_fit_batched(
        T(y, dev), ns, gs, P(par, dev), T(u, dev), max_iter=3, tol=0.0, nu_mode="exact")
    assert np.all(status == 0), status
    off = np.concatenate([[0], np.cumsum(gs)])
    for k, c in enumerate(cases):
        ref = orc.em_fit(c["y"], c["params"], u, max_iter=3, tol=0.0, nu_mode=orc.NU_EXACT)
        np.testing.assert_allclose(trace[k, :4], ref["trace"], rtol=1e-10)
        got = {kk: fit[kk].cpu().numpy()[off[k]:off[k + 1]] for kk in keys}
        err = parity.params_rel_err(got, ref)
        assert max(err.values()) < 1e-9, (k, err)


def test_exact_em_is_monotone(dev):
    """With the exact nu step every CM step maximises its conditional
    likelihood, so l^(t) does not decrease (up to the small inconsistency of
    the QMC estimates: the moments are ratios of estimates, not the exact
    derivatives of the estimated likelihood)."""
    from paper_2005_06848_amd import inputs, native
    c = inputs.config(2, n=4000)
    print("[gpu] exact em_fit monotone n=4000", flush=True)
    fit = native.cfust_em_fit(T(c["y"], dev), P(c["init"], dev), T(c["u"], dev), max_iter=40,
                              tol=0.0, nu_mode="exact")
    tr = np.array(fit["trace"])
    steps = np.diff(tr)
    print("  smallest step", steps.min(), "final", tr[-1])
    assert np.all(steps > -1e-8 * np.abs(tr[1:]))


def test_exact_rejected_with_surrogate(dev):
    from paper_2005_06848_amd import inputs, native, surrogate
    c = inputs.random_case(5, 50, 6, 6, 2, 64)
    net = native.Surrogate.load(surrogate.DEFAULT_PATH)
    with pytest.raises(native.CfustError):
        native.cfust_estep(T(c["y"], dev), P(c["params"], dev), T(c["u"], dev), nu_mode="exact",
                           surrogate=net)
