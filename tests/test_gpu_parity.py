"""GPU path (HIP kernels through the C ABI) against the FP64 oracle.

Bar (FP64): 1e-10 per quantity, measured as in tests/parity.py."""
import math
import sys

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


def T(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def gpu_params(par, dev):
    return {k: T(v, dev) for k, v in par.items() if k in ("pi", "mu", "Sigma", "Delta", "nu")}


def to_np(d):
    out = {}
    for k, v in d.items():
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
            if k == "loglik":
                v = float(v[0])
        out[k] = v
    return out


def run_pair(dev, y, par, u, precision="fp64"):
    from paper_2005_06848_amd import native
    print(f"[gpu] estep n={y.shape[0]} p={y.shape[1]} q={par['Delta'].shape[2]} g={len(par['pi'])} "
          f"N={u.shape[0]} {precision}", flush=True)
    g = native.cfust_estep(T(y, dev), gpu_params(par, dev), T(u, dev), precision=precision)
    return to_np(g)


def check(err, tol=TOL):
    bad = {k: v for k, v in err.items() if not (v <= tol)}
    assert not bad, err


def test_special_functions(dev):
    from scipy import special as sp
    from paper_2005_06848_amd import native
    import torch
    x = np.concatenate([np.linspace(-35, 8, 300), [-36.5, -40.0, -60.0]])
    phi = native.cfust_eval_special(0, T(x, dev)).cpu().numpy()
    lphi = native.cfust_eval_special(1, T(x, dev)).cpu().numpy()
    ok = x > -37
    rel = np.abs(phi[ok] / sp.ndtr(x[ok]) - 1)
    assert np.all(rel <= 5e-16 * (4 + x[ok] ** 2)), rel.max()
    np.testing.assert_allclose(lphi, sp.log_ndtr(x), rtol=1e-14)
    p = np.concatenate([np.logspace(-300, -1, 80), np.linspace(0.02, 0.98, 49)])
    w = native.cfust_eval_special(2, T(p, dev)).cpu().numpy()
    ref = sp.ndtri(p)
    assert np.all(np.abs(w - ref) <= 1e-14 * np.maximum(np.abs(ref), 1.0)), np.max(np.abs(w - ref))
    lp = np.array([-800.0, -2000.0, -1e5])
    wl = native.cfust_eval_special(3, T(lp, dev)).cpu().numpy()
    np.testing.assert_allclose(sp.log_ndtr(wl), lp, rtol=1e-13)
    uu = np.array([0.5 / 2 ** 30, 1e-6, 0.3, 0.5, 0.77, 1 - 0.5 / 2 ** 30])
    for dof in [5.0, 9.3, 14.0, 30.0]:
        q = native.cfust_eval_special(4, T(uu, dev), T(np.full(uu.size, dof), dev)).cpu().numpy()
        ref = np.where(uu <= 0.5, 2 * sp.gammaincinv(dof / 2, uu), 2 * sp.gammainccinv(dof / 2, 1 - uu))
        np.testing.assert_allclose(q, ref, rtol=1e-13)
    xs = np.array([0.3, 1.0, 2.5, 7.9, 8.0, 30.0, 101.0])
    np.testing.assert_allclose(native.cfust_eval_special(5, T(xs, dev)).cpu().numpy(), sp.digamma(xs), rtol=1e-14)
    np.testing.assert_allclose(native.cfust_eval_special(6, T(xs, dev)).cpu().numpy(), sp.polygamma(1, xs), rtol=1e-11)
    # the device log and sqrt used inside the quantile
    xl = np.concatenate([np.logspace(-300, 300, 200), [0.5, 1.0, 1.0 + 2 ** -40, 2.0]])
    np.testing.assert_allclose(native.cfust_eval_special(9, T(xl, dev)).cpu().numpy(), np.log(xl), rtol=4e-16, atol=4e-16)
    xs2 = np.logspace(-200, 200, 200)
    np.testing.assert_allclose(native.cfust_eval_special(10, T(xs2, dev)).cpu().numpy(), np.sqrt(xs2), rtol=3e-16)
    # pieces of the exact nu step: the chi-square quantile's derivative in
    # the dof (against the oracle's, itself pinned by mpmath) and the
    # inverse Mills ratio phi/Phi (against scipy), FP64 and FP32
    import oracle
    for dof in [3.5, 9.3, 17.0, 60.0, 212.0]:
        uq = np.array([0.5 / 2 ** 30, 1e-6, 0.3, 0.5, 0.77, 0.999, 0.99994])
        d = native.cfust_eval_special(11, T(uq, dev), T(np.full(uq.size, dof), dev)).cpu().numpy()
        ref = np.array([oracle.chi2_quantile_ddof(v, dof) for v in uq])
        tol = np.where(uq > 0.99, 1e-10, 1e-12)
        assert np.all(np.abs(d - ref) <= tol * np.abs(ref)), (dof, d, ref)
    xm = np.concatenate([np.linspace(-30, 9, 157), [-200.0, 20.0]])
    # below zero phi/Phi = sqrt(2/pi) / erfcx(-x/sqrt 2) (no cancellation)
    with np.errstate(invalid="ignore"):
        mref = np.where(xm < 0, np.sqrt(2 / np.pi) / sp.erfcx(-xm / np.sqrt(2)),
                        np.exp(-0.5 * xm * xm) / np.sqrt(2 * np.pi) / sp.ndtr(xm))
    m64 = native.cfust_eval_special(12, T(xm, dev)).cpu().numpy()
    np.testing.assert_allclose(m64, mref, rtol=1e-13)
    # FP32: above zero the ratio carries exp(-x^2/2), whose float argument
    # has a relative rounding of about x^2 * 6e-8 / 2 (2.4e-6 at x = 9)
    m32 = native.cfust_eval_special(13, T(xm, dev)).cpu().numpy()
    ok32 = xm < 9  # above that phi(x) is below the float range
    np.testing.assert_allclose(m32[ok32], mref[ok32], rtol=1e-5)
    # the per-call cost probes compute what the point loop computes: the
    # coordinate step Phi^-1(u Phi(b)) (against scipy), and the weight's
    # accumulation into a running sum with its reference exponent (exact:
    # power-of-two scalings and one rounded add, redone in numpy)
    rng = np.random.default_rng(9)
    b = rng.uniform(-8.0, 5.0, 400)
    u = rng.uniform(0.0, 1.0, 400)
    wref = sp.ndtri(u * sp.ndtr(b))
    w64 = native.cfust_eval_special(14, T(b, dev), T(u, dev)).cpu().numpy()
    assert np.all(np.abs(w64 - wref) <= 1e-12 * np.maximum(np.abs(wref), 1.0))
    w32 = native.cfust_eval_special(15, T(b, dev), T(u, dev)).cpu().numpy()
    assert np.all(np.abs(w32 - wref) <= 2e-5 * np.maximum(np.abs(wref), 1.0))
    m = rng.uniform(0.5, 1.0, 401)
    e = rng.integers(-20, 21, 401).astype(np.float64)
    e[::7] += 70.0  # some points move the reference (re-scaling the sum)
    nb = np.arange(401) ^ 1
    nb[nb >= 401] = 400
    for fn, kr, mm in ((16, 64, m), (17, 32, m.astype(np.float32).astype(np.float64))):
        # the running sum is a double in both; the FP32 weight is a float
        s0, ref0 = m[nb].copy(), e[nb].copy()
        up = e > ref0 + kr
        s0[up] *= 2.0 ** (ref0[up] - e[up])
        ref0[up] = e[up]
        expect = s0 + mm * 2.0 ** (e - ref0)
        got = native.cfust_eval_special(fn, T(m, dev), T(e, dev)).cpu().numpy()
        np.testing.assert_array_equal(got, expect)


def test_estep_config1(dev, orc):
    from paper_2005_06848_amd import inputs
    c = inputs.config(1)
    ref = orc.estep(c["y"], c["init"], c["u"])
    gpu = run_pair(dev, c["y"], c["init"], c["u"])
    err = __import__("parity").estep_errors(gpu, ref, c["p"], c["q"])
    print(err)
    check(err)


SHAPES = [  # n, p, q, g, N : tiles, ragged tails, N below and above one wave
    (1, 1, 1, 1, 64), (63, 2, 1, 2, 100), (64, 3, 3, 1, 63), (65, 2, 2, 3, 1),
    (130, 5, 4, 2, 200), (37, 6, 6, 3, 129), (20, 4, 5, 4, 256), (17, 3, 2, 6, 77),
    (9, 7, 7, 2, 65), (5, 8, 8, 2, 70), (40, 1, 3, 2, 128),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_estep_shapes(dev, orc, shape):
    from paper_2005_06848_amd import inputs
    n, p, q, g, N = shape
    c = inputs.random_case(100 + sum(shape), n, p, q, g, N)
    ref = orc.estep(c["y"], c["params"], c["u"])
    gpu = run_pair(dev, c["y"], c["params"], c["u"])
    err = __import__("parity").estep_errors(gpu, ref, p, q)
    check(err)


def test_estep_config2_reduced(dev, orc):
    """The config-2 recipe (p=q=4, g=3, N=4096) on its first 160 observations."""
    from paper_2005_06848_amd import inputs
    c = inputs.config(2)
    y = c["y"][:160]
    ref = orc.estep(y, c["init"], c["u"])
    gpu = run_pair(dev, y, c["init"], c["u"])
    err = __import__("parity").estep_errors(gpu, ref, 4, 4)
    print(err)
    check(err)


def test_estep_config2_full_vs_oracle(dev):
    """Full config 2 (n=20000, 60000 pairs) in the benchmark's launch
    configuration against the oracle run over all observations: every
    per-pair output, all partial sums s1..s8 and the log-likelihood at the
    FP64 bar."""
    from paper_2005_06848_amd import inputs
    import oracle_pool
    import parity
    c = inputs.config(2)
    gpu = run_pair(dev, c["y"], c["init"], c["u"])
    print("[cpu] oracle E-step on all 20000 observations", flush=True)
    ref = oracle_pool.estep_parallel(c["y"], c["init"], c["u"])
    err = parity.estep_errors(gpu, ref, 4, 4)
    print(err, flush=True)
    check(err)
    np.testing.assert_allclose(gpu["tau"].sum(1), 1.0, rtol=1e-13)


def test_loglik_and_mstep(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.random_case(7, 300, 3, 3, 3, 512)
    ll_gpu, lf_gpu = native.cfust_loglik(T(c["y"], dev), gpu_params(c["params"], dev), T(c["u"], dev),
                                         want_logf=True)
    ll_ref, lf_ref = orc.loglik(c["y"], c["params"], c["u"], want_logf=True)
    assert float(ll_gpu.cpu()[0]) == pytest.approx(ll_ref, rel=TOL)
    assert np.max(np.abs(lf_gpu.cpu().numpy() - lf_ref)) < TOL
    ref = orc.estep(c["y"], c["params"], c["u"])
    new_ref = orc.mstep(ref["stats"], 300, c["params"])
    new_gpu = native.cfust_mstep(T(ref["stats"], dev), 300, gpu_params(c["params"], dev))
    err = parity.params_rel_err({k: v.cpu().numpy() for k, v in new_gpu.items()}, new_ref)
    assert max(err.values()) < 1e-12, err
    for mode, kw in [("fixed", dict(nu_mode=orc.NU_FIXED)), ("d0", dict(fix_delta_zero=True))]:
        r = orc.mstep(ref["stats"], 300, c["params"], **kw)
        gkw = dict(nu_mode="fixed") if mode == "fixed" else dict(fix_delta_zero=True)
        gg = native.cfust_mstep(T(ref["stats"], dev), 300, gpu_params(c["params"], dev), **gkw)
        err = parity.params_rel_err({k: v.cpu().numpy() for k, v in gg.items()}, r)
        assert max(err.values()) < 1e-12, (mode, err)


def test_em_fit_config1(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.config(1)
    ref = orc.em_fit(c["y"], c["init"], c["u"], max_iter=10, tol=0.0)
    print("[gpu] em_fit config 1", flush=True)
    fit = native.cfust_em_fit(T(c["y"], dev), gpu_params(c["init"], dev), T(c["u"], dev),
                              max_iter=10, tol=0.0)
    assert fit["n_iter"] == ref["n_iter"] == 10
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=TOL)
    err = parity.params_rel_err({k: fit[k].cpu().numpy() for k in ("pi", "mu", "Sigma", "Delta", "nu")}, ref)
    assert max(err.values()) < 1e-9, err
    # same MAP labels (the paper's "same final clustering")
    fr = {k: fit[k].cpu().numpy() for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    a = orc.estep(c["y"], fr, c["u"])["tau"].argmax(1)
    b = orc.estep(c["y"], ref, c["u"])["tau"].argmax(1)
    assert np.array_equal(a, b)


def test_em_fit_stops_like_oracle(dev, orc):
    from paper_2005_06848_amd import inputs, native
    c = inputs.random_case(21, 400, 2, 2, 2, 256)
    ref = orc.em_fit(c["y"], c["params"], c["u"], max_iter=60, tol=1e-3)
    fit = native.cfust_em_fit(T(c["y"], dev), gpu_params(c["params"], dev), T(c["u"], dev),
                              max_iter=60, tol=1e-3)
    assert fit["n_iter"] == ref["n_iter"]
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=1e-9)


def test_delta_zero_fit(dev, orc):
    from paper_2005_06848_amd import inputs, native
    c = inputs.random_case(22, 300, 3, 2, 2, 256)
    par = {k: np.array(v) for k, v in c["params"].items()}
    par["Delta"][:] = 0.0
    ref = orc.em_fit(c["y"], par, c["u"], max_iter=5, tol=0.0, fix_delta_zero=True)
    fit = native.cfust_em_fit(T(c["y"], dev), gpu_params(par, dev), T(c["u"], dev), max_iter=5,
                              tol=0.0, fix_delta_zero=True)
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=1e-12)
    np.testing.assert_allclose(fit["nu"].cpu().numpy(), ref["nu"], rtol=1e-10)


def test_edge_cases(dev, orc):
    from paper_2005_06848_amd import inputs, native
    import torch
    # empty input
    c = inputs.random_case(31, 0, 2, 2, 2, 64)
    g = native.cfust_estep(torch.empty((0, 2), dtype=torch.float64, device=dev),
                           gpu_params(c["params"], dev), T(c["u"], dev))
    assert float(g["loglik"].cpu()[0]) == 0.0
    assert torch.all(g["stats"] == 0)
    # deep tail observation: finite and equal to the oracle
    c = inputs.random_case(15, 5, 2, 2, 2, 256)
    y = c["y"].copy()
    y[0] = c["params"]["mu"][0] - 4000.0 * c["params"]["Delta"][0].sum(1)
    ref = orc.estep(y, c["params"], c["u"])
    gpu = run_pair(dev, y, c["params"], c["u"])
    assert np.all(np.isfinite(gpu["logf"])) and np.all(np.isfinite(gpu["tau"]))
    err = __import__("parity").estep_errors(gpu, ref, 2, 2)
    print("deep tail", err, flush=True)
    check(err)
    # the far observation's own pairs (tau 1 - 5e-8 and 5e-8), each
    # quantity by the measure of tests/parity.py: log f absolute, e1
    # relative to max(|e1|, 1), e2..e4 normwise relative
    assert np.max(np.abs(gpu["logf"][0] - ref["logf"][0])) <= TOL
    for i in range(2):
        assert abs(gpu["e1"][0, i] - ref["e1"][0, i]) <= TOL * max(abs(ref["e1"][0, i]), 1.0)
        for k in ("e2", "e3", "e4"):
            a, r = gpu[k][0, i], ref[k][0, i]
            assert np.max(np.abs(a - r)) <= TOL * np.max(np.abs(r)), (k, i, a, r)
    # error paths
    c = inputs.random_case(17, 10, 2, 2, 2, 64)
    bad = {k: np.array(v, copy=True) for k, v in c["params"].items()}
    bad["nu"][1] = -1.0
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep(T(c["y"], dev), gpu_params(bad, dev), T(c["u"], dev))
    assert e.value.code == native.EINVAL
    bad = {k: np.array(v, copy=True) for k, v in c["params"].items()}
    bad["Sigma"][1] = -np.eye(2) * 5
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep(T(c["y"], dev), gpu_params(bad, dev), T(c["u"], dev))
    assert e.value.code == native.ENOTPD and e.value.bad == 1
    y = c["y"].copy()
    y[3, 1] = np.nan
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep(T(y, dev), gpu_params(c["params"], dev), T(c["u"], dev))
    assert e.value.code == native.ENONFINITE
    u = c["u"].copy()
    u[5, 0] = 1.0
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep(T(c["y"], dev), gpu_params(c["params"], dev), T(u, dev))
    assert e.value.code == native.EINVAL
    # a good call after the failures still works
    gpu = run_pair(dev, c["y"], c["params"], c["u"])
    assert np.all(np.isfinite(gpu["tau"]))


def test_deterministic(dev):
    """Ten E-steps of the full config-2 workload (n=20000, p=q=4, g=3,
    N=4096) in the benchmark's launch configuration give bit-identical
    per-pair outputs, partial sums and log-likelihood (fixed-order
    reductions, no atomics in any sum)."""
    from paper_2005_06848_amd import inputs
    c = inputs.config(2)
    first = run_pair(dev, c["y"], c["init"], c["u"])
    for r in range(9):
        again = run_pair(dev, c["y"], c["init"], c["u"])
        for k in ("tau", "logf", "e1", "e2", "e3", "e4", "stats"):
            assert np.array_equal(first[k], again[k]), (r, k)
        assert first["loglik"] == again["loglik"], r


def test_em_fit_resume_is_bitwise(dev):
    """cfust_em_fit for k1 iterations, then again from its output for k2,
    equals one run of k1 + k2 iterations bit for bit (trace and parameters):
    the fit keeps no hidden state between calls."""
    from paper_2005_06848_amd import inputs, native
    c = inputs.config(1)
    keys = ("pi", "mu", "Sigma", "Delta", "nu")
    for graph in (True, False):
        print(f"[gpu] resume test graph={graph}", flush=True)
        full = native.cfust_em_fit(T(c["y"], dev), gpu_params(c["init"], dev), T(c["u"], dev),
                                   max_iter=7, tol=0.0, graph=graph)
        a = native.cfust_em_fit(T(c["y"], dev), gpu_params(c["init"], dev), T(c["u"], dev),
                                max_iter=3, tol=0.0, graph=graph)
        b = native.cfust_em_fit(T(c["y"], dev), {k: a[k].clone() for k in keys}, T(c["u"], dev),
                                max_iter=4, tol=0.0, graph=graph)
        assert full["n_iter"] == 7 and a["n_iter"] == 3 and b["n_iter"] == 4
        np.testing.assert_array_equal(np.asarray(a["trace"]), np.asarray(full["trace"])[:4])
        np.testing.assert_array_equal(np.asarray(b["trace"]), np.asarray(full["trace"])[3:])
        for k in keys:
            np.testing.assert_array_equal(b[k].cpu().numpy(), full[k].cpu().numpy())


def test_setup_error_paths(dev, orc):
    """Every failure of the per-component set-up reports the oracle's code (and
    the failing component): non-finite Sigma, Delta or mu (ENONFINITE); pi off the simplex
    (EINVAL); a non-positive diagonal of Lambda, and an indefinite R with a
    positive diagonal, which fails in R's Cholesky factor (ENOTPD).  The
    last two have an indefinite Sigma with Omega = Sigma + Delta Delta^T
    positive definite.  Each case is set up on the host; the kernels finish
    and report a status.  The E-step and the M-step-free log-likelihood both
    take the set-up, and so does the batched form (one poisoned problem)."""
    from paper_2005_06848_amd import inputs, native

    def put(name, comp, idx, val):
        def edit(par):
            par[name][comp][idx] = val
        return edit

    def lam_diag(par):
        par["Sigma"][1] = np.diag([-0.5, 1.0])
        par["Delta"][1] = np.diag([1.0, 0.0])

    def r_indefinite(par):
        # Lambda = I - Omega^{-1} with Delta = I: [[0.1, -0.3], [-0.3, 0.8]]
        par["Sigma"][1] = np.linalg.inv(np.array([[0.9, 0.3], [0.3, 0.2]])) - np.eye(2)
        par["Delta"][1] = np.eye(2)

    def near_singular_r(eig):
        # Delta = I: Lambda = M (M + I)^{-1} with Sigma = M = V diag(1, eig) V^T
        # (V a 45-degree rotation), so R has eigenvalues near 2 and 4 eig and
        # its second pivot is about 4 eig
        def edit(par):
            v = np.array([[1.0, -1.0], [1.0, 1.0]]) / np.sqrt(2.0)
            par["Sigma"][1] = v @ np.diag([1.0, eig]) @ v.T
            par["Delta"][1] = np.eye(2)
        return edit

    def pi_off(par):
        par["pi"][0] += 1e-6

    c = inputs.random_case(17, 10, 2, 2, 2, 64)
    cases = [("Sigma NaN", put("Sigma", 1, (0, 1), np.nan), native.ENONFINITE, 1),
             ("Delta Inf", put("Delta", 0, (1, 0), np.inf), native.ENONFINITE, 0),
             ("mu NaN", put("mu", 1, 1, np.nan), native.ENONFINITE, 1),
             ("pi off the simplex", pi_off, native.EINVAL, None),
             ("Lambda diagonal", lam_diag, native.ENOTPD, 1),
             ("R indefinite", r_indefinite, native.ENOTPD, 1),
             ("R pivot below 1e-10", near_singular_r(1e-12), native.ENOTPD, 1)]
    for name, edit, code, bad in cases:
        par = {k: np.array(v, copy=True) for k, v in c["params"].items()}
        edit(par)
        with pytest.raises(orc.OracleError) as eo:
            orc.estep(c["y"], par, c["u"])
        assert eo.value.code == code, (name, eo.value.code)
        print(f"[gpu] set-up error path: {name}", flush=True)
        for call in (native.cfust_estep, native.cfust_loglik):
            with pytest.raises(native.CfustError) as e:
                call(T(c["y"], dev), gpu_params(par, dev), T(c["u"], dev))
            assert e.value.code == code, (name, call.__name__, e.value.code)
            # cfust_loglik has no bad-component output
            if bad is not None and call is native.cfust_estep:
                assert e.value.bad == bad, (name, e.value.bad)
    # the batched form: one problem with an indefinite R fails alone
    probs = [inputs.random_case(300 + k, 40, 2, 2, 2, 256) for k in range(3)]
    r_indefinite(probs[1]["params"])
    y = np.concatenate([q["y"] for q in probs])
    P = {k: T(np.concatenate([q["params"][k] for q in probs]), dev)
         for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    print("[gpu] set-up error path: batched", flush=True)
    _, _, _, st = native.cfust_em_fit_batched(T(y, dev), [40, 40, 40], [2, 2, 2], P,
                                              T(probs[0]["u"], dev), max_iter=2, tol=0.0,
                                              precision="fp64")
    assert st[1] == native.ENOTPD and st[0] == 0 and st[2] == 0, st
    # a good call afterwards still works
    gpu = run_pair(dev, c["y"], c["params"], c["u"])
    assert np.all(np.isfinite(gpu["tau"]))


@pytest.mark.parametrize("shape", [(400, 32, 2, 3, 128), (300, 12, 12, 7, 64), (400, 8, 8, 16, 64)])
def test_large_blocks_fallback_paths(dev, orc, shape):
    """Shapes whose component blocks do not fit the set-up's and the M-step's
    48 KB of LDS (52.6/80.2 KB, 50.0/67.2 KB and 51.7/69.6 KB): both kernels
    then build them in device memory with the same phases.  E-step,
    log-likelihood and M-step against the oracle.  The M-step bar is 1e-11:
    with components of 5-60 units of responsibility in up to 32 dimensions,
    the oracle's own M-step moves by up to 1e-13 under 1e-15 relative noise
    in the statistics."""
    from paper_2005_06848_amd import inputs, native
    import parity
    n, p, q, g, N = shape
    c = inputs.random_case(400 + p + q + g, n, p, q, g, N)
    ref = orc.estep(c["y"], c["params"], c["u"])
    gpu = run_pair(dev, c["y"], c["params"], c["u"])
    check(parity.estep_errors(gpu, ref, p, q))
    ll = float(native.cfust_loglik(T(c["y"], dev), gpu_params(c["params"], dev), T(c["u"], dev)).cpu()[0])
    assert ll == pytest.approx(ref["loglik"], rel=TOL)
    print(f"[gpu] mstep p={p} q={q} g={g}", flush=True)
    new_ref = orc.mstep(ref["stats"], n, c["params"])
    new_gpu = native.cfust_mstep(T(ref["stats"], dev), n, gpu_params(c["params"], dev))
    err = parity.params_rel_err({k: v.cpu().numpy() for k, v in new_gpu.items()}, new_ref)
    assert max(err.values()) < 1e-11, err

@pytest.mark.parametrize("shape", [(7, 3, 3, 2, 1000), (40, 4, 4, 3, 4096), (90, 2, 2, 2, 515),
                                   (33, 6, 5, 2, 2048)])
def test_split_waves_parity(dev, orc, shape):
    """FP64 launches with few pairs spread each pair's points over K waves
    (here K = 3, 16, 2 and 16) and combine the partial sums; the E-step, the
    exact-nu E-step and the log-likelihood still match the oracle."""
    from paper_2005_06848_amd import inputs, native
    import parity
    n, p, q, g, N = shape
    c = inputs.random_case(201 + n, n, p, q, g, N)
    y, par, u = c["y"], c["params"], c["u"]
    for mode, omode in (("osl", orc.NU_OSL), ("exact", orc.NU_EXACT)):
        ref = orc.estep(y, par, u, nu_mode=omode)
        print(f"[gpu] split estep n={n} q={q} g={g} N={N} {mode}", flush=True)
        g_ = native.cfust_estep(T(y, dev), gpu_params(par, dev), T(u, dev), nu_mode=mode)
        got = {k: v.cpu().numpy() for k, v in g_.items()}
        got["loglik"] = float(got["loglik"][0])
        err = parity.estep_errors(got, ref, p, q)
        assert max(err.values()) <= TOL, (mode, err)
    ll_ref = orc.loglik(y, par, u)
    ll = float(native.cfust_loglik(T(y, dev), gpu_params(par, dev), T(u, dev)).cpu()[0])
    assert abs(ll - ll_ref) <= TOL * abs(ll_ref)


def test_degenerate_component_guards(dev, orc):
    """Two guards that end a fit on a degenerated component cleanly, as in
    the oracle: (a) a pair whose responsibility underflows to zero is left
    out of the partial sums (its T_B/T_A may overflow), so the E-step stays
    finite and equal to the oracle's; (b) a new Sigma whose Cholesky pivot
    falls to 2^-26 of its diagonal entry gives ENOTPD naming the component
    (relative pivots 0 and about 3e-9), while one above it (about 2.5e-8)
    is accepted."""
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.random_case(31, 30, 2, 2, 2, 128)
    par = {k: np.array(v, copy=True) for k, v in c["params"].items()}
    y = np.array(c["y"], copy=True)
    y[0] = par["mu"][0] + 0.1
    par["mu"][1] = par["mu"][0] + 1e120
    ref = orc.estep(y, par, c["u"])
    assert ref["tau"][0, 1] == 0.0
    got = run_pair(dev, y, par, c["u"])
    assert np.all(np.isfinite(got["stats"]))
    check(parity.estep_errors(got, ref, 2, 2))

    rng = np.random.default_rng(21)
    x = rng.standard_normal(50)
    noise = rng.standard_normal(50)
    c = inputs.random_case(23, 4, 2, 1, 1, 64)
    par = {k: np.array(v, copy=True) for k, v in c["params"].items()}
    par["Delta"][:] = 0.0
    for off, ok in ((0.0, False), (1e-4, False), (3e-4, True)):
        yy = np.stack([x, 2 * x + off * noise], axis=1)
        e = orc.estep(yy, par, c["u"])
        print(f"[gpu] Sigma pivot guard, offset {off}", flush=True)
        if ok:
            r = orc.mstep(e["stats"], 50, par, fix_delta_zero=True)
            gg = native.cfust_mstep(T(e["stats"], dev), 50, gpu_params(par, dev),
                                    fix_delta_zero=True)
            err = parity.params_rel_err({k: v.cpu().numpy() for k, v in gg.items()}, r)
            assert max(err.values()) < 1e-10, err
        else:
            with pytest.raises(native.CfustError) as er:
                native.cfust_mstep(T(e["stats"], dev), 50, gpu_params(par, dev),
                                   fix_delta_zero=True)
            assert er.value.code == native.ENOTPD and er.value.bad == 0
