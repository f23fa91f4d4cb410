"""Batched form: many independent EM problems in one device-driven loop,
iterations captured in a hipGraph.  Checked against the oracle per problem,
against the single-problem GPU fit, graph against eager launches, and with
one poisoned problem."""
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


def small_batch(n_problems, seed, p=3, q=2, n_lo=60, n_hi=160, N=256):
    from paper_2005_06848_amd import inputs
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(n_problems):
        g = int(rng.integers(2, 5))
        n = int(rng.integers(n_lo, n_hi))
        c = inputs.random_case(seed * 100 + k, n, p, q, g, N)
        probs.append(c)
    u = probs[0]["u"]
    return probs, u


def concat(probs):
    y = np.concatenate([c["y"] for c in probs])
    par = {k: np.concatenate([c["params"][k] for c in probs]) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    return y, par, [c["n"] for c in probs], [c["g"] for c in probs]


def split(par, g):
    out, c0 = [], 0
    for gk in g:
        out.append({k: np.asarray(v)[c0:c0 + gk] for k, v in par.items()})
        c0 += gk
    return out


def test_batched_matches_oracle_fp64(dev, orc):
    from paper_2005_06848_amd import native
    probs, u = small_batch(5, 1)
    y, par, n, g = concat(probs)
    print("[gpu] batched fp64 5 problems", flush=True)
    fit, trace, n_iter, status = native.cfust_em_fit_batched(
        T(y, dev), n, g, {k: T(v, dev) for k, v in par.items()}, T(u, dev), max_iter=6, tol=0.0,
        precision="fp64")
    assert np.all(status == 0)
    fitted = split({k: v.cpu().numpy() for k, v in fit.items() if k in par}, g)
    for k, c in enumerate(probs):
        ref = orc.em_fit(c["y"], c["params"], u, max_iter=6, tol=0.0)
        assert n_iter[k] == ref["n_iter"] == 6
        np.testing.assert_allclose(trace[k, :7], ref["trace"], rtol=1e-10)
        for key in ("pi", "mu", "Sigma", "Delta", "nu"):
            r = ref[key]
            assert np.max(np.abs(fitted[k][key] - r)) <= 1e-8 * max(np.max(np.abs(r)), 1e-300), (k, key)



def test_batched_large_blocks_fp64(dev, orc):
    """p = q = 8: the batched set-up and M-step size their LDS for 16
    components (51.7 and 69.6 KB), more than 48 KB, so both build the blocks
    in device memory; 4 EM iterations of 3 problems against the oracle."""
    from paper_2005_06848_amd import native
    probs, u = small_batch(3, 4, p=8, q=8, n_lo=250, n_hi=400, N=128)
    y, par, n, g = concat(probs)
    print("[gpu] batched fp64 p=q=8", flush=True)
    fit, trace, n_iter, status = native.cfust_em_fit_batched(
        T(y, dev), n, g, {k: T(v, dev) for k, v in par.items()}, T(u, dev), max_iter=4, tol=0.0,
        precision="fp64")
    assert np.all(status == 0), status
    fitted = split({k: v.cpu().numpy() for k, v in fit.items() if k in par}, g)
    for k, c in enumerate(probs):
        ref = orc.em_fit(c["y"], c["params"], u, max_iter=4, tol=0.0)
        np.testing.assert_allclose(trace[k, :5], ref["trace"], rtol=1e-10)
        for key in ("pi", "mu", "Sigma", "Delta", "nu"):
            r = ref[key]
            assert np.max(np.abs(fitted[k][key] - r)) <= 1e-8 * max(np.max(np.abs(r)), 1e-300), (k, key)


def test_batched_fp32_q5_matches_oracle(dev, orc):
    """The FP32 persistent pair kernel at q = 5 (four waves per SIMD, the
    64-start workload's shape): 3 problems, 2 EM iterations, against the
    FP64 oracle at the FP32 form's bars (l at Psi^(0) to 1e-7, the later
    trace to 1e-6 after M-steps on FP32 moments, parameters to 1e-4)."""
    from paper_2005_06848_amd import native
    probs, u = small_batch(3, 11, p=5, q=5, n_lo=200, n_hi=300, N=1024)
    y, par, n, g = concat(probs)
    refs = [orc.em_fit(c["y"], c["params"], u, max_iter=2, tol=0.0) for c in probs]
    # the autotuned shape, and one wave per pair pinned (the persistent
    # kernel with its values parked in LDS across integral B)
    for tile in (0, _tile(native, 1)):
        print(f"[gpu] batched fp32 q=5 3 problems tile={tile}", flush=True)
        fit, trace, n_iter, status = native.cfust_em_fit_batched(
            T(y, dev), n, g, {k: T(v, dev) for k, v in par.items()}, T(u, dev), max_iter=2,
            tol=0.0, precision="fp32", tile=tile)
        assert np.all(status == 0), status
        fitted = split({k: v.cpu().numpy() for k, v in fit.items() if k in par}, g)
        for k, ref in enumerate(refs):
            assert abs(trace[k, 0] / ref["trace"][0] - 1) <= 1e-7, (k, trace[k, 0], ref["trace"][0])
            np.testing.assert_allclose(trace[k, :3], ref["trace"], rtol=1e-6)
            for key in ("pi", "mu", "Sigma", "Delta", "nu"):
                r = ref[key]
                assert np.max(np.abs(fitted[k][key] - r)) <= 1e-4 * max(np.max(np.abs(r)), 1e-300), (k, key)

def test_batched_graph_equals_eager_and_single(dev):
    """Graph and eager batched runs agree bit for bit.  At N = 256 a
    single-problem call keeps one wave per pair, as the batched form does,
    so the two sum in the same order; at N = 1024 a single call spreads each
    pair over several waves and agrees to FP32 rounding."""
    from paper_2005_06848_amd import native
    probs, u = small_batch(7, 2, n_lo=200, n_hi=700, N=256)
    y, par, n, g = concat(probs)
    P = {k: T(v, dev) for k, v in par.items()}
    print("[gpu] batched fp32 graph vs eager", flush=True)
    fg, tg, ng, sg = native.cfust_em_fit_batched(T(y, dev), n, g, P, T(u, dev), max_iter=12,
                                                  tol=1e-6, precision="fp32", graph=True)
    fe, te, ne, se = native.cfust_em_fit_batched(T(y, dev), n, g, P, T(u, dev), max_iter=12,
                                                  tol=1e-6, precision="fp32", graph=False)
    assert np.all(sg == 0) and np.all(se == 0)
    np.testing.assert_array_equal(ng, ne)
    np.testing.assert_array_equal(np.nan_to_num(tg, nan=7.0), np.nan_to_num(te, nan=7.0))
    for key in ("pi", "mu", "Sigma", "Delta", "nu"):
        np.testing.assert_array_equal(fg[key].cpu().numpy(), fe[key].cpu().numpy())
    # the same problems one by one through the single-problem entry point
    for k, c in enumerate(probs):
        single = native.cfust_em_fit(T(c["y"], dev), {kk: T(v, dev) for kk, v in c["params"].items()},
                                     T(u, dev), max_iter=12, tol=1e-6, precision="fp32")
        assert single["n_iter"] == ng[k]
        np.testing.assert_allclose(tg[k, :ng[k] + 1], single["trace"], rtol=1e-12)
    probs, u = small_batch(4, 5, n_lo=200, n_hi=700, N=1024)
    y, par, n, g = concat(probs)
    P = {k: T(v, dev) for k, v in par.items()}
    print("[gpu] batched fp32 vs split single calls", flush=True)
    fb, tb, nb_, sb = native.cfust_em_fit_batched(T(y, dev), n, g, P, T(u, dev), max_iter=6,
                                                  tol=0.0, precision="fp32")
    assert np.all(sb == 0) and np.all(nb_ == 6)
    for k, c in enumerate(probs):
        single = native.cfust_em_fit(T(c["y"], dev), {kk: T(v, dev) for kk, v in c["params"].items()},
                                     T(u, dev), max_iter=6, tol=0.0, precision="fp32")
        np.testing.assert_allclose(tb[k, :7], single["trace"], rtol=1e-6)
    cfg = native.cfust_batched_config()
    assert cfg["n_candidates"] >= 4 and cfg["waves_per_block"] in (1, 2, 4)


def test_batched_poisoned_problem(dev):
    from paper_2005_06848_amd import native
    probs, u = small_batch(6, 3)
    y, par, n, g = concat(probs)
    bad = [dict(c) for c in probs]
    yb = bad[2]["y"].copy()
    yb[5, 0] = np.nan
    bad[2] = dict(bad[2], y=yb)
    y2, par2, _, _ = concat(bad)
    P = {k: T(v, dev) for k, v in par.items()}
    f_ok, t_ok, n_ok, s_ok = native.cfust_em_fit_batched(T(y, dev), n, g, P, T(u, dev), max_iter=5,
                                                          tol=0.0, precision="fp64")
    f_bad, t_bad, n_bad, s_bad = native.cfust_em_fit_batched(T(y2, dev), n, g, P, T(u, dev),
                                                              max_iter=5, tol=0.0, precision="fp64")
    assert s_bad[2] == native.ENONFINITE
    keep = [k for k in range(6) if k != 2]
    assert np.all(s_bad[keep] == 0)
    np.testing.assert_array_equal(t_bad[keep], t_ok[keep])
    fo = split({k: v.cpu().numpy() for k, v in f_ok.items() if k in par}, g)
    fb = split({k: v.cpu().numpy() for k, v in f_bad.items() if k in par}, g)
    for k in keep:
        for key in ("pi", "mu", "Sigma", "Delta", "nu"):
            np.testing.assert_array_equal(fb[k][key], fo[k][key])


def test_batched_workload4_shape(dev):
    """A reduced copy of the 64-start workload (n 500-2000, g 2-6, p=q=5,
    N=1024) runs to completion with per-start stopping."""
    from paper_2005_06848_amd import inputs, native
    probs = inputs.batched_problems(16, 500, 2000)
    u = inputs.qmc_points(1024, 5)
    y = np.concatenate([c["y"] for c in probs])
    par = {k: np.concatenate([c["init"][k] for c in probs]) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    n = [c["n"] for c in probs]
    g = [c["g"] for c in probs]
    f, tr, it, st = native.cfust_em_fit_batched(T(y, dev), n, g, {k: T(v, dev) for k, v in par.items()},
                                                T(u, dev), max_iter=20, tol=1e-6, precision="fp32")
    assert np.all(st == 0), st
    assert np.all(it >= 2)
    for k in range(16):
        tk = tr[k, :it[k] + 1]
        assert np.all(np.isfinite(tk))
        assert tk[-1] > tk[0]


def test_multistart_algorithm1_matches_oracle(dev):
    """Algorithm 1 on the GPU (starts evaluated together by the batched
    kernels, burn-in of 2 EM iterations, the largest l kept, then the fit)
    against the same composition in the oracle: per-start l, the selected
    start, the trace and the parameters."""
    import oracle as orc
    from paper_2005_06848_amd import inputs, native
    import parity
    c = inputs.config(1)
    starts = inputs.multistart_inits(c["y"], c["g"], c["q"], 4, seed=11)
    ref = orc.em_fit_multistart(c["y"], starts, c["u"], burn_in=2, max_iter=8, tol=0.0)
    print("[gpu] multistart config 1, 4 starts", flush=True)
    T_ = lambda a: T(a, dev)
    fit = native.cfust_em_fit_multistart(T_(c["y"]), [{k: T_(v) for k, v in s.items()} for s in starts],
                                         T_(c["u"]), burn_in=2, max_iter=8, tol=0.0)
    print("  start l:", fit["start_loglik"], "best", fit["best"], ref["best"])
    np.testing.assert_allclose(fit["start_loglik"], ref["start_loglik"], rtol=1e-10)
    assert fit["best"] == ref["best"]
    np.testing.assert_allclose(fit["trace"], ref["trace"], rtol=1e-9)
    err = parity.params_rel_err({k: fit[k].cpu().numpy() for k in ("pi", "mu", "Sigma", "Delta", "nu")}, ref)
    assert max(err.values()) < 1e-9, err


@pytest.mark.timeout(600)
def test_batched_workload4_two_full_size_starts_vs_oracle(dev):
    """Two full-size starts of the 64-start workload (the two with the
    fewest pairs: n = 10022, g = 2 and n = 8527, g = 3; p = q = 5, N = 4096)
    in one batched FP64 launch sequence, 2 EM iterations, against the same
    iterations composed from the oracle's E-step (over all observations) and
    M-step: the l trace and the parameters.  The paper's criterion for the
    parallel runs is estimates almost identical to the serial ones with the
    same final clustering; the MAP labels are compared too."""
    from paper_2005_06848_amd import inputs, native
    import oracle_pool
    import parity
    probs = inputs.batched_problems(64)
    pick = sorted(range(64), key=lambda k: probs[k]["n"] * probs[k]["g"])[:2]
    sel = [probs[k] for k in pick]
    u = inputs.qmc_points(4096, 5)
    y = np.concatenate([c["y"] for c in sel])
    par = {k: np.concatenate([c["init"][k] for c in sel]) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    n = [c["n"] for c in sel]
    g = [c["g"] for c in sel]
    print(f"[gpu] batched fp64, workload 4 starts {pick}: n={n} g={g}", flush=True)
    fit, trace, n_iter, status = native.cfust_em_fit_batched(
        T(y, dev), n, g, {k: T(v, dev) for k, v in par.items()}, T(u, dev), max_iter=2, tol=0.0,
        precision="fp64")
    assert np.all(status == 0), status
    fitted = split({k: v.cpu().numpy() for k, v in fit.items() if k in par}, g)
    for k, c in enumerate(sel):
        print(f"[cpu] oracle, start {pick[k]}: 2 EM iterations over all {c['n']} observations",
              flush=True)
        ref = oracle_pool.em_iterations(c["y"], c["init"], u, 2)
        assert n_iter[k] == 2
        np.testing.assert_allclose(trace[k, :3], ref["trace"], rtol=1e-10)
        err = parity.params_rel_err(fitted[k], ref)
        assert max(err.values()) < 1e-9, (k, err)
        # MAP labels at the two fitted parameter sets (E-steps on the GPU)
        lab = [native.cfust_estep(T(c["y"], dev), {kk: T(pp[kk], dev) for kk in par}, T(u, dev),
                                  want=("tau",))["tau"].cpu().numpy().argmax(1)
               for pp in (fitted[k], ref)]
        assert np.array_equal(lab[0], lab[1])


def _tile(native, K, wpb=1, chunk=1, wps=4):
    """opts.tile of the candidate shape with these fields."""
    k = 0
    while True:
        s = native.cfust_batched_shape(k)
        assert s is not None, (K, wpb, chunk, wps)
        if (s["waves_per_pair"], s["waves_per_block"], s["chunk"], s["waves_per_simd"]) == \
                (K, wpb, chunk, wps):
            return k + 1
        k += 1


def test_batched_split_pairs_match_oracle(dev, orc):
    """Several waves per pair in the batched form (each of a pair's K waves
    integrates N / K of its points; bpart_kernel + bfinish_kernel): K = 1,
    2, 4, 8 pinned through opts.tile, FP64, 3 EM iterations of 3 problems,
    each against the oracle at the FP64 bar, and the split runs against
    K = 1 to summation-order rounding.  The exact nu step at K = 4, FP32 at
    K = 4 against FP32 at K = 1, graph against eager, and a poisoned
    problem at K = 4."""
    from paper_2005_06848_amd import native
    import parity
    probs, u = small_batch(3, 23, p=4, q=3, n_lo=80, n_hi=140, N=2048)
    y, par, n, g = concat(probs)
    keys = ("pi", "mu", "Sigma", "Delta", "nu")
    off = np.concatenate([[0], np.cumsum(g)])
    yd, ud = T(y, dev), T(u, dev)
    P = lambda: {k: T(v, dev) for k, v in par.items()}
    refs = [orc.em_fit(c["y"], c["params"], u, max_iter=3, tol=0.0) for c in probs]
    runs = {}
    for K in (1, 2, 4, 8):
        print(f"[gpu] batched split K={K} fp64", flush=True)
        fit, trace, n_iter, status = native.cfust_em_fit_batched(
            yd, n, g, P(), ud, max_iter=3, tol=0.0, precision="fp64", tile=_tile(native, K))
        assert np.all(status == 0), (K, status)
        cfg = native.cfust_batched_config()
        assert cfg["waves_per_pair"] == K and cfg["points_per_wave"] == 2048 // K
        for k in range(3):
            np.testing.assert_allclose(trace[k, :4], refs[k]["trace"], rtol=1e-10)
            got = {kk: fit[kk].cpu().numpy()[off[k]:off[k + 1]] for kk in keys}
            err = parity.params_rel_err(got, refs[k])
            assert max(err.values()) < 1e-9, (K, k, err)
        runs[K] = (fit, trace)
    for K in (2, 4, 8):
        np.testing.assert_allclose(runs[K][1], runs[1][1], rtol=1e-12)
    print("[gpu] batched split K=4 exact nu", flush=True)
    fit, trace, n_iter, status = native.cfust_em_fit_batched(
        yd, n, g, P(), ud, max_iter=2, tol=0.0, nu_mode="exact", tile=_tile(native, 4))
    assert np.all(status == 0), status
    for k, c in enumerate(probs[:2]):
        ref = orc.em_fit(c["y"], c["params"], u, max_iter=2, tol=0.0, nu_mode=orc.NU_EXACT)
        np.testing.assert_allclose(trace[k, :3], ref["trace"], rtol=1e-10)
        got = {kk: fit[kk].cpu().numpy()[off[k]:off[k + 1]] for kk in keys}
        assert max(parity.params_rel_err(got, ref).values()) < 1e-9, k
    print("[gpu] batched split K=4 fp32 vs K=1, graph vs eager", flush=True)
    f1, t1, _, s1 = native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=3, tol=0.0,
                                                precision="fp32", tile=_tile(native, 1))
    f4, t4, _, s4 = native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=3, tol=0.0,
                                                precision="fp32", tile=_tile(native, 4))
    f4e, t4e, _, s4e = native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=3, tol=0.0,
                                                   precision="fp32", tile=_tile(native, 4),
                                                   graph=False)
    assert np.all(s1 == 0) and np.all(s4 == 0) and np.all(s4e == 0)
    np.testing.assert_allclose(t4, t1, rtol=1e-6)
    np.testing.assert_array_equal(t4, t4e)
    for key in keys:
        np.testing.assert_array_equal(f4[key].cpu().numpy(), f4e[key].cpu().numpy())
    print("[gpu] batched split K=4 poisoned problem", flush=True)
    yb = y.copy()
    yb[n[0] + 3, 1] = np.nan  # an observation of problem 1
    fb, tb, _, sb = native.cfust_em_fit_batched(T(yb, dev), n, g, P(), ud, max_iter=3, tol=0.0,
                                                precision="fp64", tile=_tile(native, 4))
    assert sb[1] == native.ENONFINITE and sb[0] == 0 and sb[2] == 0, sb
    np.testing.assert_array_equal(tb[[0, 2]], runs[4][1][[0, 2]])


def test_batched_split_limits_and_autotune(dev):
    """A shape with more waves per pair than the batch allows is rejected
    (N = 512 allows K <= 2), and the autotuner's choice for a small batch
    reports K and N / K points per wave; its result equals the same shape
    pinned through opts.tile, bit for bit."""
    from paper_2005_06848_amd import native
    probs, u = small_batch(3, 29, p=4, q=3, n_lo=80, n_hi=140, N=512)
    y, par, n, g = concat(probs)
    yd, ud = T(y, dev), T(u, dev)
    P = lambda: {k: T(v, dev) for k, v in par.items()}
    with pytest.raises(native.CfustError):
        native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=1, tol=0.0, tile=_tile(native, 4))
    print("[gpu] batched autotune, small batch", flush=True)
    fa, ta, _, sa = native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=2, tol=0.0)
    cfg = native.cfust_batched_config()
    assert np.all(sa == 0)
    assert cfg["waves_per_pair"] in (1, 2) and cfg["points_per_wave"] == 512 // cfg["waves_per_pair"]
    assert cfg["tuned_ms"] > 0
    tile = _tile(native, cfg["waves_per_pair"], cfg["waves_per_block"], cfg["chunk"],
                 cfg["waves_per_simd"])
    fp, tp, _, sp = native.cfust_em_fit_batched(yd, n, g, P(), ud, max_iter=2, tol=0.0, tile=tile)
    np.testing.assert_array_equal(ta, tp)
