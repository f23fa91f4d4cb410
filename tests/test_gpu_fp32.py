"""FP32 form: GHK integrand in float32 (its weight and moment sums in
float64), everything else in float64, against the FP64 oracle.

Bars: 1e-4 on the moments (e2, e3, e4 and the tau-weighted statistics) and
1e-7 relative on the log-likelihood; tau and log f are reported too."""
import functools

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


@functools.lru_cache(maxsize=None)
def cfg3():
    from paper_2005_06848_amd import inputs
    return inputs.config(3)


def run(dev, y, par, u, precision):
    from paper_2005_06848_amd import native
    print(f"[gpu] estep {precision} n={y.shape[0]} q={par['Delta'].shape[2]} N={u.shape[0]}", flush=True)
    g = native.cfust_estep(T(y, dev), {k: T(v, dev) for k, v in par.items()}, T(u, dev),
                           precision=precision)
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["loglik"] = float(out["loglik"][0])
    return out


def fp32_errors(gpu, ref):
    mask = ref["tau"] >= 1e-8
    e = {}
    e["tau_abs"] = float(np.max(np.abs(gpu["tau"] - ref["tau"])))
    e["logf_abs"] = float(np.max(np.abs(gpu["logf"] - ref["logf"])))
    e["e2"] = float(np.max((np.abs(gpu["e2"] - ref["e2"]) / np.abs(ref["e2"]))[mask]))
    d3 = np.max(np.abs(gpu["e3"] - ref["e3"]), -1) / np.max(np.abs(ref["e3"]), -1)
    e["e3"] = float(np.max(d3[mask]))
    d4 = np.max(np.abs(gpu["e4"] - ref["e4"]), (-1, -2)) / np.max(np.abs(ref["e4"]), (-1, -2))
    e["e4"] = float(np.max(d4[mask]))
    e["loglik_rel"] = abs(gpu["loglik"] - ref["loglik"]) / abs(ref["loglik"])
    return e


def test_fp32_config3_subsample(dev):
    """Config 3 (p=q=6, g=4, N=8192) on its seeded 2000-observation subsample."""
    import oracle_pool
    c = cfg3()
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(c["n"], size=2000, replace=False))
    y = c["y"][idx]
    g32 = run(dev, y, c["init"], c["u"], "fp32")
    ref = oracle_pool.estep_parallel(y, c["init"], c["u"])
    err = fp32_errors(g32, ref)
    print("fp32 vs oracle:", err, flush=True)
    assert err["e2"] < 1e-4 and err["e3"] < 1e-4 and err["e4"] < 1e-4, err
    assert err["loglik_rel"] < 1e-7, err
    # every partial sum s1..s8, normwise per component and block, against
    # the oracle's (summed over the same observations)
    import parity
    full = parity.estep_errors(g32, ref, c["p"], c["q"])
    print("fp32 statistics vs oracle:", full["stats"], "e1:", full["e1"], flush=True)
    assert full["stats"] < 1e-4, full
    assert full["e1"] < 1e-4, full


def test_fp32_full_config3_stats_vs_fp64(dev):
    """Full config 3 (n=200000): FP32 statistics and log-likelihood against the
    FP64 GPU path (itself oracle-matched to 1e-10)."""
    c = cfg3()
    g32 = run(dev, c["y"], c["init"], c["u"], "fp32")
    g64 = run(dev, c["y"], c["init"], c["u"], "fp64")
    assert abs(g32["loglik"] / g64["loglik"] - 1) < 1e-7
    st32, st64 = g32["stats"], g64["stats"]
    for i in range(st64.shape[0]):
        rel = np.max(np.abs(st32[i] - st64[i])) / np.max(np.abs(st64[i]))
        assert rel < 1e-4, (i, rel)


def test_fp32_small_shapes(dev, orc):
    """Launches of fewer than 4096 pairs: each pair's points are spread over
    K = 2, 4 and 2 waves and the partial sums combined; with N < 512 (the
    last two shapes) each pair keeps one wave, which at q = 5 is the
    four-wave kernel."""
    from paper_2005_06848_amd import inputs
    for shape in [(50, 2, 2, 2, 512), (40, 4, 4, 3, 1024), (30, 5, 5, 2, 700),
                  (40, 5, 5, 3, 256), (40, 6, 6, 2, 300)]:
        n, p, q, g, N = shape
        cc = inputs.random_case(500 + n, n, p, q, g, N)
        g32 = run(dev, cc["y"], cc["params"], cc["u"], "fp32")
        ref = orc.estep(cc["y"], cc["params"], cc["u"])
        err = fp32_errors(g32, ref)
        assert err["e2"] < 1e-4 and err["e3"] < 1e-4 and err["e4"] < 1e-4, (shape, err)
        assert err["loglik_rel"] < 1e-7, (shape, err)
