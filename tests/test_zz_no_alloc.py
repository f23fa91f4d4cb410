"""The allocation-free E-step (cfust_estep_noalloc: the library's static
device scratch array instead of an allocated workspace) against cfust_estep,
both through the C ABI, on two calls in a row, the second with a smaller
input: every output identical (the same kernels in the same order)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

KEYS = ("tau", "logf", "e1", "e2", "e3", "e4", "stats", "loglik")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _T(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _run(fn, y, params, u, dev, **opt):
    out = fn(_T(y, dev), {k: _T(v, dev) for k, v in params.items()}, _T(u, dev), **opt)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


def test_noalloc_estep_equals_estep_twice():
    from paper_2005_06848_amd import inputs, native
    dev = _dev()
    c2, c1 = inputs.config(2), inputs.config(1)
    keys = ("pi", "mu", "Sigma", "Delta", "nu")
    cases = [
        # 12000 pairs (one wave per pair), then a smaller call with another
        # shape whose 600 pairs are split over several waves per pair
        ("workload 2, first 4000 observations", c2["y"][:4000], c2["init"], c2["u"], {}),
        ("workload 1, first 300 observations", c1["y"][:300], c1["init"], c1["u"], {}),
        ("workload 1, first 200 observations, fp32", c1["y"][:200], c1["init"], c1["u"],
         {"precision": "fp32"}),
    ]
    for name, y, par, u, opt in cases:
        par = {k: par[k] for k in keys}
        print(f"[gpu] cfust_estep_noalloc vs cfust_estep: {name} {opt}", flush=True)
        a = _run(native.cfust_estep_noalloc, y, par, u, dev, **opt)
        b = _run(native.cfust_estep, y, par, u, dev, **opt)
        for k in KEYS:
            assert np.all(np.isfinite(a[k])), (name, k)
            assert np.array_equal(a[k], b[k]), (name, k)


def test_noalloc_estep_limits():
    """Sizes beyond the scratch array and options that would allocate are
    rejected before any launch."""
    from paper_2005_06848_amd import inputs, native
    dev = _dev()
    n, p, q, g, N = 200000, 6, 6, 4, 8192
    assert native.workspace_size(n, p, q, g, N) > 64 << 20
    rng = np.random.default_rng(3)
    y = rng.standard_normal((n, p))
    c = inputs.random_case(5, 10, p, q, g, N)
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep_noalloc(_T(y, dev), {k: _T(v, dev) for k, v in c["params"].items()},
                                   _T(c["u"], dev))
    assert e.value.code == 5  # CFUST_ENOMEM
    small = y[:10]
    ws = native.alloc_workspace(10, p, q, g, N, device=dev)
    with pytest.raises(native.CfustError) as e:
        native.cfust_estep_noalloc(_T(small, dev), {k: _T(v, dev) for k, v in c["params"].items()},
                                   _T(c["u"], dev), workspace=ws)
    assert e.value.code == 1  # CFUST_EINVAL
