"""Runs the oracle E-step over chunks of observations in worker processes
(CPU only; no GPU library is imported here)."""
import multiprocessing as mp
import os

import numpy as np


def _chunk(args):
    import oracle
    y, params, u, want, kw = args
    return oracle.estep(y, params, u, want=want, **kw)


def estep_parallel(y, params, u, want=("tau", "logf", "e1", "e2", "e3", "e4"), workers=None,
                   **kw):
    """The oracle E-step of all observations: per-observation outputs
    concatenated, the partial sums and the log-likelihood summed over the
    chunks in chunk order (sums over observations, so only their rounding
    order differs from one oracle call)."""
    n = y.shape[0]
    workers = workers or min(16, os.cpu_count() or 1)
    chunks = np.array_split(np.arange(n), max(1, min(n, workers * 2)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        parts = pool.map(_chunk, [(y[c], params, u, want, kw) for c in chunks if c.size])
    out = {k: np.concatenate([p[k] for p in parts]) for k in want}
    out["loglik"] = float(sum(p["loglik"] for p in parts))
    st = parts[0]["stats"].copy()
    for p in parts[1:]:
        st += p["stats"]
    out["stats"] = st
    return out


def _mstep_compose(y, params, u, n_iter, workers, kw):
    """n_iter EM iterations composed from the oracle's E-step (over chunks)
    and M-step: the l trace at the parameters entering each iteration and
    the final parameters."""
    import oracle
    par = {k: np.array(v, dtype=np.float64) for k, v in params.items()
           if k in ("pi", "mu", "Sigma", "Delta", "nu")}
    trace = []
    for _ in range(n_iter):
        e = estep_parallel(y, par, u, want=(), workers=workers, **kw)
        trace.append(e["loglik"])
        par = oracle.mstep(e["stats"], y.shape[0], par)
    trace.append(estep_parallel(y, par, u, want=(), workers=workers, **kw)["loglik"])
    par["trace"] = np.array(trace)
    return par


def em_iterations(y, params, u, n_iter, workers=None, **kw):
    return _mstep_compose(y, params, u, n_iter, workers, kw)
