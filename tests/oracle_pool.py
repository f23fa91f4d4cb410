"""Runs the oracle E-step over chunks of observations in worker processes
(CPU only; no GPU library is imported here)."""
import multiprocessing as mp
import os

import numpy as np


def _chunk(args):
    import oracle
    y, params, u, want = args
    out = oracle.estep(y, params, u, want=want)
    return {k: v for k, v in out.items() if k != "stats"}


def estep_parallel(y, params, u, want=("tau", "logf", "e1", "e2", "e3", "e4"), workers=None):
    """Per-observation oracle outputs (the log-likelihood summed over chunks)."""
    n = y.shape[0]
    workers = workers or min(16, os.cpu_count() or 1)
    chunks = np.array_split(np.arange(n), max(1, min(n, workers * 2)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        parts = pool.map(_chunk, [(y[c], params, u, want) for c in chunks if c.size])
    out = {k: np.concatenate([p[k] for p in parts]) for k in want}
    out["loglik"] = float(sum(p["loglik"] for p in parts))
    return out
