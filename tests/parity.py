"""Per-quantity error measures for comparing the GPU path with the oracle.

tau and log f: absolute error (log f's absolute error is T's relative error).
e1: |x - ref| / max(|ref|, 1).  e2: relative.  e3, e4: per pair
||x - ref||_inf / ||ref||_inf.  Pair quantities are compared where
tau_ref >= 1e-8 (elsewhere they do not enter the statistics).  Statistics:
normwise per component and per block s1..s8.  Log-likelihood: relative.
"""
import numpy as np


def stat_blocks(p, q):
    o3 = 2
    o4 = o3 + p
    o5 = o4 + q
    o6 = o5 + q * (q + 1) // 2
    o7 = o6 + p * q
    o8 = o7 + p * (p + 1) // 2
    return [(0, 1), (1, 2), (o3, o4), (o4, o5), (o5, o6), (o6, o7), (o7, o8), (o8, o8 + 1)]


def estep_errors(gpu, ref, p, q):
    err = {}
    mask = ref["tau"] >= 1e-8
    err["tau"] = float(np.max(np.abs(gpu["tau"] - ref["tau"]))) if gpu["tau"].size else 0.0
    err["logf"] = float(np.max(np.abs(gpu["logf"] - ref["logf"]))) if gpu["logf"].size else 0.0
    if mask.any():
        err["e1"] = float(np.max((np.abs(gpu["e1"] - ref["e1"]) / np.maximum(np.abs(ref["e1"]), 1.0))[mask]))
        err["e2"] = float(np.max((np.abs(gpu["e2"] - ref["e2"]) / np.abs(ref["e2"]))[mask]))
        d3 = np.max(np.abs(gpu["e3"] - ref["e3"]), axis=-1) / np.max(np.abs(ref["e3"]), axis=-1)
        err["e3"] = float(np.max(d3[mask]))
        d4 = np.max(np.abs(gpu["e4"] - ref["e4"]), axis=(-1, -2)) / np.max(np.abs(ref["e4"]), axis=(-1, -2))
        err["e4"] = float(np.max(d4[mask]))
    st_err = 0.0
    for (a, b) in stat_blocks(p, q):
        for i in range(ref["stats"].shape[0]):
            r = ref["stats"][i, a:b]
            x = gpu["stats"][i, a:b]
            nrm = np.max(np.abs(r))
            if nrm > 0:
                st_err = max(st_err, float(np.max(np.abs(x - r)) / nrm))
    err["stats"] = st_err
    ll = ref["loglik"]
    err["loglik"] = abs(float(gpu["loglik"]) - ll) / max(abs(ll), 1e-300) if ll != 0 else abs(float(gpu["loglik"]))
    return err


def params_rel_err(a, b):
    out = {}
    for k in ("pi", "mu", "Sigma", "Delta", "nu"):
        x = np.asarray(a[k])
        r = np.asarray(b[k])
        nrm = np.max(np.abs(r))
        out[k] = float(np.max(np.abs(x - r)) / nrm) if nrm > 0 else float(np.max(np.abs(x)))
    return out
