"""Benchmark: CFUST mixture EM iterations on one MI355X.

One step = one EM iteration of the whole hot path on the n=20000, p=q=4,
g=3, N=4096 workload (FP64): per-component precompute and chi-square tables,
the fused pair kernel (Mahalanobis distance, both GHK integrals, the
conditional expectations), responsibilities, log-likelihood, the eight
partial sums, and the M-step.  The metric is E-step (observation x component)
evaluations per second.

Prints one JSON line.  `--gpus N` with N > 1 exits: the library runs on one
GPU (the path would shard by observations with one all-reduce of the partial
sums per iteration).  The CPU baseline is the FP64 oracle on the host's
cores, one thread per block of observations, with the single-thread rate
beside it.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "cfust-em n=20000 p=4 q=4 g=3 N=4096 fp64"
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_FP32_VALU_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

# Algorithmic flop model of one (observation, component) pair (both GHK
# integrals over N points plus the pair set-up):
#   F_A = q^2 + q + q*c_phi + (q-1)*c_phiinv + c_acc
#   F_B = q^2 + q + q*c_phi + q*c_phiinv + q(q+1) + 4q + c_acc
#   F_pair = N (F_A + F_B) + 2p^2 + 2pq + 40
# with c_phi, c_phiinv the VALU flops per call of the implementation's normal
# CDF and quantile, measured with rocprofv3 on the diagnostic kernels
# (`python bench.py --cost-probe` under rocprofv3 --pmc with the
# SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 / _F32 counters: 64 lanes per
# instruction, an FMA counting 2), and c_acc the flops of the per-point
# accumulation (the exponent-aligned add of the weight: no exp is taken).
# NOMINAL are the fixed costs of the first version of the model (Phi 40,
# Phi^-1 50, an exp-scaled accumulation 20), reported beside it.
NOMINAL_COSTS = {"phi": 40, "phiinv": 50, "acc": 20}
# measured per precision; "sources" is the digest of the kernel sources they
# were measured on (the model falls back to NOMINAL when it differs).
# FP64: Phi 99 (45 FMA, 5 MUL, 3 ADD, 1 TRANS), coordinate step 191, so
# Phi^-1 191 - 99 - 1 = 91, accumulation 5 (4 ADD, 1 MUL).  FP32: Phi 41,
# step 72, Phi^-1 30, accumulation 2 (its FP64 add and scale).
MEASURED_COSTS = {"sources": "3dd56fa4769c78c8",
                  "fp64": {"phi": 99, "phiinv": 91, "acc": 5},
                  "fp32": {"phi": 41, "phiinv": 30, "acc": 2}}

# HBM bytes per launch of the FP64 pair kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, each scaled by what the counter reads for a
# plain elementwise copy of known size), with the digest of the kernel
# sources they were taken on: `traffic` is null once the sources differ.
# FETCH_SIZE 3362.33 KiB x 1.99976 + WRITE_SIZE 7968.75 KiB x 0.99999 (the
# copy probe, 262144 KiB each way, read 131087.88 and 262145.62): the writes
# are the pair records alone, the reads y, the tables once per XCD and the
# component blocks.
PAIR_KERNEL_COUNTERS = {"sources": "3dd56fa4769c78c8", "traffic": 15045174}


# the sources the pair kernels, their launches and the diagnostic
# special-function kernel are compiled from
PAIR_KERNEL_SOURCES = ("cfust_coeffs.hpp", "cfust_host.hpp", "cfust_kernels.hpp",
                       "cfust_math.hpp", "cfust_pairs.hip")


def kernel_sources_digest():
    """sha256 (first 16 hex digits) of the HIP sources of the pair kernels."""
    d = os.path.join(ROOT, "paper_2005_06848_amd", "csrc")
    h = hashlib.sha256()
    for f in PAIR_KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def flops_per_pair(p, q, N, costs=None):
    c = costs or NOMINAL_COSTS
    fa = q * q + q + q * c["phi"] + (q - 1) * c["phiinv"] + c["acc"]
    fb = q * q + q + q * c["phi"] + q * c["phiinv"] + q * (q + 1) + 4 * q + c["acc"]
    return N * (fa + fb) + 2 * p * p + 2 * p * q + 40


def cost_probe(native, torch, dev):
    """Diagnostic kernels for the per-call cost model, 2^24 evaluations each,
    one dispatch each in this order: the normal CDF (inputs uniform in
    [-6, 6]) and quantile (probabilities uniform in (0, 1)) in FP64, the
    same two in FP32, then the GHK coordinate step Phi^-1(u Phi(x)) in FP64
    and FP32, and the accumulation of a point's weight in FP64 and FP32.
    c_phi is the CDF's count; c_phiinv is the coordinate step's count less
    the CDF's and less the probe's own 1 - u; c_acc is the accumulation's
    count."""
    n = 1 << 24
    g = torch.Generator(device="cpu").manual_seed(5)
    x = (torch.rand(n, generator=g, dtype=torch.float64) * 12.0 - 6.0).to(dev)
    pr = ((torch.arange(n, dtype=torch.float64) + 0.5) / n).to(dev)
    m = (0.5 + 0.5 * torch.rand(n, generator=g, dtype=torch.float64)).to(dev)
    ex = torch.randint(-20, 21, (n,), generator=g).to(torch.float64).to(dev)
    for fn, arg, arg2 in ((0, x, None), (2, pr, None), (7, x, None), (8, pr, None),
                          (14, x, pr), (15, x, pr), (16, m, ex), (17, m, ex)):
        native.cfust_eval_special(fn, arg, arg2)
        torch.cuda.synchronize()
    print(json.dumps({"cost_probe": "dispatches: Phi f64, Phi^-1 f64, Phi f32, Phi^-1 f32, "
                                    "step f64, step f32, acc f64, acc f32",
                      "evaluations_per_dispatch": n}), flush=True)


def host_description():
    """CPU model and core counts of the host (for the CPU baseline)."""
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def precision_form(args, native, L, torch, np, inputs, dev):
    """FP32 integrand vs FP64 on the precision-form workload: one E-step each
    (precompute, chi tables, pair kernel, partial sums), same inputs."""
    c = inputs.config(3)
    n, p, q, g, N = c["n"], c["p"], c["q"], c["g"], c["n_qmc"]
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y, u = T(c["y"]), T(c["u"])
    par = {k: T(v) for k, v in c["init"].items()}
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    S = native.stats_size(p, q)
    res = {}
    for prec in ("fp64", "fp32"):
        stats = torch.empty((g, S), dtype=torch.float64, device=dev)
        ll = torch.empty(1, dtype=torch.float64, device=dev)
        ws = native.alloc_workspace(n, p, q, g, N, prec)
        prof = native.prof_buffer()
        opts = native.make_opts(precision=prec, workspace=ws, prof=prof)
        out = native.EstepOut(None, None, None, None, None, None, P(stats), P(ll), -1)
        pp = [P(par[k]) for k in ("pi", "mu", "Sigma", "Delta", "nu")]

        def estep():
            rc = L.cfust_estep(P(y), n, p, q, g, pp[0], pp[1], pp[2], pp[3], pp[4], P(u), N,
                               ctypes.byref(opts), ctypes.byref(out))
            if rc:
                raise native.CfustError(rc, "cfust_estep", out.bad_component)

        print(f"[bench] form {prec}: n={n} p={p} q={q} g={g} N={N}", file=sys.stderr, flush=True)
        estep()
        torch.cuda.synchronize()
        for s_ in range(4):
            prof[s_] = 0.0
        t0 = time.perf_counter()
        for _ in range(args.form_reps):
            estep()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.form_reps
        res[prec] = {"ms_per_estep": round(ms, 3), "pairs_per_s": round(n * g / (ms * 1e-3), 1),
                     "pair_kernel_ms": round(prof[1] / args.form_reps, 3),
                     "loglik": float(ll.cpu()[0])}
        del ws
    res["fp32_speedup_vs_fp64"] = round(res["fp64"]["ms_per_estep"] / res["fp32"]["ms_per_estep"], 3)
    res["loglik_rel_diff"] = abs(res["fp32"]["loglik"] / res["fp64"]["loglik"] - 1)
    if not args.no_form_errors:
        res["fp32_errors_vs_fp64_all_pairs"] = fp32_errors(native, torch, y, par, u, c)
    res["workload"] = "cfust E-step n=200000 p=6 q=6 g=4 N=8192"
    res["tolerance"] = "fp32 vs fp64 oracle: moments 1e-4, log-likelihood 1e-7 (tests/test_gpu_fp32.py)"
    return res


def fp32_errors(native, torch, y, par, u, c):
    """Per-quantity errors of the FP32 E-step against the FP64 GPU E-step
    (which matches the FP64 oracle to 1e-10 in the tests) on every pair of
    the precision workload, by the measures of tests/parity.py: tau and
    log f absolute; e1 relative to max(|e1|, 1); e2 relative; e3, e4
    normwise per pair; all over pairs with tau >= 1e-8; the partial sums
    normwise per component; l relative."""
    print("[bench] form errors: fp32 vs fp64 on all pairs", file=sys.stderr, flush=True)
    want = ("tau", "logf", "e1", "e2", "e3", "e4")
    r64 = native.cfust_estep(y, par, u, want=want, precision="fp64")
    r32 = native.cfust_estep(y, par, u, want=want, precision="fp32")
    mask = r64["tau"] >= 1e-8
    ab = lambda k: (r32[k] - r64[k]).abs()
    e = {"tau": ab("tau").max().item(), "logf": ab("logf").max().item(),
         "e1": (ab("e1") / r64["e1"].abs().clamp(min=1.0))[mask].max().item(),
         "e2": (ab("e2") / r64["e2"].abs())[mask].max().item(),
         "e3": (ab("e3").amax(-1) / r64["e3"].abs().amax(-1))[mask].max().item(),
         "e4": (ab("e4").amax((-1, -2)) / r64["e4"].abs().amax((-1, -2)))[mask].max().item(),
         "stats": ((r32["stats"] - r64["stats"]).abs().amax(1)
                   / r64["stats"].abs().amax(1)).max().item(),
         "loglik": abs(r32["loglik"].item() / r64["loglik"].item() - 1)}
    del r64, r32
    return {k: float(f"{v:.3e}") for k, v in e.items()}


def surrogate_form(args, native, torch, np, inputs, dev):
    """Surrogate form on the n=1000000, p=q=6, g=4, N=8192 workload: E-step
    time of the FP64 and FP32 GHK paths, of the shipped network alone, with
    the GHK check over m sampled observations (difference estimator), and
    with one adaptation (GHK labels of 16384 sampled pairs, 20 epochs) first,
    and with both; the accuracy of each against the FP64 GHK E-step on all
    1000000 observations; and the shipped network's fallback, time and
    accuracy at the true parameters.  The k-means start uses one restart
    here."""
    from paper_2005_06848_amd import surrogate as S
    print("[bench] surrogate: generating n=1000000 p=q=6 g=4", file=sys.stderr, flush=True)
    c = inputs.config(5, kmeans_restarts=1)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y, u = T(c["y"]), T(c["u"])
    par = {k: T(v) for k, v in c["init"].items()}
    ptrue = {k: T(v) for k, v in c["true"].items()}
    net = native.Surrogate.load(S.DEFAULT_PATH)
    M_CHECK = 65536

    def timed(f, reps=1):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def totals(r):
        return r["stats"].cpu().numpy(), r["loglik"].item()

    res = {"workload": "cfust E-step n=1000000 p=6 q=6 g=4 N=8192 (k-means start, 1 restart)"}
    print("[bench] surrogate: GHK E-steps (fp64, fp32)", file=sys.stderr, flush=True)
    res["fp64_ghk_ms"] = round(timed(lambda: native.cfust_estep(y, par, u, want=())), 2)
    res["fp32_ghk_ms"] = round(timed(lambda: native.cfust_estep(y, par, u, want=(), precision="fp32")), 2)
    st_ref, ll_ref = totals(native.cfust_estep(y, par, u, want=()))

    def err(r):
        st, ll = totals(r)
        per = np.abs(st - st_ref).max(1) / np.abs(st_ref).max(1)
        return {"stats_max_rel": float(per.max()), "loglik_rel": abs(ll / ll_ref - 1)}

    print("[bench] surrogate: network E-steps", file=sys.stderr, flush=True)
    res["network_ms"] = round(timed(lambda: native.cfust_estep(y, par, u, want=(), surrogate=net),
                                    args.form_reps), 2)
    res["network_fallback_pairs"] = net.fallback_count()
    res["network_checked_ms"] = round(timed(
        lambda: native.cfust_estep(y, par, u, want=(), surrogate=net, surrogate_check=M_CHECK),
        args.form_reps), 2)
    res["check_observations"] = M_CHECK
    res["network_checked_fp32_ms"] = round(timed(
        lambda: native.cfust_estep(y, par, u, want=(), surrogate=net, surrogate_check=M_CHECK,
                                   precision="fp32"), args.form_reps), 2)
    acc = {"shipped": err(native.cfust_estep(y, par, u, want=(), surrogate=net)),
           "shipped_checked": err(native.cfust_estep(y, par, u, want=(), surrogate=net,
                                                     surrogate_check=M_CHECK)),
           "shipped_checked_fp32": err(native.cfust_estep(y, par, u, want=(), surrogate=net,
                                                          surrogate_check=M_CHECK,
                                                          precision="fp32"))}
    res["adapt_plus_network_ms"] = round(timed(
        lambda: (net.adapt(y, par, u, samples=16384, epochs=20),
                 native.cfust_estep(y, par, u, want=(), surrogate=net))), 2)
    acc["adapted"] = err(native.cfust_estep(y, par, u, want=(), surrogate=net))
    acc["adapted_checked"] = err(native.cfust_estep(y, par, u, want=(), surrogate=net,
                                                    surrogate_check=M_CHECK))
    # the E-step that meets both targets after an adaptation: adaptation,
    # then the network with the check (FP64 and FP32 check pairs)
    res["adapt_plus_checked_ms"] = round(timed(
        lambda: (net.adapt(y, par, u, samples=16384, epochs=20),
                 native.cfust_estep(y, par, u, want=(), surrogate=net,
                                    surrogate_check=M_CHECK))), 2)
    res["adapt_plus_checked_fp32_ms"] = round(timed(
        lambda: (net.adapt(y, par, u, samples=16384, epochs=20),
                 native.cfust_estep(y, par, u, want=(), surrogate=net, surrogate_check=M_CHECK,
                                    precision="fp32"))), 2)
    res["accuracy_vs_fp64_ghk_all_observations"] = acc
    # at the true parameters (where EM ends): the shipped network's fallback,
    # time and accuracy, against the FP64 GHK E-step there
    print("[bench] surrogate: at the true parameters", file=sys.stderr, flush=True)
    net = native.Surrogate.load(S.DEFAULT_PATH)
    res["network_ms_at_true_params"] = round(timed(
        lambda: native.cfust_estep(y, ptrue, u, want=(), surrogate=net)), 2)
    res["fallback_pairs_at_true_params"] = net.fallback_count()
    st_ref, ll_ref = totals(native.cfust_estep(y, ptrue, u, want=()))
    res["accuracy_at_true_params"] = {
        "shipped": err(native.cfust_estep(y, ptrue, u, want=(), surrogate=net)),
        "shipped_checked": err(native.cfust_estep(y, ptrue, u, want=(), surrogate=net,
                                                  surrogate_check=M_CHECK))}
    res["pairs"] = c["n"] * c["g"]
    res["speedup_network_vs_fp64"] = round(res["fp64_ghk_ms"] / res["network_ms"], 2)
    res["speedup_network_checked_vs_fp64"] = round(res["fp64_ghk_ms"] / res["network_checked_ms"], 2)
    res["speedup_network_checked_fp32_vs_fp64"] = round(
        res["fp64_ghk_ms"] / res["network_checked_fp32_ms"], 2)
    res["speedup_adapt_plus_network_vs_fp64"] = round(res["fp64_ghk_ms"] / res["adapt_plus_network_ms"], 2)
    res["speedup_adapt_plus_checked_vs_fp64"] = round(
        res["fp64_ghk_ms"] / res["adapt_plus_checked_ms"], 2)
    res["speedup_adapt_plus_checked_fp32_vs_fp64"] = round(
        res["fp64_ghk_ms"] / res["adapt_plus_checked_fp32_ms"], 2)
    res["speedup_fp32_vs_fp64"] = round(res["fp64_ghk_ms"] / res["fp32_ghk_ms"], 2)
    # the fastest configuration that meets both targets at the start values
    ok = lambda e: e["stats_max_rel"] <= 1e-3 and e["loglik_rel"] <= 1e-5
    cands = [("shipped", "network_ms"), ("shipped_checked", "network_checked_ms"),
             ("shipped_checked_fp32", "network_checked_fp32_ms"),
             ("adapted", "adapt_plus_network_ms"), ("adapted_checked", "adapt_plus_checked_ms")]
    met = [(res[t], name) for name, t in cands if ok(acc[name])]
    if met:
        ms, name = min(met)
        res["at_tolerance"] = {"configuration": name, "ms": ms,
                               "speedup_vs_fp64_ghk": round(res["fp64_ghk_ms"] / ms, 2)}
    else:
        res["at_tolerance"] = None
    res["tolerance"] = ("target 1e-3 on moments (partial sums, normwise per component), 1e-5 "
                        "relative on the log-likelihood (tests/test_gpu_surrogate.py)")
    return res


def surrogate_em_form(args, native, torch, np, inputs, dev):
    """Whole fits on the n=1000000, p=q=6, g=4, N=8192 workload from the
    k-means start, FP32 integrand: GHK EM against the two-phase EM with the
    shipped network, adapted before every surrogate E-step (16384 pairs, 10
    epochs) and checked over 50000 observations (5%), switching at a relative
    l change below 3e-7.  Both run in calls of 40 iterations, each printing
    its l, and stop when a call with GHK E-steps stops by Aitken's rule
    (each call restarts the rule).  Reports each fit's l, iterations and
    wall time."""
    from paper_2005_06848_amd import surrogate as S
    c = inputs.config(5, kmeans_restarts=1)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y, u = T(c["y"]), T(c["u"])
    par0 = {k: T(v) for k, v in c["init"].items()}
    keys = ("pi", "mu", "Sigma", "Delta", "nu")
    tol, cap, switch = 25.0, 900, 3e-7
    res = {"workload": "cfust-em n=1000000 p=q=6 g=4 N=8192 (k-means start), fp32 integrand",
           "tol_abs": tol, "max_iter": cap, "surrogate_switch": switch, "check_observations": 50000}
    print("[bench] surrogate EM: GHK EM in chunks of 40", file=sys.stderr, flush=True)
    par, trace = dict(par0), []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while len(trace) < cap + 1:
        f = native.cfust_em_fit(y, par, u, max_iter=40, tol=tol, precision="fp32")
        trace += f["trace"] if not trace else f["trace"][1:]
        par = {k: f[k] for k in keys}
        print(f"[bench]   GHK EM: {len(trace) - 1} iterations, l {trace[-1]:.3f}",
              file=sys.stderr, flush=True)
        if f["n_iter"] < 40:  # stopped by Aitken's rule
            break
    torch.cuda.synchronize()
    res["ghk"] = {"seconds": round(time.perf_counter() - t0, 2), "iterations": len(trace) - 1,
                  "loglik_final": trace[-1]}
    print("[bench] surrogate EM: two-phase fit in chunks of 40", file=sys.stderr, flush=True)
    # chunks of 40 iterations: surrogate chunks until one switches to GHK
    # E-steps, GHK chunks after that (each chunk restarts the stopping rule)
    net = native.Surrogate.load(S.DEFAULT_PATH)
    par, ts, sw, done = dict(par0), [], -1, False
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while not done and len(ts) < cap + 1:
        if sw < 0:
            f = native.cfust_em_fit(y, par, u, max_iter=40, tol=tol, precision="fp32",
                                    surrogate=net, adapt_samples=16384, adapt_epochs=10,
                                    surrogate_check=50000, surrogate_switch=switch)
            s_ = net.em_switch()
            if s_ >= 0:
                sw = len(ts) + s_ - (1 if ts else 0)
        else:
            f = native.cfust_em_fit(y, par, u, max_iter=40, tol=tol, precision="fp32")
        # after the switch a call that ends before its cap stopped by Aitken
        done = sw >= 0 and f["n_iter"] < 40
        ts += f["trace"] if not ts else f["trace"][1:]
        par = {k: f[k] for k in keys}
        print(f"[bench]   two-phase: {len(ts) - 1} iterations, switch {sw}, l {ts[-1]:.3f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    res["two_phase"] = {"seconds": round(time.perf_counter() - t0, 2), "iterations": len(ts) - 1,
                        "switch_iteration": sw, "loglik_final": ts[-1],
                        "surrogate_phase_last_loglik": ts[sw - 1] if sw > 0 else None,
                        "ghk_loglik_at_switch": ts[sw] if sw >= 0 else None}
    res["final_loglik_rel_diff"] = abs(ts[-1] / trace[-1] - 1)
    res["speedup_two_phase_vs_ghk"] = round(res["ghk"]["seconds"] / res["two_phase"]["seconds"], 3)
    return res


def batched_form(args, native, torch, np, inputs, dev):
    """Batched form: 64 EM starts (n ~ U{5000..50000}, g ~ U{2..6}, p=q=5,
    N=4096, FP32 integrand), one device-driven loop with hipGraph-captured
    iterations and autotuned launch shape; compared with fitting the same
    starts one after another through the single-problem entry point."""
    if args.no_batched_large:
        res = {}
        if not args.no_batched_small:
            res["small_problems"] = batched_small(args, native, torch, np, inputs, dev)
        res["paper_size_problems"] = batched_paper_size(args, native, torch, np, inputs, dev)
        return res
    print("[bench] batched: generating 64 starts", file=sys.stderr, flush=True)
    probs = inputs.batched_problems(64)
    u = inputs.qmc_points(4096, 5)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y = T(np.concatenate([c["y"] for c in probs]))
    par = {k: T(np.concatenate([c["init"][k] for c in probs])) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    n = [c["n"] for c in probs]
    g = [c["g"] for c in probs]
    ut = T(u)
    it = args.batched_iters
    # warm-up (also runs the autotuner once for this shape)
    native.cfust_em_fit_batched(y, n, g, par, ut, max_iter=1, tol=1e-6, precision="fp32")
    torch.cuda.synchronize()
    print(f"[bench] batched: fit of 64 starts, up to {it} iterations", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    fit, trace, n_iter, status = native.cfust_em_fit_batched(y, n, g, par, ut, max_iter=it, tol=1e-6,
                                                             precision="fp32")
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    evals = int(sum((int(n_iter[k]) + 1) * n[k] * g[k] for k in range(len(n))))
    res = {"workload": "64 starts, n~U{5000..50000}, g~U{2..6}, p=q=5, N=4096, fp32 integrand",
           "iterations_cap": it, "seconds": round(tb, 3), "pair_evals_per_s": round(evals / tb, 1),
           "n_iter_min": int(n_iter.min()), "n_iter_max": int(n_iter.max()),
           "n_iter_mean": round(float(n_iter.mean()), 2), "failed": int((status != 0).sum()),
           "launch_shape": native.cfust_batched_config()}
    if not args.no_sequential:
        print("[bench] batched: same starts one by one", file=sys.stderr, flush=True)
        ys = [T(c["y"]) for c in probs]
        ps = [{kk: T(v) for kk, v in c["init"].items()} for c in probs]
        prof = native.prof_buffer()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq_iters = 0
        for k in range(len(probs)):
            f = native.cfust_em_fit(ys[k], ps[k], ut, max_iter=it, tol=1e-6, precision="fp32",
                                    prof=prof)
            seq_iters += int(f["n_iter"]) + 1
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        kern = sum(prof[s] for s in range(native.PROF_SLOTS)) * 1e-3
        res["sequential_seconds"] = round(ts, 3)
        res["speedup_vs_sequential"] = round(ts / tb, 3)
        # what batching can save on these problems: the one-by-one fits'
        # time outside their kernels (host round trip and launches per
        # iteration), each problem filling the GPU on its own
        res["sequential_kernel_seconds"] = round(kern, 3)
        res["sequential_host_us_per_iteration"] = round(1e6 * (ts - kern) / seq_iters, 1)
        res["sequential_kernel_ms_per_iteration"] = round(1e3 * kern / seq_iters, 3)
    if not args.no_batched_small:
        res["small_problems"] = batched_small(args, native, torch, np, inputs, dev)
    res["paper_size_problems"] = batched_paper_size(args, native, torch, np, inputs, dev)
    return res


def batched_paper_size(args, native, torch, np, inputs, dev):
    """Starts at the paper's data-set size, where one wave per pair leaves
    the chip idle at the end of every launch: 32 starts with n = 202,
    g ~ U{2..6}, p = q = 5, N = 4096, FP32 integrand, exactly 50 iterations
    (tolerance 0).  The autotuned fit (it may give each pair K waves of
    N / K points) against the fastest shape with one wave per pair, each
    K = 1 candidate pinned in turn."""
    print("[bench] batched: 32 starts of n = 202", file=sys.stderr, flush=True)
    probs = inputs.batched_problems(32, n_lo=202, n_hi=202, seed_offset=6)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    u = T(inputs.qmc_points(4096, 5))
    y = T(np.concatenate([c["y"] for c in probs]))
    par = {k: T(np.concatenate([c["init"][k] for c in probs])) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    n = [c["n"] for c in probs]
    g = [c["g"] for c in probs]
    it = 50

    def fit(tile):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, trace, n_iter, status = native.cfust_em_fit_batched(y, n, g, par, u, max_iter=it,
                                                               tol=0.0, precision="fp32",
                                                               tile=tile)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, trace, int((status != 0).sum())

    native.cfust_em_fit_batched(y, n, g, par, u, max_iter=1, tol=0.0, precision="fp32")
    ta, trace_a, failed = fit(0)
    shape = native.cfust_batched_config()
    one_wave = {}
    k = 0
    while True:
        s = native.cfust_batched_shape(k)
        if s is None:
            break
        if s["waves_per_pair"] == 1:
            one_wave[k + 1] = fit(k + 1)
        k += 1
    best = min(one_wave, key=lambda t: one_wave[t][0])
    t1, trace_1, failed_1 = one_wave[best]
    pairs = sum(n[k] * g[k] for k in range(len(n)))
    d = np.abs(trace_a[:, it] / trace_1[:, it] - 1)
    rel_diff = float(d[np.isfinite(d)].max()) if np.isfinite(d).any() else None
    return {"workload": "32 starts, n=202, g~U{2..6}, p=q=5, N=4096, fp32 integrand, 50 iterations",
            "pairs_per_iteration": pairs, "seconds": round(ta, 4), "launch_shape": shape,
            "one_wave_per_pair_best_seconds": round(t1, 4),
            "one_wave_per_pair_best_shape": native.cfust_batched_shape(best - 1),
            "speedup_of_tuned_split": round(t1 / ta, 3), "failed": failed,
            "failed_one_wave": failed_1,
            "final_loglik_rel_diff_vs_one_wave": rel_diff}


def batched_small(args, native, torch, np, inputs, dev):
    """The same recipe at the size the batched form is for: 256 starts with
    n ~ U{150..500} (the paper's data set has 202 observations), g ~ U{2..6},
    p = q = 5, N = 1024, FP32 integrand, 50 iterations; batched against one
    by one."""
    print("[bench] batched: 256 small starts", file=sys.stderr, flush=True)
    probs = inputs.batched_problems(256, n_lo=150, n_hi=500, seed_offset=5)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    u = T(inputs.qmc_points(1024, 5))
    y = T(np.concatenate([c["y"] for c in probs]))
    par = {k: T(np.concatenate([c["init"][k] for c in probs])) for k in ("pi", "mu", "Sigma", "Delta", "nu")}
    n = [c["n"] for c in probs]
    g = [c["g"] for c in probs]
    it = 50
    native.cfust_em_fit_batched(y, n, g, par, u, max_iter=1, tol=1e-6, precision="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit, trace, n_iter, status = native.cfust_em_fit_batched(y, n, g, par, u, max_iter=it, tol=1e-6,
                                                             precision="fp32")
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    res = {"workload": "256 starts, n~U{150..500}, g~U{2..6}, p=q=5, N=1024, fp32 integrand",
           "iterations_cap": it, "seconds": round(tb, 4),
           "n_iter_mean": round(float(n_iter.mean()), 2), "failed": int((status != 0).sum())}
    if not args.no_sequential:
        ys = [T(c["y"]) for c in probs]
        ps = [{k: T(v) for k, v in c["init"].items()} for c in probs]
        prof = native.prof_buffer()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        points = 0
        for k in range(len(probs)):
            f = native.cfust_em_fit(ys[k], ps[k], u, max_iter=it, tol=1e-6, precision="fp32",
                                    prof=prof)
            points += (int(f["n_iter"]) + 1) * n[k] * g[k] * 1024
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        res["sequential_seconds"] = round(ts, 4)
        res["speedup_vs_sequential"] = round(ts / tb, 2)
        # the one-by-one fits' pair kernels (each pair split over several
        # waves at these sizes) per pair and QMC point, for comparison with
        # the persistent batched kernel's (from its kernel trace)
        res["sequential_pair_kernel_ps_per_pair_point"] = round(prof[1] * 1e9 / points, 2)
    return res


def em_fit_form(args, native, torch, np, inputs, dev):
    """The 50-iteration EM fit of the benchmark workload (n=20000, p=q=4,
    g=3, N=4096) from its k-means start, tolerance 1e-6 on the Aitken
    limit, through cfust_em_fit (graph-captured iterations), FP64 and FP32
    integrands: wall time, iterations, time per iteration and the final l."""
    c = inputs.config(2)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y, u = T(c["y"]), T(c["u"])
    res = {"workload": "cfust-em n=20000 p=4 q=4 g=3 N=4096 (k-means start), max 50 iterations, "
                       "tol 1e-6"}
    for prec in ("fp64", "fp32"):
        print(f"[bench] em fit: workload 2 {prec}", file=sys.stderr, flush=True)
        par = {k: T(v) for k, v in c["init"].items()}
        native.cfust_em_fit(y, par, u, max_iter=1, tol=1e-6, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit = native.cfust_em_fit(y, par, u, max_iter=50, tol=1e-6, precision=prec)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        it = int(fit["n_iter"])
        tr = np.asarray(fit["trace"])
        res[prec] = {"seconds": round(ts, 4), "iterations": it,
                     "ms_per_iteration": round(1e3 * ts / max(it, 1), 3),
                     "loglik_start": float(tr[0]), "loglik_final": float(tr[it])}
    return res


def high_q_form(args, native, torch, np, inputs, dev):
    """High-q stress case (workload 6: n=202, p=q=11, g=2, N=8192) from the
    k-means start.  (1) 100 EM iterations, FP64 and FP32 integrands, timed
    per iteration.  (2) The whole fit with the exact nu step, FP64, Aitken
    tolerance 1e-6, up to 600 iterations, and how it ends: with about 200
    free parameters per component and 202 observations a component
    degenerates (its Sigma turns singular, where the likelihood is
    unbounded), which the new Sigma's pivot guard reports as ENOTPD naming
    that component.  The paper's only timings are whole fits of R and
    MATLAB code on a data set of this shape (4-core PCs, iteration count
    and tolerance not stated): context, not a like-for-like baseline."""
    c = inputs.config(6)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y, par, u = T(c["y"]), {k: T(v) for k, v in c["init"].items()}, T(c["u"])
    iters = 100
    res = {"workload": f"cfust-em n=202 p=q=11 g=2 N=8192 (k-means start), {iters} iterations"}
    for prec in ("fp64", "fp32"):
        print(f"[bench] high-q: {iters} EM iterations {prec}", file=sys.stderr, flush=True)
        native.cfust_em_fit(y, par, u, max_iter=1, tol=0.0, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit = native.cfust_em_fit(y, par, u, max_iter=iters, tol=0.0, precision=prec)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        tr = np.asarray(fit["trace"])
        res[prec] = {"seconds": round(ts, 3), "ms_per_iteration": round(1e3 * ts / iters, 3),
                     "loglik_start": float(tr[0]), "loglik_max": float(tr.max()),
                     "iteration_of_max": int(tr.argmax()), "loglik_end": float(tr[-1])}
    print("[bench] high-q: whole fit, exact nu step, FP64", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        fit = native.cfust_em_fit(y, par, u, max_iter=600, tol=1e-6, nu_mode="exact")
        end = "converged (Aitken, 1e-6)" if fit["n_iter"] < 600 else "iteration cap (600)"
    except native.CfustError as e:
        if e.code != native.ENOTPD or e.partial is None:
            raise
        fit, end = e.partial, f"ENOTPD: component {e.bad} degenerated (new Sigma singular)"
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    tr = np.asarray(fit["trace"])
    res["whole_fit_exact_fp64"] = {
        "end": end, "iterations": int(fit["n_iter"]), "seconds": round(ts, 3),
        "loglik_start": float(tr[0]), "loglik_max": float(tr.max()),
        "iteration_of_max": int(tr.argmax()), "loglik_end": float(tr[-1])}
    res["paper_whole_fit_seconds_context"] = {
        "R_1_thread": 2310.83, "MATLAB_1_thread": 2635.69, "R_best": 532.29, "MATLAB_best": 516.34}
    return res


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-obs-per-thread", type=int, default=100,
                    help="observations per thread of the all-cores oracle timing")
    ap.add_argument("--cpu-obs", type=int, default=500,
                    help="observations of the workload timed on the CPU oracle")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32-form speedup leg (n=200000, p=q=6, g=4, N=8192)")
    ap.add_argument("--form-reps", type=int, default=2)
    ap.add_argument("--no-form-errors", action="store_true",
                    help="precision leg: skip the per-quantity FP32 errors on all pairs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form leg (64 starts, p=q=5, N=4096, FP32)")
    ap.add_argument("--batched-iters", type=int, default=50)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-form leg (n=1000000, p=q=6, g=4, N=8192)")
    ap.add_argument("--no-batched-large", action="store_true",
                    help="batched leg: only the 256 small problems, not the 64 starts")
    ap.add_argument("--no-batched-small", action="store_true",
                    help="batched leg: skip the 256 small problems (n 150-500)")
    ap.add_argument("--no-fit", action="store_true",
                    help="skip the 50-iteration EM fit of the benchmark workload")
    ap.add_argument("--surrogate-em", action="store_true",
                    help="also run the whole-fit comparison of GHK EM and the two-phase "
                         "surrogate EM at n=1000000 (several minutes)")
    ap.add_argument("--no-high-q", action="store_true",
                    help="skip the high-q stress leg (100 EM iterations, n=202, p=q=11, g=2, N=8192)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched leg: skip fitting the starts one by one for comparison")
    ap.add_argument("--cost-probe", action="store_true",
                    help="only run the diagnostic kernels of the per-call cost model (for "
                         "rocprofv3 counters) and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (traffic calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; use --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2005_06848_amd import inputs, native

    L = native.lib()
    dev = torch.device("cuda:0")
    if args.cost_probe:
        cost_probe(native, torch, dev)
        return
    c = inputs.config(2)
    n, p, q, g, N = c["n"], c["p"], c["q"], c["g"], c["n_qmc"]
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    y = T(c["y"])
    u = T(c["u"])
    init = {k: T(v) for k, v in c["init"].items()}
    par = {k: v.clone() for k, v in init.items()}
    S = native.stats_size(p, q)
    stats = torch.empty((g, S), dtype=torch.float64, device=dev)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    ws = native.alloc_workspace(n, p, q, g, N, args.precision)
    prof = native.prof_buffer()
    opts = native.make_opts(precision=args.precision, workspace=ws, prof=prof)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    out = native.EstepOut(None, None, None, None, None, None, P(stats), P(ll), -1)
    bad = ctypes.c_int(-1)
    pp = [P(par[k]) for k in ("pi", "mu", "Sigma", "Delta", "nu")]

    def step():
        rc = L.cfust_estep(P(y), n, p, q, g, pp[0], pp[1], pp[2], pp[3], pp[4], P(u), N,
                           ctypes.byref(opts), ctypes.byref(out))
        if rc:
            raise native.CfustError(rc, "cfust_estep", out.bad_component)
        rc = L.cfust_mstep(P(stats), n, p, q, g, pp[1], pp[3], pp[4], ctypes.byref(opts),
                           pp[0], pp[1], pp[2], pp[3], pp[4], ctypes.byref(bad))
        if rc:
            raise native.CfustError(rc, "cfust_mstep", bad.value)

    print(f"[bench] warmup {args.warmup} steps: {WORKLOAD}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in par:
        par[k].copy_(init[k])
    for s in range(4):
        prof[s] = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    pairs = n * g
    value = pairs / (ms_per_step * 1e-3)
    pair_ms = prof[1] / args.steps
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, pair kernel {pair_ms:.3f} ms, "
          f"prepare {prof[0] / args.steps:.3f} ms, stats {prof[2] / args.steps:.3f} ms, "
          f"mstep {prof[3] / args.steps:.3f} ms", file=sys.stderr, flush=True)

    if args.copy_probe_mib > 0:
        # one elementwise kernel that reads and writes exactly this many bytes
        nb = args.copy_probe_mib * (1 << 20)
        a = torch.empty(nb // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(f"[bench] copy probe {args.copy_probe_mib} MiB done", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (pair kernel): ALU-bound (FP64 VALU).
    # Per-call costs as measured on the current sources, else the nominal
    # ones; HBM traffic from counters taken on the current sources, else null.
    digest = kernel_sources_digest()
    prec_key = "fp64" if args.precision == "fp64" else "fp32"
    measured = (MEASURED_COSTS is not None and MEASURED_COSTS.get("sources") == digest)
    costs = MEASURED_COSTS[prec_key] if measured else NOMINAL_COSTS
    fpp = flops_per_pair(p, q, N, costs)
    ach = fpp * pairs / (pair_ms * 1e-3) / 1e12
    fpp_nom = flops_per_pair(p, q, N, NOMINAL_COSTS)
    ach_nom = fpp_nom * pairs / (pair_ms * 1e-3) / 1e12
    traffic = None
    if (args.precision == "fp64" and PAIR_KERNEL_COUNTERS is not None
            and PAIR_KERNEL_COUNTERS.get("sources") == digest):
        traffic = PAIR_KERNEL_COUNTERS["traffic"]
    peak = PEAK_FP64_VALU_TFLOPS if prec_key == "fp64" else PEAK_FP32_VALU_TFLOPS
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4),
            "traffic": traffic,
            "kernel": f"pair_kernel<{'double' if prec_key == 'fp64' else 'float'},{q},true>",
            "kernel_ms": round(pair_ms, 4), "flops_per_pair": fpp,
            "cost_model": ({"source": "measured per call", **costs} if measured else
                           {"source": "nominal (no measurement on these sources)", **costs}),
            "nominal_model": {"flops_per_pair": fpp_nom, "achieved": round(ach_nom, 3),
                              "frac": round(ach_nom / peak, 4)},
            "sources_digest": digest}

    forms = None
    if not args.no_forms:
        forms = precision_form(args, native, L, torch, np, inputs, dev)
    if not args.no_surrogate:
        forms = forms or {}
        forms["surrogate"] = surrogate_form(args, native, torch, np, inputs, dev)
    if not args.no_batched:
        forms = forms or {}
        forms["batched"] = batched_form(args, native, torch, np, inputs, dev)
    if not args.no_high_q:
        forms = forms or {}
        forms["high_q"] = high_q_form(args, native, torch, np, inputs, dev)
    if args.surrogate_em:
        forms = forms or {}
        forms["surrogate_em"] = surrogate_em_form(args, native, torch, np, inputs, dev)
    if not args.no_fit:
        forms = forms or {}
        forms["em_fit"] = em_fit_form(args, native, torch, np, inputs, dev)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        m = min(args.cpu_obs, n)
        print(f"[bench] cpu baseline: oracle E-step on {m} observations", file=sys.stderr, flush=True)
        tc0 = time.perf_counter()
        oracle.estep(c["y"][:m], c["init"], c["u"], want=())
        tc = time.perf_counter() - tc0
        # one thread per block of observations (the paper's J_l blocks) on
        # the host cores this process may use, at most 16: the host's CPU
        # share for one GPU; the oracle's C calls release the GIL
        from concurrent.futures import ThreadPoolExecutor
        host = host_description()
        nt = max(1, min(16, host["affinity"]))
        per = max(1, min(args.cpu_obs_per_thread, (n - m) // nt))
        blocks = [c["y"][m + t * per:m + (t + 1) * per] for t in range(nt)]
        print(f"[bench] cpu baseline: oracle E-step on {nt} threads x {per} observations",
              file=sys.stderr, flush=True)
        with ThreadPoolExecutor(nt) as ex:
            tm0 = time.perf_counter()
            list(ex.map(lambda yb: oracle.estep(yb, c["init"], c["u"], want=()), blocks))
            tm = time.perf_counter() - tm0
        cpu = {"value": round(nt * per * g / tm, 3), "unit": "pairs/s", "cores": nt,
               "kind": "oracle",
               "sample": f"observations {m}..{m + nt * per - 1} of the workload "
                         f"({nt * per * g} pairs), full N={N}, E-step incl. tau and partial "
                         f"sums, {nt} threads of {per} observations each, {tm:.1f} s",
               "single_thread": {"value": round(m * g / tc, 3), "cores": 1,
                                 "sample": f"first {m} observations ({m * g} pairs), "
                                           f"{tc:.1f} s"},
               "host": host}

    line = {
        "metric": "E-step (obs x comp) evals/sec at stated tol; FP32/surrogate vs FP64 QMC speedup",
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": n, "p": p, "q": q, "g": g, "n_qmc": N,
                   "step": "one EM iteration (E-step + M-step)", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
