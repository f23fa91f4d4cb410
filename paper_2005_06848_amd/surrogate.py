"""Training set and training of the surrogate network for the GHK integrals.

Training set (q = 6): half the samples with correlation matrices
R ~ LKJ(2) (onion method), degrees of freedom uniform on a 0.25 grid in
[5, 20] and truncation points h uniform on [-4, 6]^6; the other half are the
(h, R, dof) of pairs logged along EM runs on other draws of the surrogate
workload's recipe (p = q = 6, g = 4), at the starting values and at later
iterates.  Labels are GHK estimates by the library's own kernel
(cfust_ghk_batch) with 2^14 points; the network learns the covariance in
place of E[V V^T].  Training runs the library's BF16 matrix-core forward/backward and
Adam kernels (cfust_surrogate_train).

Run:  python -m paper_2005_06848_amd.surrogate --out <file>

Options reach beyond that recipe: --h-lo lowers the bottom of the h box
(uniform samples then fill the core [-4, 6]^6 for --core-share of them and
the whole box for the rest; proposal bounds above the top are lowered to it,
as the E-step does), --with-true adds the draws' true parameters to the
logged points, and --init starts from a saved network (its parameters and
standardisation, under the new box).
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np
import torch

from . import inputs
from . import native as nat

Q = 6
H_LO, H_HI = -4.0, 6.0
DOF_LO, DOF_HI = 5.0, 20.0
R_MAX = 0.95
EIG_PERCENTILE = 1.0
N_LABEL = 1 << 14
# other draws of the surrogate workload's recipe (the workload itself uses
# its own seed, so the network never sees the benchmark's data)
PROPOSAL_SEEDS = tuple(range(9001, 9009))
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "surrogate_q6.bin")


def log(msg):
    print(f"[surrogate] {msg}", flush=True)


def feature_rows(h, R, dof):
    """(h | entries of R above the diagonal, row by row | dof) per sample."""
    q = h.shape[1]
    iu = np.triu_indices(q, 1)
    return np.ascontiguousarray(np.concatenate([h, R[:, iu[0], iu[1]], dof[:, None]], axis=1))


def eig_threshold(R):
    """The EIG_PERCENTILE-th percentile of the smallest eigenvalue of R."""
    return float(np.percentile(np.linalg.eigvalsh(R)[:, 0], EIG_PERCENTILE))


def proposal_rows(seeds=PROPOSAL_SEEDS, n_obs=50_000, iterates=(0, 3, 10, 30), per_iterate=100_000,
                  device="cuda", with_true=False, clamp_top=False):
    """Feature rows (h | r | dof) of both integrals of the pairs of FP32 EM
    runs on other draws of the surrogate workload's recipe (n_obs
    observations, p = q = 6, g = 4), logged at the starting values and at
    later iterates; rows inside the training box only, per_iterate of them
    per logged iterate."""
    rng = np.random.default_rng(12345)
    rows = []
    for sd in seeds:
        c = inputs.config(5, n=n_obs, seed=sd)
        y = torch.tensor(c["y"], device=device)
        u = torch.tensor(c["u"], device=device)
        par = {k: torch.tensor(np.asarray(v, dtype=np.float64), device=device)
               for k, v in c["init"].items()}
        true = {k: torch.tensor(np.asarray(v, dtype=np.float64), device=device)
                for k, v in c["true"].items() if k in ("pi", "mu", "Sigma", "Delta", "nu")}
        done = 0
        for it in list(iterates) + ([None] if with_true else []):
            if it is None:
                par = true
            elif it > done:
                res = nat.cfust_em_fit(y, par, u, max_iter=it - done, tol=0.0, precision="fp32")
                par = {k: res[k] for k in ("pi", "mu", "Sigma", "Delta", "nu")}
                done = it
            f = nat.cfust_pair_features(y, par).cpu().numpy()
            if clamp_top:
                f[:, :Q] = np.minimum(f[:, :Q], H_HI)
            keep = (np.all((f[:, :Q] >= H_LO) & (f[:, :Q] <= H_HI), axis=1)
                    & np.all(np.abs(f[:, Q:-1]) <= R_MAX, axis=1)
                    & (f[:, -1] >= DOF_LO) & (f[:, -1] <= DOF_HI))
            f = f[keep]
            rows.append(f[rng.permutation(len(f))[:per_iterate]])
        log(f"proposal: draw {sd}: {sum(len(r) for r in rows)} rows so far")
    return np.concatenate(rows)


def corr_from_rows(r, q=Q):
    """Correlation matrices from the entries above the diagonal, row by row."""
    R = np.zeros((len(r), q, q))
    iu = np.triu_indices(q, 1)
    R[:, iu[0], iu[1]] = r
    R[:, iu[1], iu[0]] = r
    R[:, np.arange(q), np.arange(q)] = 1.0
    return R


def label(h, R, dof, u, chunk=1 << 18, device="cuda"):
    """GHK labels (log T | E[V] | E[V V^T] upper) by the library kernel."""
    out = []
    for s in range(0, len(h), chunk):
        e = min(len(h), s + chunk)
        out.append(nat.cfust_ghk_batch(torch.tensor(h[s:e], device=device),
                                       torch.tensor(R[s:e], device=device),
                                       torch.tensor(dof[s:e], device=device), u))
    return torch.cat(out)


def training_set(m, seed=1, proposal=None, n_label=N_LABEL, device="cuda", core_share=0.0):
    """Feature rows (device [m][22]) and labels (device [m][28]): the first
    half (all rows without a proposal) with R ~ LKJ(2), dof on the grid and h
    uniform in the box, the second half drawn from the proposal rows.  Also
    returns the smallest-eigenvalue threshold of the LKJ part."""
    rng = np.random.default_rng(seed)
    k = m if proposal is None or not len(proposal) else m - m // 2
    core = None
    if core_share > 0.0:
        core = rng.uniform(-4.0, 6.0, size=(int(core_share * k), Q))
    h, R, dof = inputs.surrogate_samples(rng, k, Q, H_LO, H_HI, DOF_LO, DOF_HI, 0.25, 2.0,
                                         h_extra=core)
    thr = eig_threshold(R)
    if k < m:
        pr = proposal[rng.integers(0, len(proposal), size=m - k)]
        h = np.concatenate([h, pr[:, :Q]])
        R = np.concatenate([R, corr_from_rows(pr[:, Q:-1])])
        dof = np.concatenate([dof, pr[:, -1]])
    u = torch.tensor(inputs.qmc_points(n_label, Q, seed=0x51), device=device)
    targ = label(h, R, dof, u, device=device)
    feat = torch.tensor(feature_rows(h, R, dof), device=device)
    return feat, targ, thr


def output_weights(q=Q):
    """Loss weight per output: log T counts as much as all moments together."""
    T = 1 + q + q * (q + 1) // 2
    w = np.ones(T, dtype=np.float32)
    w[0] = T - 1
    return w


def train(m=2_000_000, epochs=200, batch=4096, lr0=2e-3, lr1=2e-6, seed=7, device="cuda",
          with_true=False, clamp_top=False, core_share=0.0, init=None):
    t0 = time.time()
    prop = proposal_rows(device=device, with_true=with_true, clamp_top=clamp_top)
    log(f"proposal rows {len(prop)} ({time.time() - t0:.1f} s)")
    feat, targ, thr = training_set(m, seed=seed, proposal=prop, device=device,
                                   core_share=core_share)
    torch.cuda.synchronize()
    log(f"training set {m} samples labelled ({time.time() - t0:.1f} s)")
    rng_ = [H_LO, H_HI, DOF_LO, DOF_HI, R_MAX, thr]
    net = nat.Surrogate.create(Q, rng_, seed=seed)
    if init is not None:
        # start from a saved network: its parameters and standardisation
        net.set_state(*nat.Surrogate.load(init).get_state())
    trace = []
    step = 10
    for e0 in range(0, epochs, step):
        ne = min(step, epochs - e0)
        # one cosine schedule over all epochs, split into calls of `step` epochs
        a = 0.5 * (1 + np.cos(np.pi * e0 / epochs))
        b = 0.5 * (1 + np.cos(np.pi * (e0 + ne) / epochs))
        lra = lr1 + (lr0 - lr1) * a
        lrb = lr1 + (lr0 - lr1) * b
        trace += net.train(feat, targ, ne, batch=batch, lr0=lra, lr1=lrb, seed=seed + e0,
                           wo=output_weights())
        log(f"epoch {e0 + ne}: loss {trace[-1]:.3e} ({time.time() - t0:.1f} s)")
    return net, trace, rng_


def main():
    global H_LO
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--samples", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr0", type=float, default=2e-3)
    ap.add_argument("--lr1", type=float, default=2e-6)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--h-lo", type=float, default=H_LO, help="bottom of the h box")
    ap.add_argument("--core-share", type=float, default=0.0,
                    help="share of the uniform samples drawn in the core box [-4, 6]^6")
    ap.add_argument("--with-true", action="store_true",
                    help="log the draws' true parameters too")
    ap.add_argument("--init", default=None, help="start from this saved network")
    a = ap.parse_args()
    H_LO = a.h_lo
    net, trace, rng_ = train(a.samples, a.epochs, a.batch, a.lr0, a.lr1, a.seed,
                             with_true=a.with_true, clamp_top=a.h_lo != -4.0 or a.with_true,
                             core_share=a.core_share, init=a.init)
    net.save(a.out)
    log(f"saved {a.out}; range {rng_}; final loss {trace[-1]:.3e}")


if __name__ == "__main__":
    main()
