"""Learned sigma proposal for the improved forcing scheme.

The paper chooses the constant sigma of Eq. (31) by running flat-interface
simulations with several sigma and keeping the one whose coexistence
densities fit the Maxwell construction (Sec. IV.B; sigma = 0.105 for C-S).
This module automates that with a surrogate:

  1. dataset:  batched flat-interface runs (one persistent launch per step for
               hundreds of uneven lattices) over (T/Tc, tau, sigma), recording
               (log rho_l, log rho_g) of each run that did not diverge;
  2. fit:      the 3-64-64-2 network trained by the library's own kernels;
  3. propose:  for a new (T/Tc, tau), the sigma on a fine grid in [0, 0.2]
               whose predicted densities are closest (in log space) to the
               Maxwell densities;
  4. verify:   an FP64 lattice run at the proposed sigma decides.  When it
               misses, one Newton step on sigma uses the network's slope
               d log(rho_g)/d sigma with the measured lattice density, and a
               second run decides; LB bisection on sigma is the last fallback.

Every lattice update and every network pass runs in the HIP library; this
file only prepares parameters and moves arrays.
"""
from __future__ import annotations

import math
import time

import numpy as np

import synth

from . import lbm
from . import mlp as mlpb

CS = dict(eos=lbm.LBM_EOS_CS, a=1.0, b=4.0, R=1.0, omega=0.0)


def critical_T():
    return lbm.lbm_critical_point(CS["eos"], CS["a"], CS["b"], CS["R"], CS["omega"])[0]


def maxwell(t_over_tc):
    Tc = critical_T()
    rl, rg, _ = lbm.lbm_maxwell(CS["eos"], CS["a"], CS["b"], CS["R"], CS["omega"], t_over_tc * Tc)
    return rl, rg


def slab_runs(runs, precision, seed=synth.BASE_SEED, noise=0.01, rho_ref=math.nan):
    """lbm_params and initial densities of flat-interface runs (slab [nx/4, 3nx/4))."""
    Tc = critical_T()
    ps, rhos = [], []
    for i, r in enumerate(runs):
        rl, rg = maxwell(r["t_over_tc"])
        ps.append(lbm.params(r["nx"], r["ny"], tau=r["tau"], T=r["t_over_tc"] * Tc,
                             scheme=lbm.LBM_SCHEME_IMPROVED, sigma=r["sigma"], precision=precision,
                             rho_ref=rho_ref, **CS))
        rhos.append(synth.slab(r["nx"], r["ny"], rl, rg, r["nx"] / 4, 3 * r["nx"] / 4, 2.0, noise, seed, i))
    return ps, rhos


def run_batch(runs, steps, precision=lbm.LBM_PREC_F32DEV, graph_steps=100, tune=True, seed=synth.BASE_SEED,
              rho_ref=math.nan, window=2000, samples=10):
    """Advance a batch of flat-interface runs for `steps` steps and return their
    coexistence densities averaged over `samples` snapshots spread over the last
    `window` steps (slowly damped sound waves in wide vapour regions make a single
    snapshot noisy), plus the relative spread of those snapshots."""
    import torch
    ps, rhos = slab_runs(runs, precision, seed, rho_ref=rho_ref)
    b = lbm.Batch(ps, rhos)
    if tune:
        b.tune()
    if graph_steps:
        b.set_graph_steps(graph_steps)
    nodes = sum(p.nx * p.ny for p in ps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    window = min(window, steps // 2)
    every = max(1, window // samples)
    b.step(steps - every * samples)
    L, G = [], []
    for _ in range(samples):
        b.step(every)
        l, g, st, dv = b.coexistence()
        L.append(l)
        G.append(g)
    el = time.perf_counter() - t0
    b.close()
    L, G = np.asarray(L), np.asarray(G)
    with np.errstate(invalid="ignore", divide="ignore"):
        rl, rg = L.mean(0), G.mean(0)
        spread = np.maximum((L.max(0) - L.min(0)) / rl, (G.max(0) - G.min(0)) / rg)
    return dict(rho_l=rl, rho_g=rg, status=st, diverged_at=dv, spread=spread, seconds=el,
                lups=nodes * steps)


def dataset(nruns, steps, precision=lbm.LBM_PREC_F32DEV, batch=256, seed=synth.BASE_SEED,
            t_range=(0.5, 0.95), max_spread=0.02, rho_ref=0.0, log=None):
    """Sweep runs drawn as in the batched coexistence sweep; X = (T/Tc, tau, sigma),
    Y = (log rho_l, log rho_g) (time-averaged) of the runs that stayed finite and
    whose snapshots over the averaging window spread by less than max_spread.  By
    default the populations are stored as plain FP32 values (rho_ref = 0) with FP32
    collision arithmetic (mass and momentum change restored in FP64 per node)."""
    X, Y, ndiv, nmov, secs, lups = [], [], 0, 0, 0.0, 0
    for k in range(0, nruns, batch):
        runs = synth.sweep_runs(min(batch, nruns - k), seed=seed + k, t_range=t_range)
        out = run_batch(runs, steps, precision, seed=seed + k, rho_ref=rho_ref)
        secs += out["seconds"]
        lups += out["lups"]
        for r, l, g, s, dr in zip(runs, out["rho_l"], out["rho_g"], out["status"], out["spread"]):
            if s != lbm.LBM_OK or not (l > 0 and g > 0 and math.isfinite(l) and math.isfinite(g)):
                ndiv += 1
            elif not dr <= max_spread:
                nmov += 1
            else:
                X.append((r["t_over_tc"], r["tau"], r["sigma"]))
                Y.append((math.log(l), math.log(g)))
        if log:
            log(f"dataset: {k + batch}/{nruns} runs, {ndiv} diverged, {nmov} not settled, "
                f"{lups / secs / 1e6:.0f} MLUPS")
    return (np.asarray(X, dtype=np.float32), np.asarray(Y, dtype=np.float32),
            dict(diverged=ndiv, unsettled=nmov, seconds=secs, lups=lups))


def fit(X, Y, steps=4000, lr=2e-3, batch=1024, seed=synth.BASE_SEED, split=0.8):
    """Train on a seeded split of the runs; returns (net, report)."""
    n = X.shape[0]
    order = np.argsort(synth.uniform(seed, 99, np.arange(n, dtype=np.uint64)))
    ntr = int(split * n)
    tr, te = order[:ntr], order[ntr:]
    Xtr, Ytr = X[tr], Y[tr]
    norm = mlpb.make_norm(Xtr.mean(0), Xtr.std(0) + 1e-6, Ytr.mean(0), Ytr.std(0) + 1e-6)
    net = mlpb.Mlp(synth.mlp_init(seed), norm, max_batch=max(batch, 4096))
    hist = net.train(Xtr, Ytr, steps=steps, lr=lr, batch=batch, seed=seed, log_every=max(1, steps // 10))
    report = dict(train_runs=int(ntr), test_runs=int(n - ntr), loss_history=hist)
    if n - ntr > 0:
        pred = np.concatenate([net.forward(X[te][i:i + 4096]) for i in range(0, n - ntr, 4096)])
        err = np.abs(np.exp(pred - Y[te]) - 1)
        report["heldout_rel_err_median"] = [float(v) for v in np.median(err, 0)]
        report["heldout_rel_err_p95"] = [float(v) for v in np.quantile(err, 0.95, axis=0)]
    return net, report


def propose_sigma(net, t_over_tc, tau, grid=None):
    """sigma in [0, 0.2] whose predicted (log rho_l, log rho_g) is closest to Maxwell."""
    grid = np.linspace(0.0, 0.2, 4001) if grid is None else np.asarray(grid)
    rl, rg = maxwell(t_over_tc)
    X = np.column_stack([np.full(grid.size, t_over_tc), np.full(grid.size, tau), grid]).astype(np.float32)
    Y = net.forward(X).astype(np.float64)
    d = (Y[:, 0] - math.log(rl)) ** 2 + (Y[:, 1] - math.log(rg)) ** 2
    i = int(np.argmin(d))
    return float(grid[i]), (float(math.exp(Y[i, 0])), float(math.exp(Y[i, 1])))


def slope_log_rho_g(net, t_over_tc, tau, sigma, h=2e-3):
    """d log(rho_g) / d sigma of the network at (T/Tc, tau, sigma) (central difference)."""
    X = np.array([[t_over_tc, tau, sigma - h], [t_over_tc, tau, sigma + h]], dtype=np.float32)
    Y = net.forward(X).astype(np.float64)
    return (Y[1, 1] - Y[0, 1]) / (2 * h)


def propose_and_verify(net, pairs, steps=30000, tol=0.01, bisect_iters=8, nx=256, ny=32):
    """The learned proposal, each pick checked by a lattice run.  Returns per pair the sigma
    used, its relative errors against Maxwell (rho_l, rho_g) and how many FP64
    lattice runs it took."""
    sig = np.array([propose_sigma(net, t, tau)[0] for t, tau in pairs])
    err, out = verify(pairs, sig, steps, nx, ny)
    runs = np.ones(len(pairs), dtype=int)
    miss = np.nonzero(np.max(err, axis=1) > tol)[0]
    if miss.size:
        new = sig.copy()
        for i in miss:
            t, tau = pairs[i]
            g = out["rho_g"][i]
            if math.isfinite(g) and g > 0:
                s = slope_log_rho_g(net, t, tau, sig[i])
                if s > 0:
                    new[i] = float(np.clip(sig[i] + (math.log(maxwell(t)[1]) - math.log(g)) / s, 0.0, 0.2))
        e2, _ = verify([pairs[i] for i in miss], new[miss], steps, nx, ny)
        runs[miss] += 1
        for k, i in enumerate(miss):
            if np.max(e2[k]) < np.max(err[i]):
                sig[i], err[i] = new[i], e2[k]
        still = [i for i in miss if np.max(err[i]) > tol]
        if still:
            sb, _ = bisect_sigma([pairs[i] for i in still], steps, bisect_iters, nx, ny)
            eb, _ = verify([pairs[i] for i in still], sb, steps, nx, ny)
            for k, i in enumerate(still):
                runs[i] += bisect_iters + 1
                if np.max(eb[k]) < np.max(err[i]):
                    sig[i], err[i] = sb[k], eb[k]
    return sig, err, runs


def verify(pairs, sigmas, steps=30000, nx=256, ny=32, precision=lbm.LBM_PREC_F64, seed=synth.BASE_SEED + 777):
    """FP64 lattice runs (nx x ny, slab [nx/4, 3nx/4)) at the given sigma for each
    (T/Tc, tau); returns relative errors of rho_l, rho_g against Maxwell."""
    runs = [dict(nx=nx, ny=ny, t_over_tc=t, tau=tau, sigma=s) for (t, tau), s in zip(pairs, sigmas)]
    out = run_batch(runs, steps, precision, seed=seed)
    errs = []
    for (t, _), l, g, s in zip(pairs, out["rho_l"], out["rho_g"], out["status"]):
        rl, rg = maxwell(t)
        errs.append((abs(l / rl - 1), abs(g / rg - 1)) if s == lbm.LBM_OK else (math.inf, math.inf))
    return np.asarray(errs), out


def bisect_sigma(pairs, steps=30000, iters=10, nx=256, ny=32, precision=lbm.LBM_PREC_F64):
    """The method without the surrogate: bisection on sigma with one lattice run per
    pair and iteration (rho_g increases with sigma), all pairs batched together."""
    lo = np.zeros(len(pairs))
    hi = np.full(len(pairs), 0.2)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        _, out = verify(pairs, mid, steps, nx, ny, precision)
        for i, ((t, _), g) in enumerate(zip(pairs, out["rho_g"])):
            if math.isfinite(g) and g < maxwell(t)[1]:
                lo[i] = mid[i]
            else:
                hi[i] = mid[i]
    return 0.5 * (lo + hi), iters * len(pairs)


def heldout_pairs(n=32, seed=synth.BASE_SEED + 4242, t_range=(0.63, 0.95), tau_range=(0.6, 1.5)):
    u = synth.uniform(seed, 0, np.arange(2 * n, dtype=np.uint64)).reshape(n, 2)
    return [(float(t_range[0] + (t_range[1] - t_range[0]) * a), float(tau_range[0] + (tau_range[1] - tau_range[0]) * b))
            for a, b in u]
