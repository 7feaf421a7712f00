"""Stability limits of the forcing schemes.

The paper measures, for a circular droplet (200 x 200 periodic lattice,
radius 30, Carnahan-Starling EOS, tanh profile of Eq. 24), the lowest reduced
temperature T_min/Tc at which each forcing scheme still runs (Sec. III.C,
Figs. 1-2: Shan-Chen, EDM, Guo et al., modified EDM; Sec. IV.B: the improved
scheme).  This module runs that experiment as one batched launch per chunk of
runs: every (scheme, tau, sigma) case at every temperature of a grid is an
independent lattice of the batch, and the batch's per-run divergence status
(a non-finite or non-positive density, or a density outside the EOS range of
Eq. 8) decides stability.

The paper states neither the run length nor its divergence criterion, so the
limits found here are comparable with its figures only in their order.
Every lattice update runs in the HIP library; this file prepares parameters
and reads back statuses.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import synth

from . import lbm

CS = dict(eos=lbm.LBM_EOS_CS, a=1.0, b=4.0, R=1.0, omega=0.0)

SCHEME_NAMES = {lbm.LBM_SCHEME_SHANCHEN: "Shan-Chen", lbm.LBM_SCHEME_EDM: "EDM",
                lbm.LBM_SCHEME_IMPROVED: "improved", lbm.LBM_SCHEME_EDM_MODIFIED: "modified EDM",
                lbm.LBM_SCHEME_LADD: "Ladd"}


@dataclass(frozen=True)
class Case:
    """One forcing scheme at one relaxation time (sigma: improved scheme only)."""
    scheme: int
    tau: float
    sigma: float = 0.0

    @property
    def name(self) -> str:
        n = SCHEME_NAMES[self.scheme]
        if self.scheme == lbm.LBM_SCHEME_IMPROVED:
            n = "Guo et al." if self.sigma == 0.0 else f"improved sigma={self.sigma:g}"
        return f"{n}, tau={self.tau:g}"


def critical_T() -> float:
    return lbm.lbm_critical_point(CS["eos"], CS["a"], CS["b"], CS["R"], CS["omega"])[0]


def droplet_runs(cases, t_grid, nx=200, ny=200, r0=30.0, width=2.0, precision=lbm.LBM_PREC_F64):
    """lbm_params and initial densities for every (case, T/Tc): a droplet of
    radius r0 at the lattice centre between the Maxwell densities at T."""
    Tc = critical_T()
    ps, rhos, keys = [], [], []
    for case in cases:
        for t in t_grid:
            rl, rg, _ = lbm.lbm_maxwell(CS["eos"], CS["a"], CS["b"], CS["R"], CS["omega"], t * Tc)
            ps.append(lbm.params(nx, ny, tau=case.tau, T=t * Tc, scheme=case.scheme,
                                 sigma=case.sigma, precision=precision, **CS))
            rhos.append(synth.droplet(nx, ny, rl, rg, r0, width))
            keys.append((case, float(t)))
    return ps, rhos, keys


def lowest_stable(t_grid, stable):
    """Lowest grid temperature T such that every grid temperature >= T is stable
    (None when the highest is unstable), and whether stability is monotone in T
    (no stable temperature below an unstable one)."""
    t = np.asarray(t_grid, dtype=float)
    s = np.asarray(stable, dtype=bool)
    order = np.argsort(-t)
    tmin = None
    first_bad = None
    for k, i in enumerate(order):
        if not s[i]:
            first_bad = k
            break
        tmin = float(t[i])
    monotone = first_bad is None or not np.any(s[order[first_bad:]])
    return tmin, bool(monotone)


def sweep(cases, t_grid, steps=20000, nx=200, ny=200, r0=30.0, width=2.0,
          precision=lbm.LBM_PREC_F64, graph_steps=100, max_runs=256, tune=True):
    """Run every case at every grid temperature for `steps` steps.  Returns one
    dict per case: t_grid, status, diverged_at (step, -1 if stable), t_min,
    monotone; plus a summary of the launch (runs, lattice updates)."""
    import torch
    t_grid = [float(t) for t in t_grid]
    ps, rhos, keys = droplet_runs(cases, t_grid, nx, ny, r0, width, precision)
    status = np.zeros(len(ps), dtype=np.int32)
    div = np.full(len(ps), -1, dtype=np.int64)
    for s in range(0, len(ps), max_runs):
        e = min(len(ps), s + max_runs)
        b = lbm.Batch(ps[s:e], rhos[s:e])
        if tune:
            b.tune()
        if graph_steps:
            b.set_graph_steps(graph_steps)
        b.step(steps)
        _, _, st, dv = b.coexistence()
        torch.cuda.synchronize()
        b.close()
        status[s:e] = st
        div[s:e] = np.where(st == lbm.LBM_OK, -1, dv)
    out = []
    n = len(t_grid)
    for k, case in enumerate(cases):
        st = status[k * n:(k + 1) * n]
        dv = div[k * n:(k + 1) * n]
        tmin, mono = lowest_stable(t_grid, st == lbm.LBM_OK)
        out.append(dict(case=case, name=case.name, t_grid=t_grid, status=st.tolist(),
                        diverged_at=dv.tolist(), t_min=tmin, monotone=mono))
    return out, dict(runs=len(ps), lattice_updates=len(ps) * nx * ny * steps, keys=keys,
                     status=status, diverged_at=div)


def table(results) -> str:
    """Plain-text table of T_min/Tc per case."""
    lines = [f"{'case':34s} T_min/Tc  monotone"]
    for r in results:
        tm = "unstable" if r["t_min"] is None else f"{r['t_min']:.3f}"
        lines.append(f"{r['name']:34s} {tm:>8s}  {r['monotone']}")
    return "\n".join(lines)
