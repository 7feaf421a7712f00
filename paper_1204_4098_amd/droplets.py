"""Per-droplet diagnostics of the many-droplet workload.

The reduced-precision large run holds 64 droplets (radius 40-120, seeded
non-overlapping layout) on a 4096 x 4096 periodic lattice.  For each droplet
this module reports its mass (the sum of rho over the nodes within r + 8 of
its initial centre) and its pressure jump, the mean p_EOS over the inner disk
(within r/2 of the centre) minus the mean p_EOS of the far vapour (nodes
farther than r_j + 16 from every centre); Laplace's law makes the jump fall as
1/r.  Both are averaged over snapshots spread over the end of the run (the
liquid still carries sound waves whose pressure swings are large).  The same
quantities of isolated droplets of the same radii, centred on 512 x 512
lattices and run in FP64 as one batched launch, are the crop-equivalent
reference (a different vapour reservoir, so a physics-level comparison, not an
elementwise one).

The fields come from the library's moments (lbm_moments); only the region
sums are taken here.
"""
from __future__ import annotations

import math

import numpy as np

import synth

from . import lbm

CS = dict(eos=lbm.LBM_EOS_CS, a=1.0, b=4.0, R=1.0, omega=0.0)


def layout(nx=4096, ny=4096, count=64, rmin=40.0, rmax=120.0, gap=16.0, seed=synth.BASE_SEED):
    """Droplet centres and radii of the workload (seeded rejection sampling)."""
    return synth.droplet_layout(nx, ny, count, rmin, rmax, gap, seed)


def _window(n, c, h):
    """Periodic indices of the window [c - h, c + h] on a ring of n points."""
    return np.arange(int(math.floor(c - h)), int(math.ceil(c + h)) + 1) % n


def _dist2(nx, ny, cx, cy, xs, ys):
    dx = np.abs(xs[None, :] - cx)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(ys[:, None] - cy)
    dy = np.minimum(dy, ny - dy)
    return dx * dx + dy * dy


def report(rho, p, centers, radii, mass_margin=8.0, far_margin=16.0):
    """Per-droplet mass, pressure jump and the far-vapour pressure of one snapshot.

    rho, p: (ny, nx) FP64 fields.  Returns dict(mass, dp, p_far, p_inner)."""
    ny, nx = rho.shape
    near = np.zeros((ny, nx), dtype=bool)
    mass, pc = [], []
    for (cx, cy), r in zip(centers, radii):
        xs = _window(nx, cx, r + far_margin)
        ys = _window(ny, cy, r + far_margin)
        d2 = _dist2(nx, ny, cx, cy, xs, ys)
        near[np.ix_(ys, xs)] |= d2 <= (r + far_margin) ** 2
        mass.append(float(rho[np.ix_(ys, xs)][d2 <= (r + mass_margin) ** 2].sum()))
        pc.append(float(p[np.ix_(ys, xs)][d2 <= (0.5 * r) ** 2].mean()))
    far = ~near
    if not far.any():
        raise ValueError("no far-vapour nodes: droplets cover the lattice")
    p_far = float(p[far].mean())
    pc = np.asarray(pc)
    return dict(mass=np.asarray(mass), dp=pc - p_far, p_far=p_far, p_inner=pc)


def _mean_reports(reps):
    return {k: np.mean([r[k] for r in reps], axis=0) for k in reps[0]}


def run_workload(precision, steps, kw, rho0, centers, radii, window=2000, samples=10, tune=True,
                 graph_steps=100, rho_ref=math.nan):
    """Advance the many-droplet workload `steps` steps and average the per-droplet
    report over `samples` snapshots spread over the last `window` steps; returns
    (report, status)."""
    import torch
    ny, nx = rho0.shape
    lat = lbm.Lattice(lbm.params(nx, ny, precision=precision, rho_ref=rho_ref, **kw), rho0)
    if tune:
        lat.tune()
    if graph_steps:
        lat.set_graph_steps(graph_steps)
    every = max(1, window // samples)
    lat.step(steps - every * samples)
    reps = []
    for _ in range(samples):
        lat.step(every)
        rho, _, _, p = lat.moments(check=False)
        reps.append(report(rho, p, centers, radii))
    torch.cuda.synchronize()
    st = lat.status()
    lat.close()
    return _mean_reports(reps), st


def crop_equivalent(radii, kw, rho_l, rho_g, steps, n=512, noise=0.005, graph_steps=100,
                    precision=lbm.LBM_PREC_F64, window=2000, samples=10):
    """Isolated droplets of the given radii, centred on n x n lattices, all in one
    batched launch, reported like run_workload; returns dict(mass, dp, status)."""
    import torch
    ps, rhos = [], []
    for i, r in enumerate(radii):
        ps.append(lbm.params(n, n, precision=precision, **kw))
        rhos.append(synth.droplet(n, n, rho_l, rho_g, float(r), 2.0, noise, synth.BASE_SEED, 100 + i))
    b = lbm.Batch(ps, rhos)
    b.tune()
    if graph_steps:
        b.set_graph_steps(graph_steps)
    every = max(1, window // samples)
    b.step(steps - every * samples)
    acc_m = np.zeros(len(radii))
    acc_p = np.zeros(len(radii))
    for _ in range(samples):
        b.step(every)
        for i, r in enumerate(radii):
            rho, _, _, p = b.moments(i)
            rep = report(rho, p, [(n / 2.0, n / 2.0)], [float(r)])
            acc_m[i] += rep["mass"][0] / samples
            acc_p[i] += rep["dp"][0] / samples
    torch.cuda.synchronize()
    _, _, st, _ = b.coexistence()
    b.close()
    return dict(mass=acc_m, dp=acc_p, status=np.asarray(st))
