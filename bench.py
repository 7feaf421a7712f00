#!/usr/bin/env python3
"""Benchmark of the fused pseudopotential D2Q9 step on one MI355X.

Prints ONE JSON line.  `value` is whole-job MLUPS (million lattice-node
updates per second) of the plain FP64 fused step on the configured lattice,
timed with inputs resident in HBM.  `roofline` reports the step kernel's
algorithmic HBM traffic (9 populations read + 9 written per node) against the
8 TB/s MI355X peak, with the kernel time measured by HIP events on the stream
the kernel runs on.  `cpu_baseline` times the plain FP64 oracle on the host
on a bounded sample of the same workload.

Workloads (all synthetic, seeded):
  droplet1024   1024 x 1024 periodic, Peng-Robinson (a=2/49, b=2/21, R=1,
                omega=0.344), one centred droplet of radius 128 (tanh, width 2,
                +-0.5 % noise), improved forcing sigma = 0.105, tau = 1.0
  droplets4096  4096 x 4096 periodic, Carnahan-Starling at 0.7 Tc, tau = 0.8,
                improved sigma = 0.1, 64 droplets of radius U[40, 120]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_LUP = {0: 144, 1: 72, 2: 36}     # 2 x 9 populations x storage bytes
PREC_NAME = {0: "f64", 1: "f32dev", 2: "f16dev"}


def workload(name: str, t_over_tc: float | None):
    import synth
    from paper_1204_4098_amd import lbm
    if name == "droplet1024":
        eos = dict(eos=lbm.LBM_EOS_PR, a=2 / 49, b=2 / 21, R=1.0, omega=0.344)
        t = 0.6 if t_over_tc is None else t_over_tc
        Tc, _ = lbm.lbm_critical_point(**{k: eos[k] for k in ("eos", "a", "b", "R", "omega")})
        rl, rg, _ = lbm.lbm_maxwell(eos["eos"], eos["a"], eos["b"], eos["R"], eos["omega"], t * Tc)
        nx = ny = 1024
        rho0 = synth.droplet(nx, ny, rl, rg, 128.0, 2.0, 0.005, synth.BASE_SEED)
        cfg = dict(workload="droplet1024", nx=nx, ny=ny, eos="peng-robinson", t_over_tc=t,
                   tau=1.0, scheme="improved", sigma=0.105, init="droplet r=128")
        kw = dict(tau=1.0, scheme=lbm.LBM_SCHEME_IMPROVED, sigma=0.105, T=t * Tc, **eos)
        return nx, ny, rho0, kw, cfg
    if name == "droplets4096":
        t = 0.7 if t_over_tc is None else t_over_tc
        Tc, _ = lbm.lbm_critical_point(lbm.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0)
        rl, rg, _ = lbm.lbm_maxwell(lbm.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0, t * Tc)
        nx = ny = 4096
        centers, radii = synth.droplet_layout(nx, ny, 64, 40.0, 120.0, 16.0, synth.BASE_SEED)
        rho0 = synth.droplets(nx, ny, rl, rg, centers, radii, 2.0, 0.005, synth.BASE_SEED)
        cfg = dict(workload="droplets4096", nx=nx, ny=ny, eos="carnahan-starling", t_over_tc=t,
                   tau=0.8, scheme="improved", sigma=0.1, init="64 droplets r~U[40,120]")
        kw = dict(tau=0.8, scheme=lbm.LBM_SCHEME_IMPROVED, sigma=0.1, T=t * Tc, eos=lbm.LBM_EOS_CS,
                  a=1.0, b=4.0, R=1.0, omega=0.0)
        return nx, ny, rho0, kw, cfg
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(kw, rho0, sample_n=256, steps=None, budget_s=15.0):
    """Time the FP64 oracle (single thread) on a sample_n^2 crop of the workload."""
    import numpy as np

    from oracle import lbm as olbm
    from oracle import thermo as th
    ny, nx = rho0.shape
    cy, cx = ny // 2, nx // 2
    h = sample_n // 2
    crop = np.ascontiguousarray(rho0[cy - h:cy + h, cx - h:cx + h])
    Tc = th.critical_pr()[0] if kw["eos"] == 1 else th.critical_cs()[0]
    op = olbm.Params(nx=sample_n, ny=sample_n, tau=kw["tau"], G=-1.0, eos=kw["eos"], a=kw["a"],
                     b=kw["b"], R=kw["R"], T=kw["T"], omega=kw["omega"], Tc=Tc,
                     scheme=kw["scheme"], sigma=kw["sigma"])
    f = olbm.init_equilibrium(crop)
    t0 = time.perf_counter()
    olbm.step(op, f, 2)
    per = (time.perf_counter() - t0) / 2
    if steps is None:
        steps = max(2, int(budget_s / per))
    t0 = time.perf_counter()
    olbm.step(op, f, steps)
    el = time.perf_counter() - t0
    return {"value": round(sample_n * sample_n * steps / el / 1e6, 3), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_n}x{sample_n} centre crop of the same workload, {steps} steps, "
                      f"FP64 C oracle, one thread, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="droplet1024", choices=["droplet1024", "droplets4096"])
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--t-over-tc", type=float, default=None)
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1204_4098_amd import lbm

    nx, ny, rho0, kw, cfg = workload(args.workload, args.t_over_tc)
    p = lbm.params(nx, ny, precision=args.precision, **kw)
    lat = lbm.Lattice(p, rho0, device="cuda:0")
    if not args.no_tune:
        lat.tune()
    waves, rows, depth = lat.get_tile()
    if args.graph_steps:
        lat.set_graph_steps(args.graph_steps)
    lat.step(args.warmup)
    st, _, div = lat.status()
    if st != lbm.LBM_OK:
        raise SystemExit(f"bench: the run diverged at step {div} during warm-up; timing would be invalid")

    stream = lat.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, nsteps, div = lat.status()
    if st != lbm.LBM_OK:
        raise SystemExit(f"bench: the run diverged at step {div} inside the timed region; "
                         "the measurement is invalid")
    wall = t1 - t0
    kern_ms = e0.elapsed_time(e1) / args.steps        # average per step launch on the stream
    nodes = nx * ny
    mlups = nodes * args.steps / wall / 1e6
    bpl = BYTES_PER_LUP[args.precision]
    achieved = bpl * nodes / (kern_ms * 1e-3) / 1e9
    out = {
        "metric": "D2Q9 MLUPS & %HBM roofline; batched FP32 vs plain FP64 at <=1e-4 density err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_NAME[args.precision],
        "data": "synthetic",
        "config": dict(cfg, precision=PREC_NAME[args.precision], tile_waves=waves, tile_rows=rows, tile_depth=depth,
                       graph_steps=args.graph_steps),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "k_step", "bytes_per_lup": bpl,
                     "kernel_avg_us": round(kern_ms * 1e3, 2)},
    }
    lat.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(kw, rho0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
