#!/usr/bin/env python3
"""Benchmark of the fused pseudopotential D2Q9 step on one MI355X.

Prints ONE JSON line.  `value` is whole-job MLUPS (million lattice-node
updates per second) of the plain FP64 fused step on the configured lattice,
timed with inputs resident in HBM.  `roofline` reports the step kernel's
algorithmic HBM traffic (9 populations read + 9 written per node) against the
8 TB/s MI355X peak, with the kernel time measured by HIP events on the stream
the kernel runs on.  `cpu_baseline` times the plain FP64 oracle on the host
on a bounded sample of the same workload.

Further legs (same line): `batched` -- 256 uneven flat-interface runs in one
persistent launch per step, FP32 deviations versus the same runs through the
plain FP64 path, with the FP32-vs-FP64 coexistence-density error; `precision`
-- the default lattice with FP32 and FP16 deviation storage; `droplet1024` --
the 1024 x 1024 Peng-Robinson droplet.

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
BYTES_PER_LUP = {0: 144, 1: 72, 2: 36, 3: 72}     # 2 x 9 populations x storage bytes
PREC_NAME = {0: "f64", 1: "f32dev", 2: "f16dev", 3: "f32dev_f64arith"}


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


def cpu_pool_baseline(sample_runs=16, lups_per_run=3e7):
    """Multi-core oracle throughput on the batched workload: every (256 / sample_runs)-th
    of the 256 flat-interface runs (evenly spaced, so the size mix is kept),
    each advanced by the FP64 C oracle for about lups_per_run lattice updates,
    one run per task on a thread pool over the host cores (the oracle's C step
    releases the GIL).  Initial states are the runs' own slabs between the
    oracle's Maxwell densities."""
    from concurrent.futures import ThreadPoolExecutor

    import synth
    from oracle import lbm as olbm
    from oracle import thermo as th
    runs = synth.sweep_runs(256)
    pick = list(range(0, 256, 256 // sample_runs))[:sample_runs]
    Tc = th.critical_cs()[0]
    tasks = []
    for i in pick:
        r = runs[i]
        c = th.maxwell_cs(r["t_over_tc"])
        op = olbm.Params(nx=r["nx"], ny=r["ny"], tau=r["tau"], G=-1.0, eos=0, a=1.0, b=4.0, R=1.0,
                         T=r["t_over_tc"] * Tc, omega=0.0, Tc=Tc, scheme=olbm.SCHEME_IMPROVED,
                         sigma=r["sigma"])
        rho0 = synth.slab(r["nx"], r["ny"], float(c.rho_l), float(c.rho_g), r["nx"] / 4,
                          3 * r["nx"] / 4, 2.0, 0.01, synth.BASE_SEED, i)
        steps = max(1, round(lups_per_run / (r["nx"] * r["ny"])))
        tasks.append((op, olbm.init_equilibrium(rho0), steps))
    cores = min(16, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(lambda t: olbm.step(t[0], t[1], t[2]), tasks))
    el = time.perf_counter() - t0
    # a diverged run stops at its divergence step: count the updates done
    done = [t[2] if st == olbm.OK else max(0, dv) for t, (st, dv) in zip(tasks, res)]
    lups = sum(t[0].nx * t[0].ny * n for t, n in zip(tasks, done))
    ndiv = sum(st != olbm.OK for st, _ in res)
    return {"value": round(lups / el / 1e6, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{len(tasks)} of the 256 batched flat-interface runs (every "
                      f"{256 // sample_runs}th; {ndiv} diverged and stopped early), "
                      f"~{lups_per_run:.0e} lattice updates each, FP64 C oracle, one run per "
                      f"thread, {lups:.2e} updates in {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="droplets4096", choices=["droplet1024", "droplets4096"])
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1, 2, 3])
    ap.add_argument("--t-over-tc", type=float, default=None)
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="untimed stepping before the warm-up, so the timed steps see sustained clocks")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="batched,precision,droplet1024,slab64",
                    help="comma-separated extra legs, or 'none'")
    ap.add_argument("--batch-steps", type=int, default=30000,
                    help="steps of the batched FP32-vs-FP64 coexistence comparison")
    ap.add_argument("--tile", default=None,
                    help="waves,rows,depth[,steps]: fixed launch shape (no tuning); steps = time "
                         "steps per launch (1, or 2 for the two-step kernel)")
    ap.add_argument("--batch-case", default=None, choices=["f64", "f32", "f32dev", "f32_f64arith"],
                    help="time only this case of the batched leg (no plain-path timing, no "
                         "coexistence comparison): a short run for the counter profiles")
    ap.add_argument("--batch-tile", default=None,
                    help="waves,rows,depth,steps: fixed batch tile (no tuning)")
    ap.add_argument("--batch-time-steps", type=int, default=2000,
                    help="timed steps of each batched case")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a known-size kernel "
                         "for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1204_4098_amd import lbm

    if args.calibrate_copy:
        a = torch.ones(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    nx, ny, rho0, kw, cfg = workload(args.workload, args.t_over_tc)
    res = time_lattice(lbm, torch, nx, ny, rho0, kw, args.precision, args.steps, args.warmup,
                       args.graph_steps, not args.no_tune, tile, args.settle_ms)
    bpl = BYTES_PER_LUP[args.precision]
    ts = res["tile"][3]                      # time steps per launch of the step kernel
    launch_ms = res["kernel_ms"] * ts        # average duration of one launch
    # algorithmic bytes of one launch: every population read once and written once
    achieved = bpl * nx * ny / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": "D2Q9 MLUPS & %HBM roofline; batched FP32 vs plain FP64 at <=1e-4 density err",
        "value": round(res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["wall_s"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_NAME[args.precision],
        "data": "synthetic",
        "config": dict(cfg, precision=PREC_NAME[args.precision], tile=res["tile"],
                       graph_steps=res["graph_steps"], settle_ms=args.settle_ms),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_for(args.workload, args.precision, res["tile"]),
                     "kernel": {1: "k_step", 2: "k_step2", 3: "k_step3"}[ts], "steps_per_launch": ts,
                     "bytes_per_lup": bpl / ts, "kernel_avg_us": round(launch_ms * 1e3, 2),
                     # MLUPS x the single-step 144 B/LUP over the peak (exceeds 1 only
                     # when steps are fused; not a bandwidth)
                     "single_step_equivalent_frac": round(
                         bpl * nx * ny / (res["kernel_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
    }
    rf = out["roofline"]
    rf["copy_gbs"] = round(copy_rate(torch), 1)
    if rf["traffic"]:
        # HBM bytes the kernel actually moves per second, from the counter summary
        rf["traffic_gbs"] = round(rf["traffic"] / (launch_ms * 1e-3) / 1e9, 1)
    log(f"main leg done: {out['value']} MLUPS, {out['roofline']['frac']:.3f} of HBM peak")
    legs = [] if args.legs == "none" else args.legs.split(",")
    if "precision" in legs:
        out["precision"] = {}
        for prec in (1, 2, 3):
            r = time_lattice(lbm, torch, nx, ny, rho0, kw, prec, args.steps, args.warmup,
                             args.graph_steps, not args.no_tune, settle_ms=args.settle_ms)
            gbs = BYTES_PER_LUP[prec] * nx * ny / (r["kernel_ms"] * r["tile"][3] * 1e-3) / 1e9
            out["precision"][PREC_NAME[prec]] = {"mlups": round(r["mlups"], 1), "tile": r["tile"],
                                                 "achieved_gbs": round(gbs, 1),
                                                 "frac": round(gbs / PEAK_HBM_GBS, 4),
                                                 "bytes_per_lup": BYTES_PER_LUP[prec] / r["tile"][3]}
            log(f"precision {PREC_NAME[prec]}: {r['mlups']:.0f} MLUPS")
        # the FP64 one- and two-step kernels on the same workload, each with its own
        # roofline fraction (per launch: every population read and written once),
        # when the tuner has picked the three-step one
        for name, t1 in (("f64_one_step", (16, 0, 1, 1)), ("f64_two_step", (4, 0, 2, 2))):
            r = time_lattice(lbm, torch, nx, ny, rho0, kw, 0, args.steps, args.warmup,
                             args.graph_steps, False, t1, settle_ms=args.settle_ms)
            gbs = BYTES_PER_LUP[0] * nx * ny / (r["kernel_ms"] * t1[3] * 1e-3) / 1e9
            out["precision"][name] = {"mlups": round(r["mlups"], 1), "tile": r["tile"],
                                      "kernel_avg_us": round(r["kernel_ms"] * t1[3] * 1e3, 2),
                                      "achieved_gbs": round(gbs, 1),
                                      "frac": round(gbs / PEAK_HBM_GBS, 4),
                                      "traffic": traffic_for(args.workload, 0, r["tile"])}
            log(f"{name}: {r['mlups']:.0f} MLUPS, {gbs / PEAK_HBM_GBS:.3f} of HBM peak")
    if "droplet1024" in legs and args.workload != "droplet1024":
        d = {}
        for t in (0.6, 0.8):
            nx1, ny1, rho1, kw1, cfg1 = workload("droplet1024", t)
            for prec in (0, 1):
                try:
                    r = time_lattice(lbm, torch, nx1, ny1, rho1, kw1, prec, 2000, 50, args.graph_steps,
                                     not args.no_tune)
                    d[f"t{t}_{PREC_NAME[prec]}"] = {"mlups": round(r["mlups"], 1), "tile": r["tile"]}
                except Diverged as e:
                    d[f"t{t}_{PREC_NAME[prec]}"] = {"diverged_at_step": e.step}
        log(f"droplet1024 leg: {d}")
        out["droplet1024"] = dict(d, note="1024^2 Peng-Robinson droplet r=128, tau=1, improved "
                                          "sigma=0.105; at 0.6 Tc the run leaves the EOS range")
    if "slab64" in legs:
        out["slab64"] = slab64_leg(lbm, torch)
        log(f"slab64 leg: {out['slab64']}")
    if "batched" in legs:
        btile = tuple(int(v) for v in args.batch_tile.split(",")) if args.batch_tile else None
        out["batched"] = batched_leg(lbm, torch, args.batch_steps, args.graph_steps, args.batch_case,
                                     btile, args.batch_time_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(kw, rho0)
        if "batched" in legs:
            out["cpu_baseline"]["batched_pool"] = cpu_pool_baseline()
            log(f"cpu pool oracle on batched runs: {out['cpu_baseline']['batched_pool']['value']} "
                f"MLUPS on {out['cpu_baseline']['batched_pool']['cores']} cores")
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


class Diverged(RuntimeError):
    def __init__(self, step):
        super().__init__(f"diverged at step {step}")
        self.step = step


def settle(lat, torch, ms):
    """Step the lattice untimed for about `ms` milliseconds of GPU time, so that the
    timed steps run at the GPU's sustained clocks: a kernel trace of the FP64 droplet
    workload shows launches 4-12 after a start from idle running up to 33 % slower
    (528 -> 698 us per launch) and recovering only after ~40 launches (~520 us)."""
    if ms <= 0:
        return
    t0 = time.perf_counter()
    n = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        lat.step(20)
        torch.cuda.synchronize()
        n += 20
    return n


def time_lattice(lbm, torch, nx, ny, rho0, kw, precision, steps, warmup, graph_steps, tune, tile=None,
                 settle_ms=100.0):
    """Settle, tune, capture, settle again, warm up, then time `steps` steps between a
    device sync on both sides.  Settling before the autotuner lets it compare tiles
    at sustained clocks; settling again after the graph capture (host work that
    leaves the GPU idle) restores them for the timed steps.  None of these steps
    is timed; all of them advance the state."""
    p = lbm.params(nx, ny, precision=precision, **kw)
    lat = lbm.Lattice(p, rho0, device="cuda:0")
    settle(lat, torch, settle_ms)
    if tile:
        lat.set_tile(*tile)
    elif tune:
        lat.tune()
    tile = list(lat.get_tile())
    ts = tile[3]
    # a graph holds whole launches of the tile: its length is rounded down to a
    # multiple of the tile's steps (and of 2)
    g = graph_steps - graph_steps % (6 if ts == 3 else 2) if graph_steps else 0
    if g:
        lat.set_graph_steps(g)   # captures and uploads the graphs of both parities now
    settle(lat, torch, settle_ms)
    lat.step(warmup)
    st, _, div = lat.status()
    if st != lbm.LBM_OK:
        lat.close()
        raise Diverged(div)
    # the kernel average is taken over the whole launches of the tile; a
    # remainder of fewer steps (one shorter launch) is timed after them
    n_main = steps - steps % ts
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    captures = lat.graph_captures()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(lat.stream)
    lat.step(n_main)
    e1.record(lat.stream)
    lat.step(steps - n_main)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if lat.graph_captures() != captures:
        raise RuntimeError("a graph was captured inside the timed window")
    st, _, div = lat.status()
    lat.close()
    if st != lbm.LBM_OK:
        raise Diverged(div)
    return {"mlups": nx * ny * steps / wall / 1e6, "wall_s": wall,
            "kernel_ms": e0.elapsed_time(e1) / max(n_main, 1), "tile": tile, "graph_steps": g}


def copy_rate(torch, mib=1024, reps=5):
    """GB/s of a device-to-device copy of `mib` MiB (torch's copy, read plus written
    bytes over the HIP-event time of `reps` copies): the bandwidth a plain streaming
    kernel gets from HBM in the same process, next to the nominal 8 TB/s."""
    a = torch.zeros(mib << 20, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    return 2 * (mib << 20) * reps / (ms * 1e-3) / 1e9


def traffic_for(workload, precision, tile):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    workload, precision and tile (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy's readings), or None when no summary matches."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        table = json.load(open(path))
    except (OSError, ValueError):
        return None
    key = f"{workload}/{PREC_NAME[precision]}/{tile[0]}x{tile[1]}x{tile[2]}"
    if len(tile) > 3 and tile[3] != 1:
        key += f"x{tile[3]}steps"
    e = table.get("entries", {}).get(key)
    return None if e is None else e.get("bytes_per_launch")


def slab64_leg(lbm, torch, steps=10000):
    """The 64 x 32 flat interface (C-S 0.8 Tc, tau = 1, improved sigma = 0.1), 10,000
    steps: a launch-bound lattice of 0.3 MB per step, timed as eager launches and as
    replays of captured graphs of 100 steps, with the tuned tile."""
    import synth
    Tc, _ = lbm.lbm_critical_point(lbm.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0)
    rl, rg, _ = lbm.lbm_maxwell(lbm.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0, 0.8 * Tc)
    rho0 = synth.slab(64, 32, rl, rg, 16, 48, 2.0, 0.01, synth.BASE_SEED)
    p = lbm.params(64, 32, tau=1.0, T=0.8 * Tc, scheme=lbm.LBM_SCHEME_IMPROVED, sigma=0.1,
                   eos=lbm.LBM_EOS_CS, a=1.0, b=4.0, R=1.0, omega=0.0)
    res = {}
    for name, k in (("eager", 0), ("graph100", 100)):
        lat = lbm.Lattice(p, rho0, device="cuda:0")
        lat.tune()
        if k:
            lat.set_graph_steps(k)
        lat.step(200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[f"{name}_us_per_step"] = round(wall / steps * 1e6, 3)
        res[f"{name}_tile"] = list(lat.get_tile())
        lat.close()
    return res


def batched_leg(lbm, torch, batch_steps, graph_steps, only=None, tile=None, time_steps=2000):
    """256 uneven flat-interface runs (Lx in 64..512 step 32, Ly in 16..64 step 16,
    T/Tc in [0.5, 0.95], tau in [0.6, 1.5], sigma in [0, 0.2], C-S): one persistent
    launch per step (tuned tile) in FP64 and in three FP32-storage forms, and the FP64
    runs through the plain path (one context per run, run after run).

    FP32 forms: `f32` -- plain FP32 populations (rho_ref = 0) with FP32 collision
    arithmetic, the headline; `f32dev` -- FP32 deviations from the mean density with
    FP32 arithmetic; `f32_f64arith` -- plain FP32 populations with FP64 collision
    arithmetic.  In both FP32-arithmetic forms the node's mass and momentum change
    are restored in FP64 after the collision.  The headline ratio is `f32` batched
    over FP64 batched; the ratio over the plain FP64 path is reported beside it.
    Coexistence densities after batch_steps steps are averaged over the last 4000.
    `only` restricts the leg to the timing of one case (with `tile` fixed, if given,
    and `time_steps` timed steps), for short profiled runs."""
    import numpy as np

    import synth
    from paper_1204_4098_amd import surrogate
    runs = synth.sweep_runs(256)
    nodes = sum(r["nx"] * r["ny"] for r in runs)
    res = {"runs": 256, "nodes": nodes, "coexistence_steps": batch_steps}
    cases = {"f64": (0, float("nan")), "f32": (1, 0.0), "f32dev": (1, float("nan")),
             "f32_f64arith": (3, 0.0)}
    for name, (prec, rr) in cases.items():
        if only and name != only:
            continue
        ps, rhos = surrogate.slab_runs(runs, prec, rho_ref=rr)
        b = lbm.Batch(ps, rhos)
        if tile:
            b.set_tile(*tile)
        else:
            b.tune()
        if graph_steps:
            b.set_graph_steps(100)
        b.step(200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(time_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[f"{name}_batched_mlups"] = round(nodes * time_steps / wall / 1e6, 1)
        res[f"{name}_batched_tile"] = list(b.get_tile())
        b.close()
        log(f"batched {name}: {res[f'{name}_batched_mlups']} MLUPS")
    if only:
        return res
    # the plain FP64 path: one lattice context per run, each stepped in turn
    ps, rhos = surrogate.slab_runs(runs, 0)
    lats = [lbm.Lattice(p, r) for p, r in zip(ps, rhos)]
    for lat in lats:
        lat.set_graph_steps(20)
        lat.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(200)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    res["f64_plain_mlups"] = round(nodes * 200 / wall / 1e6, 1)
    log(f"plain FP64 path: {res['f64_plain_mlups']} MLUPS")
    for name in ("f32", "f32dev", "f32_f64arith"):
        res[f"ratio_{name}_batched_vs_f64_batched"] = round(
            res[f"{name}_batched_mlups"] / res["f64_batched_mlups"], 2)
        res[f"ratio_{name}_batched_vs_f64_plain"] = round(
            res[f"{name}_batched_mlups"] / res["f64_plain_mlups"], 2)
    out = {n: surrogate.run_batch(runs, batch_steps, prec, window=4000, samples=20, rho_ref=rr)
           for n, (prec, rr) in cases.items()}
    ref = out["f64"]
    res["diverged_f64"] = int(np.sum(ref["status"] != 0))
    for n in ("f32", "f32dev", "f32_f64arith"):
        o = out[n]
        ok = (ref["status"] == 0) & (o["status"] == 0)
        err = np.maximum(np.abs(o["rho_l"][ok] / ref["rho_l"][ok] - 1), np.abs(o["rho_g"][ok] / ref["rho_g"][ok] - 1))
        res[f"{n}_diverged"] = int(np.sum(o["status"] != 0))
        res[f"{n}_coex_rel_err_median"] = float(np.median(err))
        res[f"{n}_coex_rel_err_p90"] = float(np.quantile(err, 0.9))
        res[f"{n}_coex_rel_err_max"] = float(err.max())
        res[f"{n}_runs_within_1e-4"] = f"{int(np.sum(err <= 1e-4))}/{int(ok.sum())}"
        log(f"coexistence {n}: median {res[f'{n}_coex_rel_err_median']:.2e}, within 1e-4 "
            f"{res[f'{n}_runs_within_1e-4']}")
    return res


if __name__ == "__main__":
    main()
