"""Benchmark of the implicit chemical-kinetics update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--quick]

Workload (the headline): the 9-species/38-reaction synthetic mechanism on a 1024 x 1024 grid
(2^20 cells, shock-heated band temperature field), advanced K steps of dt = 1e-6 s (default
K = 10), state resident in HBM.  A "step" advances every cell by one dt through the whole
hot path (rates, equilibrium constants, Jacobian, LU, Newton, sub-step halving, temperature
inversion).  It is timed for the plain FP64 form (the reported value) and for the FP32-LU
form; the 36-species/308-reaction mechanism on 2^18 cells (one step) is timed beside it.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def device_state(torch, st):
    d = dict(rho=torch.from_numpy(st.rho).cuda(), T=torch.from_numpy(st.T).cuda(),
             Y=torch.from_numpy(st.Y).cuda())
    return d


def time_steps(torch, ctx, kin, iid, state, dt, prec, steps, warmup, stream):
    """Warm up, reset to the input state, then time `steps` advance calls with HIP events on
    the launch stream.  Returns (total_s, per-launch seconds)."""
    for _ in range(warmup):
        ctx.advance([iid], [dt], prec=prec, stream=stream)
    ctx.state_reset(iid, state["rho"], state["T"], state["Y"], stream=stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    with torch.cuda.stream(stream):
        ev[0].record(stream)
        for k in range(steps):
            ctx.advance([iid], [dt], prec=prec, stream=stream)
            ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) * 1e-3 for k in range(steps)]
    return sum(per), per


def replay_stats(torch, ctx, iid, state, dt, prec, steps, stream):
    """Untimed replay of the same steps collecting per-step diagnostics."""
    ctx.state_reset(iid, state["rho"], state["T"], state["Y"], stream=stream)
    its, st_hist, lv_max = [], np.zeros(4, np.int64), 0
    out = None
    for _ in range(steps):
        ctx.advance([iid], [dt], prec=prec, stream=stream)
        torch.cuda.synchronize()
        out = ctx.download(iid)
        its.append(int(out[4].astype(np.int64).sum()))
        st_hist += np.bincount(out[2], minlength=4)[:4]
        lv_max = max(lv_max, int(out[3].max()))
    return its, st_hist, lv_max, out


def run_gpu(args):
    import torch
    from paper_1110_4903_amd import flops, kin, synth

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = kin.Context(0)
    res = {}

    # ---- headline: mech9 on the 1024x1024 band grid, K steps ------------------------------
    nx = 256 if args.quick else 1024
    m9, grid, dt9 = synth.workload_grid_mech9(nx, nx)
    t0 = time.time()
    mid9 = ctx.mech_upload(m9)
    jit9 = time.time() - t0
    st9 = device_state(torch, grid)
    iid9 = ctx.state_upload(mid9, st9["rho"], st9["T"], st9["Y"], stream=stream)
    torch.cuda.synchronize()
    f9 = flops.newton_iteration_flops(m9)["total"]
    for name, prec in (("fp64", kin.FP64), ("fp32lu", kin.FP32_LU)):
        tot, per = time_steps(torch, ctx, kin, iid9, st9, dt9, prec, args.steps, args.warmup, stream)
        its, hist, lvmax, _ = replay_stats(torch, ctx, iid9, st9, dt9, prec, args.steps, stream)
        achieved = [f9 * it / p / 1e12 for it, p in zip(its, per)]
        res[f"mech9_{name}"] = dict(
            cells=grid.n, steps=args.steps, seconds=tot, cells_per_s=grid.n * args.steps / tot,
            kernel_ms_avg=1e3 * float(np.mean(per)), newton_iters_per_cell=float(np.sum(its)) / (grid.n * args.steps),
            status_hist=hist.tolist(), max_level=lvmax, tflops_model=float(np.mean(achieved)))
    res["mech9_jit_s"] = jit9
    ctx.instance_release(iid9)

    # ---- mech36, 2^18 cells, one step ------------------------------------------------------
    n36 = (1 << 14) if args.quick else (1 << 18)
    m36, s36, dt36 = synth.workload_mech36(n36)
    mid36 = ctx.mech_upload(m36)
    st36 = device_state(torch, s36)
    iid36 = ctx.state_upload(mid36, st36["rho"], st36["T"], st36["Y"], stream=stream)
    f36 = flops.newton_iteration_flops(m36)["total"]
    steps36 = 1
    for name, prec in (("fp64", kin.FP64), ("fp32lu", kin.FP32_LU)):
        tot, per = time_steps(torch, ctx, kin, iid36, st36, dt36, prec, steps36, 1, stream)
        its, hist, lvmax, _ = replay_stats(torch, ctx, iid36, st36, dt36, prec, steps36, stream)
        res[f"mech36_{name}"] = dict(
            cells=n36, steps=steps36, seconds=tot, cells_per_s=n36 * steps36 / tot,
            kernel_ms_avg=1e3 * float(np.mean(per)), newton_iters_per_cell=float(np.sum(its)) / (n36 * steps36),
            status_hist=hist.tolist(), max_level=lvmax, tflops_model=f36 * its[0] / per[0] / 1e12)
    ctx.close()
    return res, grid, m9, dt9


def cpu_baseline(grid, m9, dt9, steps, sample_stride):
    """The FP64 oracle on the host cores over a strided sample of the headline grid."""
    from oracle import oracle
    om = oracle.OracleMech(m9)
    idx = np.arange(0, grid.n, sample_stride)
    sub = grid.subset(idx)
    e0 = om.energy_batch(sub.T, sub.Y)
    T, Y = sub.T.copy(), sub.Y.copy()
    t0 = time.time()
    for _ in range(steps):
        T, Y, _, _, _ = om.advance(sub.rho, T, Y, dt9, e0=e0)
    el = time.time() - t0
    return dict(value=idx.shape[0] * steps / el, unit="cells/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{idx.shape[0]} cells (every {sample_stride}th of the 1024x1024 grid) x {steps} steps "
                       f"of dt=1e-6 s, FP64, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="small grid, for smoke runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the per-cell kinetics update has "
                                   "no cross-GPU exchange (cells shard trivially), so --gpus must be 1"}))
        sys.exit(2)
    res, grid, m9, dt9 = run_gpu(args)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(grid, m9, dt9, args.steps, 16 if not args.quick else 4)
    h = res["mech9_fp64"]
    line = {
        "metric": "cells/s advanced one dt (9-sp & 36-sp), FP32-LU vs FP64 at stated err; p99 latency",
        "value": h["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * h["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mech9 (9 species, 38 reactions) on a {int(np.sqrt(grid.n))}x{int(np.sqrt(grid.n))} "
                               f"band grid, {args.steps} steps of dt=1e-6 s, FP64 form, state resident in HBM",
                   "cells": grid.n, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": h["tflops_model"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": h["tflops_model"] / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "kin_lane_f64"},
        "cpu_baseline": cpu,
        "forms": res,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
