"""Benchmark of the implicit chemical-kinetics update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--quick]
                    [--no-batch] [--no-serve] [--serve-requests R]

Headline (the reported value): the 9-species / 38-reaction synthetic mechanism on a 1024 x 1024
grid (2^20 cells, shock-heated band temperature field), advanced K steps of dt = 1e-6 s
(default K = 20, after W = 5 warm-up steps) with the state resident in HBM, plain FP64 form.
A "step" advances every cell by one dt through the whole hot path: rates, equilibrium
constants, third-body sums, analytic Jacobian, partially pivoted LU of I - hJ, Newton
iteration, sub-step halving and the temperature inversion.  Also measured and reported under "forms":
  * the same grid in the FP32-LU form, with its deviation from the FP64 form;
  * the 36-species / 308-reaction mechanism on 2^18 cells, one step, both forms;
  * an uneven batch of 64 instances of both mechanisms (log-uniform 1024..262144 cells, dt
    uniform in [1e-7, 1e-5] s) advanced in one graph launch in the FP32-LU form after the
    autotuner has chosen each mechanism's layout, against 64 separate launches;
  * the serving loop: Poisson arrivals at 0.5, 0.8 and 0.95 of the measured saturated rate,
    log-normal request sizes (median 16384 cells), 70/30 mix of the two mechanisms, admission
    by HBM footprint under a 256 MiB budget, 36-species requests confined to all but 32
    compute units, p50/p99 latency from arrival to results in host memory;
  * the paper's point-implicit step (one linearised backward-Euler step per dt) for both
    mechanisms, with its difference from the iterated method.
The FP64 CPU oracle is timed on a strided sample of the headline grid on the host cores.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "traffic_kin_lane_f64_mech9_grid1024.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def device_state(torch, st):
    return dict(rho=torch.from_numpy(st.rho).cuda(), T=torch.from_numpy(st.T).cuda(),
                Y=torch.from_numpy(st.Y).cuda())


def time_steps(torch, ctx, iid, state, dt, prec, steps, warmup, stream, opts=None):
    """Warm up, reset to the input state, then time `steps` advance calls with events recorded on
    the launch stream.  Returns (total_s, per-advance seconds, per-launch seconds of the advance
    kernel alone).  The latter come from the events the library records on the launch stream
    right around its advance kernel (the context is created with kernel timing on); an advance's
    own time also holds the work-counter clear and, for a cost-ordered step, the ordering
    kernels."""
    for _ in range(warmup):
        ctx.advance([iid], [dt], prec=prec, stream=stream, opts=opts)
    ctx.state_reset(iid, state["rho"], state["T"], state["Y"], stream=stream)
    torch.cuda.synchronize()
    ctx.kernel_times()  # drop the warm-up's records
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        ctx.advance([iid], [dt], prec=prec, stream=stream, opts=opts)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) * 1e-3 for k in range(steps)]
    kern = [1e-3 * t for t in ctx.kernel_times()]
    assert len(kern) == steps, (len(kern), steps)
    return sum(per), per, kern


def replay_stats(torch, ctx, iid, state, dt, prec, steps, stream, opts=None):
    """Untimed replay of the same steps collecting per-step diagnostics (the kernels are
    deterministic, so the replay takes the same iterations as the timed run)."""
    ctx.state_reset(iid, state["rho"], state["T"], state["Y"], stream=stream)
    its, st_hist, lv_max = [], np.zeros(4, np.int64), 0
    out = None
    for _ in range(steps):
        ctx.advance([iid], [dt], prec=prec, stream=stream, opts=opts)
        torch.cuda.synchronize()
        out = ctx.download(iid) + (ctx.download_schedule(iid),)
        its.append(int(out[4].astype(np.int64).sum()))
        st_hist += np.bincount(out[2], minlength=4)[:4]
        lv_max = max(lv_max, int(out[3].max()))
    return its, st_hist, lv_max, out


def form_stats(n, steps, tot, per, kern, its, hist, lvmax, flops_per_iter):
    """Throughput of a form, and the advance kernel's achieved rate: the flop model's flops per
    Newton iteration times the iterations of all timed launches, over the kernel's total time
    (total over total, not a mean of per-launch rates)."""
    return dict(cells=n, steps=steps, seconds=tot, cells_per_s=n * steps / tot,
                advance_ms_avg=1e3 * float(np.mean(per)), kernel_ms_avg=1e3 * float(np.mean(kern)),
                kernel_ms=[1e3 * k for k in kern], newton_iters=[int(i) for i in its],
                newton_iters_per_cell=float(np.sum(its)) / (n * steps),
                status_hist=hist.tolist(), max_level=lvmax,
                tflops_model=flops_per_iter * float(np.sum(its)) / float(np.sum(kern)) / 1e12)


def method_difference(a, b):
    """Relative difference between two methods' one-step results on cells both accepted."""
    ok = (a[2] < 2) & (b[2] < 2)
    Ya, Yb = a[1][:, ok], b[1][:, ok]
    big = np.abs(Ya) >= 1e-6
    rel = np.where(big, np.abs(Yb - Ya) / np.maximum(np.abs(Ya), 1e-300), 0.0)
    relT = np.abs(b[0][ok] - a[0][ok]) / a[0][ok]
    return {"both_accepted": int(ok.sum()), "failed_in_b": int((b[2] == 2).sum()),
            "max_rel_Y_where_Y_ge_1e-6": float(rel.max()) if rel.size else 0.0,
            "median_rel_Y_where_Y_ge_1e-6": float(np.median(rel[big])) if big.any() else 0.0,
            "max_rel_T": float(relT.max()) if relT.size else 0.0}


def point_implicit_form(torch, ctx, kin, iid, st, dt, steps, n, flops_per_iter, newton_one_step, stream):
    """The paper's point-implicit step (one linearised backward-Euler step per dt), FP64."""
    o = kin.solver_opts(point_implicit=1)
    tot, per, kern = time_steps(torch, ctx, iid, st, dt, kin.FP64, steps, 1, stream, opts=o)
    its, hist, lvmax, _ = replay_stats(torch, ctx, iid, st, dt, kin.FP64, steps, stream, opts=o)
    ctx.kernel_times()
    r = form_stats(n, steps, tot, per, kern, its, hist, lvmax, flops_per_iter)
    one = replay_stats(torch, ctx, iid, st, dt, kin.FP64, 1, stream, opts=o)[3]
    r["difference_from_newton_be_one_step"] = method_difference(newton_one_step, one)
    return r


def deviation(a, b):
    """Relative deviation of form b from form a over cells whose status, level and sub-step
    schedule agree (the others took different step sizes and are counted)."""
    same = (a[2] == b[2]) & (a[3] == b[3]) & (a[5] == b[5]) & (a[2] < 2)
    Ya, Yb = a[1][:, same], b[1][:, same]
    big = np.abs(Ya) >= 1e-14
    rel = np.where(big, np.abs(Yb - Ya) / np.maximum(np.abs(Ya), 1e-300), 0.0)
    relT = np.abs(b[0][same] - a[0][same]) / a[0][same]
    return dict(compared=int(same.sum()), schedule_differs=int((~same).sum()),
                max_rel_Y=float(rel.max()) if rel.size else 0.0,
                max_rel_T=float(relT.max()) if relT.size else 0.0)


def run_headline(torch, ctx, kin, flops, synth, args, stream):
    nx = 256 if args.quick else 1024
    m9, grid, dt9 = synth.workload_grid_mech9(nx, nx)
    t0 = time.time()
    mid9 = ctx.mech_upload(m9)
    jit9 = time.time() - t0
    st9 = device_state(torch, grid)
    iid9 = ctx.state_upload(mid9, st9["rho"], st9["T"], st9["Y"], stream=stream)
    torch.cuda.synchronize()
    f9 = flops.newton_iteration_flops(m9)["total"]
    res, outs, traces = {}, {}, {}
    forms = (("fp64", kin.FP64), ("fp32lu", kin.FP32_LU))
    for name, prec in forms:
        log(f"mech9 grid {nx}x{nx}, {args.steps} steps, {name}")
        tot, per, kern = time_steps(torch, ctx, iid9, st9, dt9, prec, args.steps, args.warmup, stream)
        its, hist, lvmax, _ = replay_stats(torch, ctx, iid9, st9, dt9, prec, args.steps, stream)
        res[f"mech9_{name}"] = form_stats(grid.n, args.steps, tot, per, kern, its, hist, lvmax, f9)
        # one step from the input state, for the deviation between the forms; then the same step
        # with the schedule recorder, for the comparison with the oracle (cpu_baseline)
        outs[name] = replay_stats(torch, ctx, iid9, st9, dt9, prec, 1, stream)[3]
        if args.only == "all" and not args.no_cpu:
            ctx.state_reset(iid9, st9["rho"], st9["T"], st9["Y"], stream=stream)
            traces[name] = ctx.advance_trace(iid9, dt9, prec, words=16)
            again = ctx.download(iid9) + (ctx.download_schedule(iid9),)
            assert all(np.array_equal(a, b, equal_nan=True) for a, b in zip(again, outs[name]))
        ctx.kernel_times()
    res["mech9_fp32lu"]["deviation_from_fp64_one_step"] = deviation(outs["fp64"], outs["fp32lu"])
    if args.only == "all":
        log(f"mech9 grid {nx}x{nx}, {args.steps} steps, point-implicit")
        res["mech9_point_implicit_fp64"] = point_implicit_form(torch, ctx, kin, iid9, st9, dt9, args.steps, grid.n,
                                                               f9, outs["fp64"], stream)
    res["mech9_jit_s"] = jit9
    res["mech9_layout"] = [ctx.query_int(kin.Q_LAYOUT, mid9), ctx.query_int(kin.Q_BLOCK, mid9)]
    ctx.instance_release(iid9)
    ctx.mech_release(mid9)
    return res, grid, m9, dt9, dict(outs=outs, traces=traces)


def run_config0_end_to_end(torch, ctx, kin, synth, stream):
    """4096 cells of the 9-species mechanism (the small parity input) with host buffers at the
    boundary: reset from host memory, advance one dt, download to host memory, wall time per
    round over 20 rounds (PCIe-inclusive; not the reported value)."""
    m, st, dt = synth.workload_small_mech9()
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload(mid, st.rho, st.T, st.Y)
    T = np.empty(st.n)
    Y = np.empty((m.ns, st.n))
    for _ in range(2):
        ctx.state_reset(iid, st.rho, st.T, st.Y)
        ctx.advance([iid], [dt])
        ctx.download(iid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        ctx.state_reset(iid, st.rho, st.T, st.Y)
        ctx.advance([iid], [dt])
        T, Y = ctx.download(iid)[:2]
    el = time.perf_counter() - t0
    ctx.instance_release(iid)
    ctx.mech_release(mid)
    return dict(cells=st.n, rounds=reps, seconds=el, cells_per_s=st.n * reps / el,
                ms_per_round=1e3 * el / reps)


def run_conserved_adapter(torch, ctx, kin, synth, args, stream):
    """The chemistry sub-step of the operator split on the headline grid, FP64: partial
    densities and sensible energy in (device buffers), advance one dt, partial densities and
    sensible energy out.  The conserved input is made by the library itself from the grid's
    state.  Reports the time of the two conversions beside the advance."""
    nx = 256 if args.quick else 1024
    m, grid, dt = synth.workload_grid_mech9(nx, nx)
    mid = ctx.mech_upload(m)
    st = device_state(torch, grid)
    iid = ctx.state_upload(mid, st["rho"], st["T"], st["Y"], stream=stream)
    rho_s = torch.empty((m.ns, grid.n), dtype=torch.float64, device="cuda")
    E = torch.empty(grid.n, dtype=torch.float64, device="cuda")
    ctx.download_conserved_device(iid, rho_s, E, stream=stream)
    out_s = torch.empty_like(rho_s)
    out_E = torch.empty_like(E)
    for _ in range(2):
        ctx.state_reset_conserved(iid, rho_s, E, stream=stream)
        ctx.advance([iid], [dt], stream=stream)
        ctx.download_conserved_device(iid, out_s, out_E, stream=stream)
    torch.cuda.synchronize()
    steps = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        ctx.state_reset_conserved(iid, rho_s, E, stream=stream)
        ev[3 * k + 1].record(stream)
        ctx.advance([iid], [dt], stream=stream)
        ev[3 * k + 2].record(stream)
        ctx.download_conserved_device(iid, out_s, out_E, stream=stream)
        ev[3 * k + 3].record(stream)
    torch.cuda.synchronize()
    t_in = sum(ev[3 * k].elapsed_time(ev[3 * k + 1]) for k in range(steps)) / steps
    t_adv = sum(ev[3 * k + 1].elapsed_time(ev[3 * k + 2]) for k in range(steps)) / steps
    t_out = sum(ev[3 * k + 2].elapsed_time(ev[3 * k + 3]) for k in range(steps)) / steps
    total = t_in + t_adv + t_out
    ctx.instance_release(iid)
    ctx.mech_release(mid)
    return dict(cells=grid.n, steps=steps, ms_conserved_in=t_in, ms_advance=t_adv,
                ms_conserved_out=t_out, cells_per_s=grid.n / (total * 1e-3),
                adapter_share=(t_in + t_out) / total)


def run_global_tier(torch, ctx, kin, flops, synth, args, stream):
    """The global-memory layout (one wavefront per cell, the cell's matrix in HBM, as in the
    paper's first kinetics kernel) on a generated 100-species / 600-reaction mechanism, beyond the
    wave layout's 63 species: one FP64 step of 1e-6 s on 65536 cells (Dirichlet(0.5), seed 7).
    Achieved bandwidth = the algorithmic bytes of a Newton iteration (flops.global_tier_bytes)
    times the iterations of the launch, over its duration."""
    n = 4096 if args.quick else 65536
    m = synth.make_mechanism(synth.MechRecipe("gen100", seed=1100, n_elements=5, n_species=100,
                                              n_reactions=600, frac_third_body=0.15,
                                              frac_irreversible=0.3))
    mid = ctx.mech_upload(m)
    st = device_state(torch, synth.uniform_cells(7, n, m.ns, 0.5))
    warm = device_state(torch, synth.uniform_cells(8, 1024, m.ns, 0.5))
    wid = ctx.state_upload(mid, warm["rho"], warm["T"], warm["Y"], stream=stream)
    ctx.advance([wid], [0.0], stream=stream)  # a zero step (one iteration) sets up the workspace pool
    iid = ctx.state_upload(mid, st["rho"], st["T"], st["Y"], stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.advance([iid], [1e-6], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    out = ctx.download(iid)
    iters = float(out[4].astype(np.float64).sum())
    b = flops.global_tier_bytes(m)
    gbs = b["total"] * iters / sec / 1e9
    res = dict(mechanism="generated 100 species / 600 reactions", cells=n, seconds=sec, cells_per_s=n / sec,
               newton_iters_per_cell=iters / n, status_hist=np.bincount(out[2], minlength=4).tolist(),
               layout=ctx.query_int(kin.Q_LAYOUT, mid), bytes_per_iteration=b["total"],
               achieved_GB_s=gbs, hbm_peak_GB_s=8000.0, frac=gbs / 8000.0)
    for i in (wid, iid):
        ctx.instance_release(i)
    ctx.mech_release(mid)
    return res


def run_fluid(torch, ctx, kin, synth, args, stream):
    """The fluid step (Sec. 3.1: dimensionally split MP5 / HLLE sweeps, three Runge-Kutta stages
    each) and the operator-split step (Sec. 2: the fluid step, then the chemistry sub-step through
    the conserved-variable adapter) on the headline's band grid of the 9-species mixture, FP64,
    periodic, 0.1 mm cells, with a shear flow u = 50 sin(2 pi y) m/s, v = 30 cos(2 pi x) m/s
    added to the band state.  The conserved input is made by the library from (rho, T, Y) through
    its adapter.  The step size is the CFL bound at 0.4.  Reported: fluid steps per second and
    cells/s, the split step's time and the chemistry's share of it, and the fluid step's
    algorithmic HBM bandwidth (each of the six stages reads its input state, stages 2 and 3 also
    the sweep's start state, and writes its output: 128 (Ns + 3) bytes per cell-step)."""
    nx = 256 if args.quick else 1024
    m, grid, _ = synth.workload_grid_mech9(nx, nx)
    ns, n = m.ns, grid.n
    mid = ctx.mech_upload(m)
    st = device_state(torch, grid)
    iid = ctx.state_upload(mid, st["rho"], st["T"], st["Y"], stream=stream)
    rho_s = torch.empty((ns, n), dtype=torch.float64, device="cuda")
    Es = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.download_conserved_device(iid, rho_s, Es, stream=stream)
    x = (torch.arange(nx, dtype=torch.float64, device="cuda") + 0.5) / nx
    u = (50.0 * torch.sin(2 * np.pi * x))[:, None].expand(nx, nx).reshape(n)       # varies with y (rows)
    v = (30.0 * torch.cos(2 * np.pi * x))[None, :].expand(nx, nx).reshape(n)       # varies with x
    rho = st["rho"]
    Q = torch.cat([rho_s, (rho * u)[None], (rho * v)[None], (Es + 0.5 * rho * (u * u + v * v))[None]]).contiguous()
    fid = ctx.fluid_create(mid, nx, nx, 1e-4, 1e-4, kin.BC_PERIODIC)
    ctx.fluid_upload(fid, Q, stream=stream)
    dt = ctx.fluid_max_dt(fid, 0.4, stream=stream)
    steps = args.steps
    for k in range(2):
        ctx.fluid_step(fid, dt, y_first=bool(k & 1), stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        ctx.fluid_step(fid, dt, y_first=bool(k & 1), stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_fluid = e0.elapsed_time(e1) * 1e-3 / steps
    ctx.fluid_upload(fid, Q, stream=stream)
    ctx.split_step(fid, iid, dt, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(steps):
        ctx.split_step(fid, iid, dt, y_first=bool(k & 1), stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_split = e0.elapsed_time(e1) * 1e-3 / steps
    status = ctx.download(iid)[2]
    bytes_step = 128 * (ns + 3) * n
    res = dict(grid=f"{nx}x{nx}", cells=n, dt=dt, steps=steps, fluid_ms_per_step=1e3 * t_fluid,
               fluid_cells_per_s=n / t_fluid, split_ms_per_step=1e3 * t_split, split_cells_per_s=n / t_split,
               chemistry_share_of_split=(t_split - t_fluid) / t_split,
               chemistry_status_hist=np.bincount(status, minlength=4).tolist(),
               algorithmic_bytes_per_cell_step=128 * (ns + 3), achieved_GB_s=bytes_step / t_fluid / 1e9,
               hbm_peak_GB_s=8000.0, frac=bytes_step / t_fluid / 1e9 / 8000.0)
    ctx.fluid_release(fid)
    ctx.instance_release(iid)
    ctx.mech_release(mid)
    return res


def run_mech36(torch, ctx, kin, flops, synth, args, stream):
    n36 = (1 << 14) if args.quick else (1 << 18)
    m36, s36, dt36 = synth.workload_mech36(n36)
    mid36 = ctx.mech_upload(m36)
    st36 = device_state(torch, s36)
    iid36 = ctx.state_upload(mid36, st36["rho"], st36["T"], st36["Y"], stream=stream)
    f36 = flops.newton_iteration_flops(m36)["total"]
    res, outs = {}, {}
    for name, prec in (("fp64", kin.FP64), ("fp32lu", kin.FP32_LU)):
        log(f"mech36 {n36} cells, 1 step, {name}")
        tot, per, kern = time_steps(torch, ctx, iid36, st36, dt36, prec, 1, 1, stream)
        its, hist, lvmax, out = replay_stats(torch, ctx, iid36, st36, dt36, prec, 1, stream)
        ctx.kernel_times()
        res[f"mech36_{name}"] = form_stats(n36, 1, tot, per, kern, its, hist, lvmax, f36)
        outs[name] = out
    res["mech36_fp32lu"]["deviation_from_fp64_one_step"] = deviation(outs["fp64"], outs["fp32lu"])
    log(f"mech36 {n36} cells, 1 step, point-implicit")
    res["mech36_point_implicit_fp64"] = point_implicit_form(torch, ctx, kin, iid36, st36, dt36, 1, n36, f36,
                                                            outs["fp64"], stream)
    res["mech36_layout"] = [ctx.query_int(kin.Q_LAYOUT, mid36), ctx.query_int(kin.Q_BLOCK, mid36)]
    ctx.instance_release(iid36)
    ctx.mech_release(mid36)
    return res


def run_batch(torch, kin, synth, args, stream):
    """64 uneven instances, FP32-LU, one graph launch vs 64 separate launches.  The autotuner
    picks each mechanism's layout at the size class of that mechanism's launch in the batch (all
    its instances together: about 837k cells of mech9 and 1.26M of mech36), probing with the
    launch's cell count capped at 262144 (the top size class starts there)."""
    n_inst = 16 if args.quick else 64
    hi = 16384 if args.quick else 262144
    insts = synth.batch_instances(seed=3, n_inst=n_inst, min_cells=1024, max_cells=hi)
    cache = os.path.join(tempfile.mkdtemp(prefix="kin_tune_"), "tune.json")
    res = {}
    names = {0: "auto", 1: "lane", 2: "wave", 3: "global"}
    with kin.Context(0, tune_cache=cache) as ctx:
        mids, layouts = {}, {}
        for name in ("mech9", "mech36"):
            m = synth.mechanism(name)
            mids[name] = ctx.mech_upload(m)
            group = sum(ins.n_cells for ins in insts if ins.mech == name)
            if group == 0:
                continue
            probe = synth.uniform_cells(7, min(group, 262144), m.ns, 1.0 if name == "mech9" else 0.5)
            pid = ctx.state_upload(mids[name], probe.rho, probe.T, probe.Y)
            log(f"autotune {name} at {probe.n} cells (launch of {group})")
            lay, blk, ms = ctx.autotune(mids[name], pid, 1e-6, kin.FP32_LU)
            layouts[name] = lay
            res[f"autotune_{name}"] = dict(layout=names[lay], block=blk, ms=ms, probe_cells=probe.n,
                                           launch_cells=group, size_class=kin.size_class(group))
            ctx.instance_release(pid)
        states, ids = [], []
        for ins in insts:
            st = device_state(torch, ins.states())
            states.append(st)
            ids.append(ctx.state_upload(mids[ins.mech], st["rho"], st["T"], st["Y"], stream=stream))
        dts = [ins.dt for ins in insts]
        cells = sum(ins.n_cells for ins in insts)

        def reset():
            for i, st in zip(ids, states):
                ctx.state_reset(i, st["rho"], st["T"], st["Y"], stream=stream)
            torch.cuda.synchronize()

        def snapshot():
            out = []
            for i, ins in zip(ids, insts):
                ns = synth.mechanism(ins.mech).ns
                T = torch.empty(ins.n_cells, dtype=torch.float64, device="cuda")
                Y = torch.empty((ns, ins.n_cells), dtype=torch.float64, device="cuda")
                ctx.download_device(i, T, Y, stream=stream)
                out.append((T, Y))
            torch.cuda.synchronize()
            return out

        log(f"batch of {len(insts)} instances, {cells} cells: graph build")
        ctx.advance(ids, dts, prec=kin.FP32_LU, stream=stream)   # builds and caches the graph
        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        log("batch: one graph launch")
        e0.record(stream)
        ctx.advance(ids, dts, prec=kin.FP32_LU, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t_graph = e0.elapsed_time(e1) * 1e-3
        g = snapshot()
        reset()
        log("batch: 64 separate launches")
        # the same layouts as the graph's launches, so that the results compare bitwise (a lone
        # instance's own size class could pick another layout)
        sep_opts = {k: kin.solver_opts(layout=v) for k, v in layouts.items()}
        e0.record(stream)
        for i, dt, ins in zip(ids, dts, insts):
            ctx.advance([i], [dt], prec=kin.FP32_LU, stream=stream, opts=sep_opts[ins.mech])
        e1.record(stream)
        torch.cuda.synchronize()
        t_sep = e0.elapsed_time(e1) * 1e-3
        s = snapshot()
        same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(g, s))
        res.update(instances=len(insts), cells=cells, graph_s=t_graph, separate_s=t_sep,
                   cells_per_s_graph=cells / t_graph, cells_per_s_separate=cells / t_sep,
                   graph_equals_separate_bitwise=bool(same))
        for i in ids:
            ctx.instance_release(i)
    return res


def run_serving(torch, kin, serve, synth, args):
    """Calibrate the saturated rate with every request present at t = 0, then serve Poisson
    arrivals at fractions of it.  The 36-species requests run on two streams confined to all
    but 32 compute units (reserve_cu), the 9-species requests on two other streams, which keeps
    the 9-species requests from queueing behind them, for compute units or in a hardware queue.
    Kept for comparison: one stream per slot, no reservation, and requests above 65536 cells
    served as parts of at most that size (serve.split)."""
    n_req = 20 if args.quick else args.serve_requests
    budget = 256 << 20
    out = {}
    # (name, precision, reserved CUs, split size, streams per class, loads)
    plan = (("fp32lu", kin.FP32_LU, 32, None, 2, (0.5, 0.8, 0.95)), ("fp64", kin.FP64, 32, None, 2, (0.8,)),
            ("fp32lu_stream_per_slot", kin.FP32_LU, 32, None, None, (0.8,)),
            ("fp32lu_no_reserve", kin.FP32_LU, 0, None, 2, (0.8,)),
            ("fp32lu_split_65536", kin.FP32_LU, 32, 65536, 2, (0.8,)))
    with kin.Context(0, hbm_budget=budget) as ctx:
        mids = {name: ctx.mech_upload(synth.mechanism(name)) for name in ("mech9", "mech36")}
        for name, prec, reserve, chunk, nstreams, loads in plan:
            be = serve.KinBackend(ctx, mids, prec, n_slots=16, reserve_cu=reserve, n_streams=nstreams)
            reqs = synth.serving_requests(4, n_req, rate_per_s=1.0)
            jobs = serve.make_jobs(reqs, time_scale=0.0)
            for j, r in zip(jobs, reqs):
                be.prepare(j, r.inst.states(), max_chunk=chunk)
            log(f"serving {name}: saturation run, {n_req} requests")
            sat = serve.run(jobs, be, budget, 16, max_chunk=chunk).summary()
            rate = sat["cells_per_s"] / synth.mean_request_cells()
            runs = {"reserve_cu": reserve, "max_chunk": chunk, "streams_per_class": nstreams or 16, "saturated": sat}
            for load in loads:
                reqs = synth.serving_requests(4, n_req, rate_per_s=load * rate)
                jobs = serve.make_jobs(reqs)
                for j, r in zip(jobs, reqs):
                    be.prepare(j, r.inst.states(), max_chunk=chunk)
                log(f"serving {name}: load {load}")
                runs[f"load_{load}"] = serve.run(jobs, be, budget, 16, max_chunk=chunk).summary()
            be.close()
            out[name] = runs
    return out


def run_copy(torch):
    """A plain device-to-device copy of 512 MiB (torch's copy kernel): the reference for scaling
    the HBM byte counters."""
    a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}


def run_gpu(args):
    import torch
    from paper_1110_4903_amd import flops, kin, serve, synth

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    res = {}
    grid = m9 = dt9 = one_step = None
    if args.only == "copy":
        return run_copy(torch), None, None, None, None
    with kin.Context(0, time_kernels=True) as ctx:
        if args.only in ("all", "headline"):
            head, grid, m9, dt9, one_step = run_headline(torch, ctx, kin, flops, synth, args, stream)
            res.update(head)
        if args.only in ("all", "mech36"):
            res.update(run_mech36(torch, ctx, kin, flops, synth, args, stream))
        if args.only == "all":
            log("config 0 end to end (host buffers)")
            res["mech9_4096_end_to_end_host_buffers"] = run_config0_end_to_end(torch, ctx, kin, synth, stream)
        if args.only in ("all", "adapter"):
            log("operator-split adapter on the headline grid")
            res["mech9_conserved_adapter_fp64"] = run_conserved_adapter(torch, ctx, kin, synth, args, stream)
        if args.only in ("all", "global"):
            log("global-memory layout, 100 species, 65536 cells")
            res["gen100_global_fp64"] = run_global_tier(torch, ctx, kin, flops, synth, args, stream)
        if args.only in ("all", "fluid"):
            log("fluid step and operator-split step on the headline grid")
            res["mech9_fluid_split_fp64"] = run_fluid(torch, ctx, kin, synth, args, stream)
    if args.only in ("all", "batch") and not args.no_batch:
        res["batch64"] = run_batch(torch, kin, synth, args, stream)
    if args.only in ("all", "serve") and not args.no_serve:
        res["serving"] = run_serving(torch, kin, serve, synth, args)
    return res, grid, m9, dt9, one_step


def error_vs_oracle(om, grid, dt, gpu, ref, trace, rtol):
    """Error of one GPU step against the FP64 oracle, every cell of the grid: cells whose
    sub-step schedule (status, level, schedule hash) matches the oracle's own are compared with
    its adaptive step, the others with the oracle following the GPU's recorded schedule.  Per
    result: the largest relative error of T and of the mass fractions of at least 1e-14, the
    99.9th percentile of the latter, the count of results beyond the form's gate rtol (mass
    fractions of at least 1e-10; smaller ones are reported by their largest absolute error) and
    the count of cells with any result beyond it."""
    same = (gpu[2] == ref[2]) & (gpu[3] == ref[3]) & (gpu[5] == ref[5])
    mis = np.flatnonzero(~same)
    Tr, Yr, sr = ref[0].copy(), ref[1].copy(), ref[2].copy()
    follow_fail = 0
    if mis.size:
        sub = grid.subset(mis)
        e0 = om.energy_batch(sub.T, sub.Y)
        fol = om.follow(sub.rho, sub.T, sub.Y, dt, e0, trace[mis])
        follow_fail = int(((fol[2] < 0) | (fol[5] != gpu[5][mis])).sum())
        Tr[mis], Yr[:, mis], sr[mis] = fol[0], fol[1], fol[2]
    ok = (sr < 2) & (gpu[2] < 2)
    Yg, Yo = gpu[1][:, ok], Yr[:, ok]
    dY = np.abs(Yg - Yo)
    big = np.abs(Yo) >= 1e-14
    rel = np.where(big, dY / np.maximum(np.abs(Yo), 1e-300), 0.0)
    relT = np.abs(gpu[0][ok] - Tr[ok]) / Tr[ok]
    gated = np.abs(Yo) >= 1e-10
    return dict(cells=int(gpu[2].shape[0]), own_schedule=int(same.sum()), followed_gpu_schedule=int(mis.size),
                follow_fail=follow_fail, compared=int(ok.sum()), gate_rtol=rtol,
                max_rel_Y=float(rel.max()), p999_rel_Y=float(np.quantile(rel[big], 0.999)),
                max_rel_T=float(relT.max()), beyond_gate_Y=int((gated & (rel > rtol)).sum()),
                beyond_gate_T=int((relT > rtol).sum()),
                cells_beyond_gate=int(((gated & (rel > rtol)).any(0) | (relT > rtol)).sum()),
                max_abs_Y_below_1em10=float(dY[~gated].max()) if (~gated).any() else 0.0)


def cpu_baseline(grid, m9, dt9, steps, sample_stride, one_step=None):
    """The FP64 oracle on the host cores over a strided sample of the headline grid.  With the
    GPU's one-step results and schedule records of the full grid (one_step), the oracle's first
    step also states each form's error against the oracle, per result."""
    from oracle import oracle
    om = oracle.OracleMech(m9)
    idx = np.arange(0, grid.n, sample_stride)
    sub = grid.subset(idx)
    e0 = om.energy_batch(sub.T, sub.Y)
    T, Y = sub.T.copy(), sub.Y.copy()
    first = None
    t0 = time.time()
    for k in range(steps):
        T, Y, st_, lv_, it_, sh_ = om.advance(sub.rho, T, Y, dt9, e0=e0, with_sched=True)
        if k == 0:
            first = (T, Y, st_, lv_, it_, sh_)
    el = time.time() - t0
    # the same oracle on one thread, over every 64th cell of that sample
    sub1 = grid.subset(idx[::64])
    e1 = om.energy_batch(sub1.T, sub1.Y)
    T, Y = sub1.T.copy(), sub1.Y.copy()
    t1 = time.time()
    for _ in range(steps):
        T, Y, _, _, _ = om.advance(sub1.rho, T, Y, dt9, e0=e1, nthreads=1)
    el1 = time.time() - t1
    out = dict(value=idx.shape[0] * steps / el, unit="cells/s", cores=oracle.num_threads(), kind="oracle",
               sample=f"{idx.shape[0]} cells (every {sample_stride}th of the {int(np.sqrt(grid.n))}^2 grid) x "
                      f"{steps} steps of dt=1e-6 s, FP64, {el:.1f} s",
               single_thread_cells_per_s=sub1.n * steps / el1,
               single_thread_sample=f"{sub1.n} cells x {steps} steps, {el1:.1f} s")
    if one_step is not None and sample_stride == 1:
        for name, rtol in (("fp64", 1e-10), ("fp32lu", 1e-6)):
            if name in one_step["traces"]:
                log(f"error of the {name} form against the oracle, every cell of one step")
                out[f"error_vs_oracle_{name}_one_step"] = error_vs_oracle(
                    om, grid, dt9, one_step["outs"][name], first, one_step["traces"][name], rtol)
    return out


def kernel_source_hash() -> str:
    """Hash of the sources that define the headline kernel (lane layout): template and
    generator.  A traffic figure measured for another hash is stale."""
    h = hashlib.sha256()
    for f in ("kin_lane_template.h", "kin_codegen.cpp"):
        with open(os.path.join(HERE, "paper_1110_4903_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_cells):
    """HBM bytes per launch of the headline kernel from the committed counter summary, scaled
    to this launch's cell count; None when the summary is missing or the kernel has changed."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.split("=", 1) for line in f.read().splitlines() if "=" in line and not line.startswith("#"))
        if kv.get("kernel_source_hash", "").strip() != kernel_source_hash():
            return None
        return float(kv["hbm_bytes_per_cell_step"]) * launch_cells
    except (OSError, KeyError, ValueError):
        return None


VALU_PROFILE = os.path.join(HERE, "profiles", "valu_kin_lane_f64_mech9_grid1024.txt")


def measured_valu(h):
    """FP64 vector work of the headline kernel from the committed counter summary (rocprofv3 SQ
    instruction counters over the profiled run's timed launches): floating-point operations per
    Newton iteration (64 lanes per wave instruction, FMA 2, add, multiply and transcendental 1),
    times this run's iterations, over this run's kernel time.  None when the summary is missing
    or the kernel has changed since."""
    try:
        with open(VALU_PROFILE) as f:
            kv = dict(line.split("=", 1) for line in f.read().splitlines() if "=" in line and not line.startswith("#"))
        if kv.get("kernel_source_hash", "").strip() != kernel_source_hash():
            return None
        per_iter = float(kv["fp64_flop_per_timed_run"]) / float(kv["newton_iterations_per_timed_run"])
        flop = per_iter * float(np.sum(h["newton_iters"]))
        secs = 1e-3 * float(np.sum(h["kernel_ms"]))
        return {"fp64_flop_per_newton_iteration_counter": per_iter, "fp64_flop_this_run": flop,
                "achieved_TFLOPs_counter": flop / secs / 1e12,
                "frac_counter": flop / secs / 1e12 / FP64_PEAK_TFLOPS,
                "valu_fp64_share": float(kv["valu_fp64_share"]), "valu_busy": float(kv["valu_busy"]),
                "source": os.path.relpath(VALU_PROFILE, HERE)}
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=160)
    ap.add_argument("--quick", action="store_true", help="small sizes, for smoke runs")
    ap.add_argument("--only", default="all", choices=("all", "headline", "mech36", "adapter", "global", "fluid", "batch", "serve", "copy"),
                    help="run one part (for profiler runs); the JSON line needs the headline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU: the per-cell kinetics update has no "
                                   "cross-GPU exchange (cells shard trivially), so --gpus must be 1"}))
        sys.exit(2)
    res, grid, m9, dt9, one_step = run_gpu(args)
    if grid is None:
        print(json.dumps({"only": args.only, "forms": res}))
        return
    cpu = None
    if not args.no_cpu and args.only == "all":
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(grid, m9, dt9, args.steps, 1 if not args.quick else 4, one_step)
    h = res["mech9_fp64"]
    traffic = measured_traffic(grid.n)
    from paper_1110_4903_amd import flops, synth
    fl = flops.newton_iteration_flops(synth.mechanism("mech9"))
    counters = measured_valu(h)
    side = int(np.sqrt(grid.n))
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
        "config": {"workload": f"mech9 (9 species, 38 reactions) on a {side}x{side} band grid, {args.steps} steps "
                               f"of dt=1e-6 s, FP64 form, state resident in HBM",
                   "cells": grid.n, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": h["tflops_model"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": h["tflops_model"] / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "kin_lane_f64",
                     "flops_per_newton_iteration": fl["total"],
                     "flops_per_newton_iteration_exp_as_1": fl["total"] - (flops.TRANSCENDENTAL - 1) * fl["transcendentals"],
                     "newton_iterations": int(np.sum(h["newton_iters"])),
                     "kernel_seconds": 1e-3 * float(np.sum(h["kernel_ms"])),
                     "frac_exp_as_1": (fl["total"] - (flops.TRANSCENDENTAL - 1) * fl["transcendentals"]) *
                                      float(np.sum(h["newton_iters"])) / (1e-3 * float(np.sum(h["kernel_ms"]))) /
                                      1e12 / FP64_PEAK_TFLOPS,
                     "counters": counters},
        "cpu_baseline": cpu,
        "forms": res,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
