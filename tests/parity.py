"""Comparison helpers shared by the GPU parity tests (test infrastructure).

Gate (per result, every cell, every species and T): |y_gpu - y_ref| <= rtol |y_ref| + floor,
where the floor 1e3 * eps64 * S_s uses the term scale S_s of the backward-Euler residual row
of species s (the magnitude of the terms that cancel in it), as computed by the oracle.  T has
no floor.  rtol is 1e-10 for the FP64 form and 1e-6 for the FP32-LU form.
"""
from __future__ import annotations

import numpy as np

EPS64 = np.finfo(np.float64).eps


def term_scales(om, rho, Y0, T1, Y1, dt):
    S = np.empty_like(Y1)
    for i in range(rho.shape[0]):
        S[:, i] = om.term_scale(rho[i], Y0[:, i], np.r_[Y1[:, i], T1[i]], dt)
    return S


def compare(gpu, ref, rho, Y0, dt, om, rtol, sample=None, extra=None):
    """gpu, ref: (T, Y, status, level, iters[, schedule hash]).  Cells are compared when their
    status, level and (if both sides give one) sub-step schedule hash agree.  extra: optional
    ([Ns][n_cells], [n_cells]) added to the mass-fraction and temperature tolerances.  Returns
    a dict of statistics."""
    Tg, Yg, sg, lg, ig = gpu[:5]
    Tr, Yr, sr, lr, ir = ref[:5]
    idx = np.arange(Tg.shape[0]) if sample is None else np.asarray(sample)
    same_sched = (sg[idx] == sr[idx]) & (lg[idx] == lr[idx])
    sched_mismatch = 0
    if len(gpu) > 5 and len(ref) > 5:
        same_hash = gpu[5][idx] == ref[5][idx]
        sched_mismatch = int((~same_hash).sum())
        same_sched &= same_hash
    ok_cells = idx[(sr[idx] < 2) & same_sched]
    S = term_scales(om, rho[ok_cells], Y0[:, ok_cells], Tr[ok_cells], Yr[:, ok_cells], dt)
    dY = np.abs(Yg[:, ok_cells] - Yr[:, ok_cells])
    tolY = rtol * np.abs(Yr[:, ok_cells]) + 1e3 * EPS64 * S
    if extra is not None:
        tolY = tolY + extra[0][:, ok_cells]
    dT = np.abs(Tg[ok_cells] - Tr[ok_cells])
    tolT = rtol * np.abs(Tr[ok_cells])
    if extra is not None:
        tolT = tolT + extra[1][ok_cells]
    big = np.abs(Yr[:, ok_cells]) >= 1e-14
    rel = np.where(big, dY / np.maximum(np.abs(Yr[:, ok_cells]), 1e-300), 0.0)
    return dict(
        n=int(idx.shape[0]),
        status_mismatch=int((sg[idx] != sr[idx]).sum()),
        schedule_mismatch=sched_mismatch,
        level_mismatch=int((lg[idx] != lr[idx]).sum()),
        iters_mismatch=int((ig[idx] != ir[idx]).sum()),
        compared=int(ok_cells.shape[0]),
        fail_Y=int((dY > tolY).any(0).sum()),
        fail_T=int((dT > tolT).sum()),
        max_rel_Y=float(rel.max()) if rel.size else 0.0,
        max_rel_T=float((dT / Tr[ok_cells]).max()) if ok_cells.size else 0.0,
        floor_active=int(((dY > rtol * np.abs(Yr[:, ok_cells])) & (dY <= tolY)).sum()),
    )


def point_implicit_floor(om, rho, Y0, T0, Y1, T1, dt, eps, cap=1e-6):
    """Extra tolerance of the point-implicit step, whose result is a single linear solve
    (I - dt J(x_n)) dx = dt f(x_n) with no Newton correction: a perturbation of A of relative
    size eps moves dx by up to cond(A) eps |dx|.  The mass-fraction floor is
    1e3 eps cond_1(D A) |dx_s| per cell, with D the row equilibration the FP32-LU form applies,
    capped at cap |dx_s|.  The temperature follows from the mass fractions through
    e(Y, T) = e0, so its floor is sum_s |e_s| floor_s / c_v.  Returns (floor_Y, floor_T, over):
    `over` marks the cells whose uncapped floor passed the cap; the value gate does not hold
    for them, and their solve is checked by its backward error instead (point_implicit_residual)."""
    n, ns = Y0.shape[1], Y0.shape[0]
    fy = np.zeros_like(Y0)
    ft = np.zeros(n)
    over = np.zeros(n, bool)
    unit = np.eye(ns)
    for c in range(n):
        x = np.r_[Y0[:, c], T0[c]]
        A = np.eye(ns + 1) - dt * om.jacobian(rho[c], x)
        A = A / np.abs(A).max(axis=1, keepdims=True)
        k = 1e3 * eps * np.linalg.cond(A, 1)
        over[c] = k > cap
        fy[:, c] = min(k, cap) * np.abs(Y1[:, c] - Y0[:, c])
        es = np.array([om.energy(unit[s], T1[c]) for s in range(ns)])
        ft[c] = np.abs(es) @ fy[:, c] / om.cv(Y1[:, c], T1[c])
    return fy, ft, over


def point_implicit_residual(om, rho, Y0, T0, Y_gpu, dt):
    """Componentwise backward error of the GPU's point-implicit solve, evaluated in long double
    with the oracle's J(x_n) and f(x_n): dx_Y = Y_gpu - Y0 and the temperature change dx_T that
    fits the whole system best (the GPU reports T after the energy inversion, not T + dx_T:
    weighted least squares over all rows, weights the rows' scales, two passes), then max over
    the rows of |r_i| / (sum_j |A_ij| (|dx_j| + eps |Y_gpu,j|) + dt |f_i|), r = A dx - dt f
    (the eps term covers the rounding of Y0 + dx).  Small whatever cond(A) is: it checks the
    solve itself, not its sensitivity."""
    n, ns = Y0.shape[1], Y0.shape[0]
    out = np.zeros(n)
    ld = np.longdouble
    for c in range(n):
        x = np.r_[Y0[:, c], T0[c]]
        A = np.eye(ns + 1, dtype=ld) - ld(dt) * om.jacobian(rho[c], x).astype(ld)
        b = ld(dt) * om.rhs(rho[c], x).astype(ld)
        dx = np.zeros(ns + 1, dtype=ld)
        dx[:ns] = Y_gpu[:, c].astype(ld) - Y0[:, c].astype(ld)
        rest = A[:, :ns] @ dx[:ns] - b              # residual without the temperature change
        roun = np.abs(A[:, :ns]) @ (EPS64 * np.abs(Y_gpu[:, c]).astype(ld))
        scale = np.abs(A[:, :ns]) @ np.abs(dx[:ns]) + np.abs(b) + roun
        for _ in range(2):
            w2 = 1 / scale ** 2
            dx[ns] = -np.sum(w2 * A[:, ns] * rest) / np.sum(w2 * A[:, ns] ** 2)
            scale = np.abs(A) @ np.abs(dx) + np.abs(b) + roun
        out[c] = float(np.max(np.abs(rest + A[:, ns] * dx[ns]) / scale))
    return out


def gpu_traces(ctx, mech_id, st, dt, prec, opts=None, steps=1, words=64):
    """Advance cells on the GPU with the schedule recorder, step by step: per step the schedule
    record [n][words] and the GPU's (T, Y, status, level, iters, schedule hash) after it."""
    iid = ctx.state_upload(mech_id, st.rho, st.T, st.Y)
    traces, outs = [], []
    for _ in range(steps):
        traces.append(ctx.advance_trace(iid, dt, prec=prec, opts=opts, words=words))
        outs.append(ctx.download(iid) + (ctx.download_schedule(iid),))
    ctx.instance_release(iid)
    return traces, outs


def oracle_follow(om, st, dt, traces, opts=None, e0=None):
    """The oracle advanced along the GPU's own sub-step schedules, step after step, from the same
    inputs (its own e0 unless given): its backward-Euler solution over exactly the GPU's
    sub-steps.  Returns (T, Y, status, level, iters, schedule hash) of the last step."""
    e0 = om.energy_batch(st.T, st.Y) if e0 is None else e0
    T, Y = st.T.copy(), st.Y.copy()
    out = None
    for tr in traces:
        out = om.follow(st.rho, T, Y, dt, e0, tr, opts=opts)
        T, Y = out[0], out[1]
    return out


def check_every_cell(ctx, orc, mech, mech_id, st, dt, prec, gpu, ref, rtol, opts=None, orc_opts=None,
                     extra=None):
    """Every cell of a single step, against the oracle.  Cells whose sub-step schedule matches the
    oracle's own (status, level and schedule hash equal) are compared with the oracle's adaptive
    result; the others are advanced again on the GPU with the schedule recorder, and compared with
    the oracle following the GPU's schedule.  Returns the statistics of both comparisons and
    their union; 'unchecked' counts cells of neither kind (it should be zero), 'follow_fail'
    cells whose recorded schedule the oracle could not follow or whose recorded schedule's hash
    differs from the first run's, and 'ok_vs_failed' cells that one side finished and the other
    failed."""
    om = orc.OracleMech(mech)
    s = compare(gpu, ref, st.rho, st.Y, dt, om, rtol, extra=extra)
    sg, sr = gpu[2], ref[2]
    same = (sg == sr) & (gpu[3] == ref[3]) & (gpu[5] == ref[5])
    mis = np.flatnonzero(~same)
    out = dict(s)
    out.update(followed=0, follow_fail=0, fail_Y_followed=0, fail_T_followed=0, max_rel_Y_followed=0.0,
               max_rel_T_followed=0.0, ok_vs_failed=int(((sg < 2) != (sr < 2)).sum()))
    if mis.size:
        sub = st.subset(mis)
        traces, g2 = gpu_traces(ctx, mech_id, sub, dt, prec, opts)
        gsub = tuple(a[..., mis] for a in gpu)
        rerun_same = all(np.array_equal(x, y, equal_nan=True) for x, y in zip(g2[-1], gsub))
        fol = oracle_follow(om, sub, dt, traces, opts=orc_opts)
        bad = (fol[2] < 0) | (fol[5] != gsub[5]) | (fol[2] != gsub[2])
        ex = None if extra is None else (extra[0][:, mis], extra[1][mis])
        s2 = compare(gsub, fol, sub.rho, sub.Y, dt, om, rtol, extra=ex)
        out.update(followed=int(s2["compared"]), follow_fail=int(bad.sum()) + (0 if rerun_same else mis.size),
                   fail_Y_followed=s2["fail_Y"], fail_T_followed=s2["fail_T"],
                   max_rel_Y_followed=s2["max_rel_Y"], max_rel_T_followed=s2["max_rel_T"])
    n_valid = int((sr < 3).sum())
    out["checked"] = out["compared"] + out["followed"]
    out["unchecked"] = n_valid - out["checked"] - int((sg == 2).sum())
    out["failed_gpu"] = int((sg == 2).sum())
    return out
