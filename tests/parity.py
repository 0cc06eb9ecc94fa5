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


def point_implicit_floor(om, rho, Y0, T0, Y1, T1, dt, eps):
    """Extra tolerance of the point-implicit step, whose result is a single linear solve
    (I - dt J(x_n)) dx = dt f(x_n) with no Newton correction: a perturbation of A of relative
    size eps moves dx by up to cond(A) eps |dx|.  The mass-fraction floor is
    1e3 eps cond_1(D A) |dx_s| per cell, with D the row equilibration the FP32-LU form applies.
    The temperature follows from the mass fractions through e(Y, T) = e0, so its floor is
    sum_s |e_s| floor_s / c_v."""
    n, ns = Y0.shape[1], Y0.shape[0]
    fy = np.zeros_like(Y0)
    ft = np.zeros(n)
    unit = np.eye(ns)
    for c in range(n):
        x = np.r_[Y0[:, c], T0[c]]
        A = np.eye(ns + 1) - dt * om.jacobian(rho[c], x)
        A = A / np.abs(A).max(axis=1, keepdims=True)
        fy[:, c] = 1e3 * eps * np.linalg.cond(A, 1) * np.abs(Y1[:, c] - Y0[:, c])
        es = np.array([om.energy(unit[s], T1[c]) for s in range(ns)])
        ft[c] = np.abs(es) @ fy[:, c] / om.cv(Y1[:, c], T1[c])
    return fy, ft
