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


def compare(gpu, ref, rho, Y0, dt, om, rtol, sample=None):
    """gpu, ref: (T, Y, status, level, iters[, schedule hash]).  Cells are compared when their
    status, level and (if both sides give one) sub-step schedule hash agree.  Returns a dict
    of statistics."""
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
    dT = np.abs(Tg[ok_cells] - Tr[ok_cells])
    tolT = rtol * np.abs(Tr[ok_cells])
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
