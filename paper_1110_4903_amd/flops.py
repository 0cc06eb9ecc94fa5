"""Algorithmic work model of one Newton iteration of the implicit kinetics update.

Counts floating-point operations of the method as written (Sec. 3.2 of the paper: rates,
equilibrium constants, third-body sums, production terms, the analytic Jacobian, the Newton
matrix I - hJ and its Gaussian elimination), independent of how a kernel schedules them:
an FMA counts 2, an add, multiply, divide or compare 1, and each exp/log a nominal 25 (the
polynomial and range-reduction cost of an FP64 exponential).  Selects, loads and stores are
not counted.  The temperature inversion after an accepted sub-step is not counted either
(a few percent of a Newton iteration).
"""
from __future__ import annotations

TRANSCENDENTAL = 25


def _parts(mech, r):
    sp = {}
    for j in range(3):
        for idx, nu, sign in ((mech.reac_idx[r, j], mech.reac_nu[r, j], -1),
                              (mech.prod_idx[r, j], mech.prod_nu[r, j], +1)):
            if idx >= 0:
                sp[int(idx)] = sp.get(int(idx), 0) + sign * int(nu)
    return sp


def newton_iteration_flops(mech) -> dict:
    """Per-iteration flops by phase, plus the transcendental count."""
    ns = mech.ns
    N = ns + 1
    setup = 1 + TRANSCENDENTAL + 4          # 1/T, ln T, rho scaling, ln(P/RT)
    thermo = ns * (12 + 10 + 1 + 2)          # h/RT, s/R, g/RT, concentration
    rates = 0
    scatter = 0
    n_exp = 1
    for r in range(mech.nr):
        parts = _parts(mech, r)
        npart = len(parts)
        nnz = sum(1 for v in parts.values() if v != 0)
        nreac = int((mech.reac_idx[r] >= 0).sum())
        nprod = int((mech.prod_idx[r] >= 0).sum())
        tb = mech.tb[r] >= 0
        f = 4 + TRANSCENDENTAL + 3 + nreac        # ln kf, kf, d ln kf/dT, forward product
        n_exp += 1
        if mech.reversible[r]:
            f += 4 * npart + 2 + TRANSCENDENTAL + 2 + nprod + 1   # ln Kc, kb, d ln Kc/dT, pb, D
            n_exp += 1
        if tb:
            f += 2 * ns
        f += 1 + 5 + 3 * npart                     # q, dq/dT, dq/dc per participant
        rates += f
        scatter += nnz * 2 * (2 + npart + (ns if tb else 0))
    closing = 2 * ns + 2 + ns * (8 + 6 + 3 + 2 + 6) + 2 * ns * ns + 2 * ns + 2 * ns + 4
    newton_matrix = 2 * N * N + 3 * N
    lu = (2 * N ** 3) // 3 - (N * N) // 2 - N // 6 + N
    solve = 2 * N * N - N
    control = 4 * N
    out = dict(setup=setup, thermo=thermo, rates=rates, jacobian_scatter=scatter,
               closing=closing, newton_matrix=newton_matrix, lu=lu, solve=solve, control=control)
    out["total"] = sum(out.values())
    out["transcendentals"] = n_exp
    return out


def global_tier_bytes(mech) -> dict:
    """Algorithmic memory traffic (bytes) of one Newton iteration of one cell when the cell's
    (Ns+1)^2 matrix lives in global memory (the paper's first kinetics kernel, Sec. 4.2), by
    phase.  Every element the method touches is counted once per pass that touches it: the
    Jacobian is cleared (write), assembled by read-modify-write of each nonzero reaction
    contribution, completed in one pass over its columns (read and write: the dense
    third-body terms and the energy row are formed on chip, the matrix becomes I - hJ), and
    eliminated in panels of `panel` columns (8 up to 128 unknowns, else 4): a panel's columns
    are read for the rows not yet pivoted and written back for the rows it pivots, and every
    column right of the panel is read and written once per panel for the rows not yet
    pivoted.  The back substitution reads the upper triangle.  Padding of the stored system
    is not counted."""
    ns = mech.ns
    N = ns + 1
    panel = 8 if N <= 128 else 4
    clear = 8 * N * N
    scatter = 0
    for r in range(mech.nr):
        parts = _parts(mech, r)
        n = sum(1 for v in parts.values() if v != 0)
        scatter += 16 * (n * n + 2 * n)            # J block, T column and production sums
    columns = 16 * N * N
    lu = 0
    for k0 in range(0, N, panel):
        kb = min(panel, N - k0)
        rows = N - k0
        lu += 8 * kb * rows + 8 * kb * kb + 16 * (N - k0 - kb) * rows
    back = 8 * N * (N - 1) // 2 + 16 * N
    out = dict(clear=clear, scatter=scatter, column_pass=columns, elimination=lu, back_substitution=back)
    out["total"] = sum(out.values())
    return out
