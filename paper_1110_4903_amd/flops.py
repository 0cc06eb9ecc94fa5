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
    Jacobian is cleared (write), assembled by read-modify-write of each nonzero contribution,
    closed by the energy row (reads of the species block), turned into I - hJ (read and
    write), and eliminated: at pivot step k the search reads column k below the diagonal and
    every trailing element is read and written once (the pivot row's reuse across rows is
    not counted again).  The back substitution reads the upper triangle."""
    ns = mech.ns
    N = ns + 1
    clear = 8 * N * N
    scatter = 0
    for r in range(mech.nr):
        parts = _parts(mech, r)
        n = sum(1 for v in parts.values() if v != 0)
        scatter += 16 * (n * n + 2 * n)            # J block, T column and production sums
    tb = int((mech.tb >= 0).sum()) if hasattr(mech.tb, "__len__") else 0
    dense_tb = 0
    for r in range(mech.nr):
        if mech.tb[r] >= 0:
            dense_tb += 16 * ns * sum(1 for v in _parts(mech, r).values() if v != 0)
    energy_row = 8 * ns * ns + 8 * N
    newton = 16 * N * N
    lu = sum(8 * (N - k) + 16 * (N - k - 1) ** 2 for k in range(N))
    back = 8 * N * (N - 1) // 2 + 16 * N
    out = dict(clear=clear, scatter=scatter, third_body=dense_tb + 8 * tb * ns, energy_row=energy_row,
               newton_matrix=newton, elimination=lu, back_substitution=back)
    out["total"] = sum(out.values())
    return out
