"""Further pins of the FP64 CPU oracle, each independent of the oracle's own arithmetic:

- the temperature row of the source term (Sec. 2, Eq. energy: the cell holds its internal
  energy, so dT/dt must make e(Y, T) stationary along the trajectory), checked through the
  separately pinned mixture energy e(Y, T), an exactly energy-conserving two-species case and
  the second-order energy defect of a backward-Euler step;
- the adaptive sub-step controller (halving on failure, coarsening when aligned), re-run by an
  independent driver over the oracle's single sub-step with exact rational time;
- the Arrhenius forward rate and the equilibrium constant (Sec. 3.2), re-evaluated in 50-digit
  decimal arithmetic from the same inputs, within the rounding bound of an FP64 evaluation.
"""
import decimal
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1110_4903_amd import synth
from tests.test_oracle_pins import nasa_const, two_species_heat_release

EPS = np.finfo(np.float64).eps
SCHED_SEED, SCHED_PRIME = 0xcbf29ce484222325, 0x100000001b3


def species_energies(om, T):
    unit = np.eye(om.ns)
    return np.array([om.energy(unit[s], T) for s in range(om.ns)])


# ---------------------------------------------------------------------------------------------
# Temperature row (Sec. 2, Eq. energy; constant density and constant internal energy)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,alpha", [("mech9", 1.0), ("mech36", 0.5)])
def test_energy_is_stationary_along_the_source(orc, name, alpha):
    """d/de of e(Y + eps f_Y, T + eps f_T) at eps = 0 vanishes: the source term moves the state
    along a level set of the mixture energy.  Central differences of the oracle's e(Y, T) (pinned
    elsewhere by the c_v quadrature and closed forms) give a derivative at rounding level of the
    terms sum_s |e_s f_s| + |c_v f_T| that cancel in it; using c_p instead of c_v in f_T leaves a
    residue of order (1 - c_v/c_p) of those terms."""
    m = synth.mechanism(name)
    om = orc.OracleMech(m)
    st = synth.uniform_cells(81, 24, m.ns, alpha)
    for i in range(st.n):
        x = np.r_[st.Y[:, i], st.T[i]]
        f = om.rhs(st.rho[i], x)
        rate = max(abs(f[-1]) / x[-1], np.abs(f[:-1]).max())
        eps = 1e-6 / rate

        def e_at(a):
            return om.energy(x[:-1] + a * f[:-1], x[-1] + a * f[-1])

        D = (e_at(eps) - e_at(-eps)) / (2 * eps)
        scale = np.abs(species_energies(om, x[-1]) * f[:-1]).sum() + abs(om.cv(x[:-1], x[-1]) * f[-1])
        assert abs(D) <= 1e-8 * scale, (i, D / scale)


@pytest.mark.parametrize("dh_R,rho,yA,T", [(3000.0, 0.3, 0.9, 1200.0), (-2000.0, 1.0, 0.2, 2500.0),
                                           (8000.0, 0.02, 0.6, 800.0)])
def test_two_species_backward_euler_conserves_energy_exactly(orc, dh_R, rho, yA, T):
    """A <=> B with equal constant c_p and equal molar mass: e is linear in (Y, T) at fixed
    sum Y, so the backward-Euler step of (Y, T) itself conserves e, and the converged Newton
    iterate's temperature must already be the root of e(Y, T) = e0 that the inversion returns.
    Its T change is also the closed form T_be - T_n = -(h_B - h_A)/(R (c_p/R - 1)) (Y_B - Y_B,n)."""
    m = two_species_heat_release(dh_R)
    om = orc.OracleMech(m)
    x = np.array([yA, 1 - yA, T])
    e0 = om.energy(x[:-1], T)
    rc, xout, it, xbe = om.be_substep(rho, e0, x, 1e-6)
    assert rc == 0
    assert abs(xbe[-1] - xout[-1]) <= 1e-12 * T, (xbe[-1], xout[-1])
    dT = dh_R / 2.5 * (xbe[1] - x[1])
    assert abs(dT) > 1.0  # the step converts enough to move T
    assert abs((xbe[-1] - T) - dT) <= 1e-9 * abs(dT) + 1e-12 * T


def test_backward_euler_energy_defect_is_second_order(orc):
    """For a general mechanism backward Euler on the (Y, T) system conserves e only to O(h^2):
    the defect e(Y_be, T_be) - e0 of the converged Newton iterate falls about four-fold per
    halving of h.  A wrong energy row (c_p in place of c_v) adds an O(h) defect, which only
    halves."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(81, 24, m.ns, 1.0)
    ratios = []
    for i in range(st.n):
        x = np.r_[st.Y[:, i], st.T[i]]
        e0 = om.energy(x[:-1], x[-1])
        f = om.rhs(st.rho[i], x)
        h0 = 1e-2 / max(abs(f[-1]) / x[-1], np.abs(f[:-1]).max())
        d = []
        for k in range(5):
            rc, _, _, xbe = om.be_substep(st.rho[i], e0, x, h0 / 2 ** k)
            assert rc == 0
            d.append(om.energy(xbe[:-1], xbe[-1]) - e0)
        if abs(d[-1]) > 1e3 * EPS * abs(e0):  # above the rounding of e itself
            ratios.append(d[-2] / d[-1])
    assert len(ratios) >= 16
    med = float(np.median(ratios))
    assert 3.5 <= med <= 4.5, (med, ratios)


# ---------------------------------------------------------------------------------------------
# Adaptive sub-step controller (halving on failure), driven independently
# ---------------------------------------------------------------------------------------------

def controller_reference(orc, om, rho, e0, x0, dt, opts):
    """The dyadic controller as the design states it, over the oracle's single sub-step:
    time is exact (Fraction of dt); a sub-step at level l has size dt/2^l and starts from the
    last accepted state; a failure retries the same start at level l + 1 (the cell fails when
    l would pass L_max, or when max_iters Newton iterations are used before the step ends);
    after an acceptance the level drops by one when the elapsed time is a whole number of
    coarser sub-steps 2 dt/2^l.  Returns (status, x, deepest level, iterations, schedule hash,
    accepted sizes as fractions of dt)."""
    x = np.array(x0, dtype=np.float64)
    t, l, deepest, iters, failed = Fraction(0), 0, 0, 0, False
    sched, taken = SCHED_SEED, []
    outcomes = controller_reference.outcomes = []
    while t < 1:
        if iters >= opts.max_iters:
            return orc.FAILED, np.array(x0), deepest, iters, sched, taken
        rc, xn, it, _ = om.be_substep(rho, e0, x, math.ldexp(dt, -l), opts)
        iters += it
        ok = rc == 0
        outcomes.append(ok)
        sched = ((sched ^ (2 * l + int(ok))) * SCHED_PRIME) % (1 << 64)
        if ok:
            x = xn
            t += Fraction(1, 2 ** l)
            taken.append(Fraction(1, 2 ** l))
            if l > 0 and (t / Fraction(2, 2 ** l)).denominator == 1:
                l -= 1
        else:
            failed = True
            l += 1
            deepest = max(deepest, l)
            if l > opts.L_max:
                return orc.FAILED, np.array(x0), opts.L_max, iters, sched, taken
    return (orc.OK_HALVED if failed else orc.OK), x, deepest, iters, sched, taken


@pytest.mark.parametrize("name,alpha,n,dt", [("mech9", 1.0, 96, 1e-6), ("mech36", 0.5, 6, 1e-6)])
def test_adaptive_controller_matches_independent_driver(orc, name, alpha, n, dt):
    """orc_advance's adaptive sub-stepping equals, bitwise (state, status, level, iterations,
    schedule hash), the independent driver above; the accepted sub-steps of every finished cell
    add up to exactly dt; enough cells halve and coarsen again for the comparison to bite."""
    m = synth.mechanism(name)
    om = orc.OracleMech(m)
    st = synth.uniform_cells(91, n, m.ns, alpha)
    e0 = om.energy_batch(st.T, st.Y)
    opts = orc.default_opts()
    T1, Y1, s1, l1, i1, h1 = om.advance(st.rho, st.T, st.Y, dt, e0=e0, with_sched=True)
    coarsened = 0
    for c in range(st.n):
        s, x, lv, it, sh, taken = controller_reference(orc, om, st.rho[c], e0[c],
                                                       np.r_[st.Y[:, c], st.T[c]], dt, opts)
        assert (s, lv, it, sh) == (s1[c], l1[c], i1[c], int(h1[c])), c
        assert np.array_equal(x, np.r_[Y1[:, c], T1[c]]), c
        if s < 2:
            assert sum(taken) == 1
        levels = [-int(math.log2(f)) for f in taken]
        coarsened += any(b < a for a, b in zip(levels, levels[1:]))
    assert (s1 == 1).sum() >= n // 8 and coarsened >= n // 16, ((s1 == 1).sum(), coarsened)


def test_controller_with_tiny_level_cap_and_iteration_budget(orc):
    """The two ways a cell fails: L_max = 1 and a 12-iteration budget, each against the
    independent driver."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(92, 48, m.ns, 1.0)
    e0 = om.energy_batch(st.T, st.Y)
    for kw in (dict(L_max=1), dict(max_iters=12)):
        opts = orc.make_opts(**kw)
        T1, Y1, s1, l1, i1, h1 = om.advance(st.rho, st.T, st.Y, 1e-6, e0=e0, opts=opts, with_sched=True)
        assert (s1 == 2).sum() > 0 and (s1 < 2).sum() > 0, kw
        for c in range(st.n):
            s, x, lv, it, sh, _ = controller_reference(orc, om, st.rho[c], e0[c],
                                                       np.r_[st.Y[:, c], st.T[c]], 1e-6, opts)
            assert (s, lv, it, sh) == (s1[c], l1[c], i1[c], int(h1[c])), (kw, c)
            assert np.array_equal(x, np.r_[Y1[:, c], T1[c]]), (kw, c)


def pack_schedule(outcomes, words):
    """Schedule record of one cell: word 0 the attempt count, then the accept bits."""
    rec = np.zeros(words, np.uint64)
    rec[0] = len(outcomes)
    for j, ok in enumerate(outcomes[:64 * (words - 1)]):
        if ok:
            rec[1 + j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return rec


def test_follow_own_schedule_is_bitwise_the_adaptive_step(orc):
    """Following a recorded schedule: fed the accept/reject sequence that the independent driver
    above records for the oracle's own adaptive run, orc_follow reproduces that run bitwise
    (state, status, level, schedule hash): an accepted attempt is the same Newton iteration
    sequence to the same converged iterate, a rejected one is skipped.  A schedule cut short
    (the other side failed the cell) leaves the input state with status 2, and a truncated
    record is refused (-2)."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(93, 64, m.ns, 1.0)
    e0 = om.energy_batch(st.T, st.Y)
    opts = orc.default_opts()
    T1, Y1, s1, l1, i1, h1 = om.advance(st.rho, st.T, st.Y, 1e-6, e0=e0, with_sched=True)
    recs = []
    for c in range(st.n):
        controller_reference(orc, om, st.rho[c], e0[c], np.r_[st.Y[:, c], st.T[c]], 1e-6, opts)
        recs.append(pack_schedule(controller_reference.outcomes, 8))
    trace = np.array(recs)
    assert (trace[:, 0] > 1).sum() >= 8
    T2, Y2, s2, l2, i2, h2 = om.follow(st.rho, st.T, st.Y, 1e-6, e0, trace)
    assert np.array_equal(s2, s1) and np.array_equal(l2, l1) and np.array_equal(h2, h1)
    assert np.array_equal(T2, T1) and np.array_equal(Y2, Y1)
    assert np.all(i2 <= i1)  # rejected attempts cost nothing when followed
    cut = trace.copy()
    cut[:, 0] = np.maximum(cut[:, 0].astype(np.int64) - 1, 0).astype(np.uint64)
    T3, Y3, s3 = om.follow(st.rho, st.T, st.Y, 1e-6, e0, cut)[:3]
    assert np.all(s3 == 2) and np.array_equal(T3, st.T) and np.array_equal(Y3, st.Y)
    short = np.array([pack_schedule([True] * 70, 2)] * 2)
    assert np.all(om.follow(st.rho[:2], st.T[:2], st.Y[:, :2], 1e-6, e0[:2], short)[2] == -2)


# ---------------------------------------------------------------------------------------------
# Arrhenius rate and equilibrium constant in 50-digit arithmetic (Sec. 3.2)
# ---------------------------------------------------------------------------------------------

D = decimal.Decimal


def _nasa_dec(a, T):
    """h/RT and s/R of one NASA-7 set at T, in decimal."""
    a1, a2, a3, a4, a5, a6, a7 = (D(float(v)) for v in a)
    h = a1 + a2 * T / 2 + a3 * T ** 2 / 3 + a4 * T ** 3 / 4 + a5 * T ** 4 / 5 + a6 / T
    s = a1 * T.ln() + a2 * T + a3 * T ** 2 / 2 + a4 * T ** 3 / 3 + a5 * T ** 4 / 4 + a7
    return h, s


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_rate_constants_against_50_digit_evaluation(orc, name):
    """k_f = A T^b exp(-Ta/T) and k_b = k_f / K_c with K_c = (P_a/(R T))^(sum nu) exp(-dG/RT),
    evaluated in 50-digit decimal from the exact binary inputs, against the oracle's FP64 values.
    Bound: a few units of rounding of the exponent's terms, eps (3 + |b ln T| + Ta/T) for k_f and
    in addition eps (sum |nu (h/RT - s/R)| + |sum nu ln(P_a/(RT))|) for k_b."""
    m = synth.mechanism(name)
    om = orc.OracleMech(m)
    ctx = decimal.Context(prec=50)
    decimal.setcontext(ctx)
    Pa, R = D("1.01325e6"), D("8.31446261815324e7")
    worst_f = worst_b = 0.0
    for Tf in (812.5, 1000.0, 1733.3, 2950.0, 4400.0):
        T = D(Tf)
        r = om.rates(0.2, np.full(m.ns, 1.0 / m.ns), Tf)
        g = []
        for s in range(m.ns):
            h, sR = _nasa_dec(m.nasa[s, 0 if Tf < m.T_mid[s] else 1], T)
            g.append((h, sR))
        for k in range(m.nr):
            b, Ta = D(float(m.b[k])), D(float(m.Ta[k]))
            kf = D(float(m.A[k])) * (b * T.ln()).exp() * (-Ta / T).exp()
            errf = abs(D(float(r["kf"][k])) / kf - 1)
            bound_f = EPS * (3 + abs(float(m.b[k]) * math.log(Tf)) + float(m.Ta[k]) / Tf)
            assert float(errf) <= bound_f, (k, float(errf), bound_f)
            worst_f = max(worst_f, float(errf) / bound_f)
            if not m.reversible[k]:
                assert r["kb"][k] == 0.0
                continue
            dnu, dG, scale = 0, D(0), 0.0
            for idx, nu, sign in ((m.prod_idx[k], m.prod_nu[k], 1), (m.reac_idx[k], m.reac_nu[k], -1)):
                for s, v in zip(idx, nu):
                    if s >= 0:
                        dnu += sign * int(v)
                        term = D(sign * int(v)) * (g[s][0] - g[s][1])
                        dG += term
                        scale += abs(float(g[s][0])) * v + abs(float(g[s][1])) * v
            lnPRT = (Pa / (R * T)).ln()
            Kc = (D(dnu) * lnPRT - dG).exp()
            kb = kf / Kc
            errb = abs(D(float(r["kb"][k])) / kb - 1)
            bound_b = bound_f + EPS * 4 * (scale + abs(dnu * float(lnPRT)) + 1)
            assert float(errb) <= bound_b, (k, float(errb), bound_b)
            worst_b = max(worst_b, float(errb) / bound_b)
    print(f"\n[{name}] worst error / bound: k_f {worst_f:.3f}, k_b {worst_b:.3f}")
