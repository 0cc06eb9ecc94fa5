"""Pins of the FP64 CPU oracle against mathematics that does not depend on its code:
closed forms, conservation laws, detailed balance at a constructed equilibrium, finite
differences, LAPACK's getrf/getrs and the exact backward-Euler step of a linear isomerisation.
Each test names the passage of the paper (Sec. 3.2 unless stated) whose quantity it pins."""
import math

import numpy as np
import pytest
import scipy.linalg

from paper_1110_4903_amd import synth

RU = 8.31446261815324
PATM_CGS = 1.01325e6
RU_CGS = RU * 1e7


# ---------------------------------------------------------------------------------------------
# Small hand mechanisms
# ---------------------------------------------------------------------------------------------

def nasa_const(cp_R, hf_R, s_R, T0=298.15):
    """NASA-7 set of a species with constant cp/R: h/R(T0) = hf_R, s/R(T0) = s_R."""
    a6 = hf_R - cp_R * T0
    a7 = s_R - cp_R * math.log(T0)
    row = [cp_R, 0, 0, 0, 0, a6, a7]
    return [row, row]


def isomer_mech(k_f, K):
    """A <=> B with identical composition, a1..a6 equal and a7 differing by ln K, so the
    equilibrium constant is exactly K at every T and u_A = u_B (T stays constant)."""
    a = nasa_const(3.5, -1000.0, 30.0)
    b = [list(r) for r in a]
    for r in b:
        r[6] += math.log(K)
    return synth.mechanism_from_lists(
        "iso", ("H",), [[2], [2]], [a, b],
        [dict(reac=[(0, 1)], prod=[(1, 1)], A=k_f, b=0.0, Ta=0.0)])


def tb_mech(eff_row, A=1e12, b=0.3, Ta=5000.0):
    """2 H (+M) <=> H2 plus an inert N2, used for third-body properties."""
    nas = [nasa_const(2.5, 26000.0, 14.0), nasa_const(3.5, 0.0, 16.0), nasa_const(3.5, 0.0, 23.0)]
    return synth.mechanism_from_lists(
        "tb", ("H", "N"), [[1, 0], [2, 0], [0, 2]], nas,
        [dict(reac=[(0, 2)], prod=[(1, 1)], A=A, b=b, Ta=Ta, tb=0)], eff=[eff_row])


def cells(mech, n, seed, alpha=1.0):
    return synth.uniform_cells(seed, n, mech.ns, alpha)


# ---------------------------------------------------------------------------------------------
# Thermodynamics (NASA-7 polynomials feeding the equilibrium constant)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_thermo_identities(orc, name):
    """cp = dh/dT and ds/dT = cp/T for every species (Richardson-extrapolated differences)."""
    om = orc.OracleMech(synth.mechanism(name))
    for T in (350.0, 900.0, 1700.0, 2900.0, 4800.0):
        cp, hRT, sR, dcp = om.thermo(T)

        def H(t):  # h/R
            return om.thermo(t)[1] * t

        def S(t):
            return om.thermo(t)[2]

        def CP(t):
            return om.thermo(t)[0]

        def rich(F, t, d):
            d1 = (F(t + d) - F(t - d)) / (2 * d)
            d2 = (F(t + d / 2) - F(t - d / 2)) / d
            return (4 * d2 - d1) / 3

        d = 1e-2 * T
        np.testing.assert_allclose(rich(H, T, d), cp, rtol=1e-10)
        np.testing.assert_allclose(rich(S, T, d), cp / T, rtol=1e-8)
        np.testing.assert_allclose(rich(CP, T, d), dcp, rtol=1e-8, atol=1e-12)


def test_thermo_closed_form(orc):
    """Constant-cp species: h/R = hf/R + cp/R (T - T0), s/R = s0/R + cp/R ln(T/T0)."""
    m = tb_mech([1.0, 1.0, 1.0])
    om = orc.OracleMech(m)
    for T in (298.15, 1000.0, 2500.0):
        cp, hRT, sR, dcp = om.thermo(T)
        hf = np.array([26000.0, 0.0, 0.0])
        s0 = np.array([14.0, 16.0, 23.0])
        c = np.array([2.5, 3.5, 3.5])
        np.testing.assert_allclose(hRT * T, hf + c * (T - 298.15), rtol=1e-13, atol=1e-9)
        np.testing.assert_allclose(sR, s0 + c * np.log(T / 298.15), rtol=1e-13)
        np.testing.assert_allclose(cp, c, rtol=0)
        assert np.all(dcp == 0)


def test_thermo_range_selection(orc):
    """The low set applies below T_mid and the high set at and above it."""
    lo = nasa_const(3.0, 0.0, 20.0)[0]
    hi = nasa_const(5.0, 100.0, 30.0)[0]
    m = synth.mechanism_from_lists("rng", ("H",), [[1], [2]], [[lo, hi], [lo, lo]],
                                   [dict(reac=[(0, 2)], prod=[(1, 1)], A=1.0)])
    om = orc.OracleMech(m)
    assert om.thermo(999.0)[0][0] == 3.0
    assert om.thermo(1000.0)[0][0] == 5.0
    assert om.thermo(1000.0)[0][1] == 3.0


# ---------------------------------------------------------------------------------------------
# Rates: Arrhenius, equilibrium constant, third body, production
# ---------------------------------------------------------------------------------------------

def test_arrhenius_properties(orc):
    """K_f = A T^beta exp(-E/RT): the Arrhenius plot of a beta = 0 reaction has slope -Ta
    exactly, a Ta = 0 reaction scales as T^beta, and beta = Ta = 0 gives K_f = A."""
    for (A, b, Ta) in ((3.7e11, 0.0, 12345.0), (2.0e9, 1.3, 0.0), (5.5e12, 0.0, 0.0)):
        m = synth.mechanism_from_lists("arr", ("H",), [[1], [2]],
                                       [nasa_const(2.5, 0, 20), nasa_const(3.5, 0, 25)],
                                       [dict(reac=[(0, 2)], prod=[(1, 1)], A=A, b=b, Ta=Ta)])
        om = orc.OracleMech(m)
        k1 = om.rates(0.1, [0.5, 0.5], 1200.0)["kf"][0]
        k2 = om.rates(0.1, [0.5, 0.5], 2400.0)["kf"][0]
        if b == 0 and Ta:
            assert abs(math.log(k2 / k1) - Ta * (1 / 1200.0 - 1 / 2400.0)) < 1e-12 * Ta / 1200
        elif Ta == 0 and b:
            assert abs(k2 / k1 - 2.0 ** b) < 1e-14 * 2.0 ** b
        else:
            assert k1 == A and k2 == A


def _equilibrium_state(om, mech, T, seed):
    """Composition satisfying detailed balance for every element-balanced reaction:
    c_s = (P_a/RT) exp(-g_s/RT + sum_e a_es lambda_e) for arbitrary lambda_e."""
    cp, hRT, sR, _ = om.thermo(T)
    g = hRT - sR
    rng = np.random.default_rng(seed)
    target = rng.uniform(-3, 0, size=mech.ns)
    lam, *_ = np.linalg.lstsq(mech.comp.astype(float), g + target, rcond=None)
    c = PATM_CGS / (RU_CGS * T) * np.exp(-g + mech.comp @ lam)
    rho_cgs = float(np.sum(c * mech.M))
    Y = c * mech.M / rho_cgs
    return rho_cgs * 1e3, Y


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_detailed_balance(orc, name):
    """K_e = K_f/K_b = (P_a/RT)^(sum nu) exp(-dG0/RT): at a constructed equilibrium the
    forward and backward progress of every reversible reaction are equal."""
    mech = synth.mechanism(name)
    om = orc.OracleMech(mech)
    for T, seed in ((1100.0, 1), (2300.0, 2), (3700.0, 3)):
        rho, Y = _equilibrium_state(om, mech, T, seed)
        r = om.rates(rho, Y, T)
        rev = mech.reversible == 1
        qf, qb = r["qf"][rev], r["qb"][rev]
        assert np.all(qf > 0)
        np.testing.assert_allclose(qb, qf, rtol=2e-12)
        assert np.all(r["kb"][~rev] == 0)


@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_production_conserves_mass_and_elements(orc, name):
    """sum_s M_s wdot_s = 0 (Sec. 3.2) and, per element, sum_s a_es wdot_s = 0."""
    mech = synth.mechanism(name)
    om = orc.OracleMech(mech)
    st = cells(mech, 16, 7, 0.7)
    for i in range(st.n):
        r = om.rates(st.rho[i], st.Y[:, i], st.T[i])
        w = r["wdot"]
        scale = np.zeros(mech.ns)
        for k in range(mech.nr):
            for j in range(3):
                for idx in (mech.reac_idx[k, j], mech.prod_idx[k, j]):
                    if idx >= 0:
                        scale[idx] += 2 * abs(r["q"][k])
        assert abs(np.sum(mech.M * w)) <= 1e-13 * np.sum(mech.M * scale)
        for e in range(mech.ne):
            a = mech.comp[:, e].astype(float)
            assert abs(np.sum(a * w)) <= 1e-13 * np.sum(a * scale) + 1e-300


def test_third_body_properties(orc):
    """[M] = sum_s alpha_s X_s multiplies the net progress: with unit efficiencies it equals
    the total concentration, and doubling every efficiency doubles the rate."""
    st = synth.uniform_cells(5, 4, 3, 1.0)
    for i in range(st.n):
        rho, Y, T = st.rho[i], st.T[i], st.Y[:, i]
        Y, T = st.Y[:, i], st.T[i]
        m1 = orc.OracleMech(tb_mech([1.0, 1.0, 1.0]))
        m2 = orc.OracleMech(tb_mech([2.0, 2.0, 2.0]))
        r1 = m1.rates(rho, Y, T)
        r2 = m2.rates(rho, Y, T)
        ctot = float(np.sum(rho * 1e-3 * Y / m1.mech.M))
        assert abs(r1["M"][0] - ctot) <= 1e-15 * ctot
        assert abs(r2["q"][0] - 2 * r1["q"][0]) <= 1e-14 * abs(r1["q"][0])
        # an inert species with zero efficiency does not collide
        m0 = orc.OracleMech(tb_mech([1.0, 1.0, 0.0]))
        c = rho * 1e-3 * Y / m0.mech.M
        assert abs(m0.rates(rho, Y, T)["M"][0] - (c[0] + c[1])) <= 1e-15 * ctot


# ---------------------------------------------------------------------------------------------
# Jacobian
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_jacobian_matches_finite_differences(orc, name):
    """Analytic (Ns+1)^2 Jacobian of the source term vs central differences of the oracle's
    own right-hand side, column by column."""
    mech = synth.mechanism(name)
    om = orc.OracleMech(mech)
    st = cells(mech, 12, 11, 1.0)
    for i in range(st.n):
        x = np.r_[st.Y[:, i], st.T[i]]
        J = om.jacobian(st.rho[i], x)
        Jf = om.jacobian(st.rho[i], x, fd=True)
        row = np.abs(J).max(1, keepdims=True)
        err = np.abs(J - Jf)
        assert np.all(err <= 1e-5 * np.abs(J) + 1e-8 * row), (err / (np.abs(J) + row)).max()


def test_jacobian_third_body(orc):
    om = orc.OracleMech(tb_mech([0.7, 2.5, 1.3]))
    st = synth.uniform_cells(9, 5, 3, 1.0)
    for i in range(st.n):
        x = np.r_[st.Y[:, i], st.T[i]]
        J = om.jacobian(st.rho[i], x)
        Jf = om.jacobian(st.rho[i], x, fd=True)
        np.testing.assert_allclose(J, Jf, rtol=1e-6, atol=1e-7 * np.abs(J).max())


# ---------------------------------------------------------------------------------------------
# Gaussian elimination with partial pivoting (Sec. 3.2 / Sec. 4.2) vs LAPACK getrf/getrs
# ---------------------------------------------------------------------------------------------

def test_lu_matches_lapack(orc):
    rng = np.random.default_rng(3)
    mats = [rng.normal(size=(n, n)) for n in (1, 2, 5, 10, 37)]
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    st = cells(mech, 3, 4)
    for i in range(st.n):  # stiff Newton matrices I - h J
        x = np.r_[st.Y[:, i], st.T[i]]
        mats.append(np.eye(mech.ns + 1) - 1e-6 * om.jacobian(st.rho[i], x))
    for A in mats:
        n = A.shape[0]
        b = rng.normal(size=n)
        rc, LU, piv = orc.lu_factor(A)
        assert rc == 0
        lu_ref, piv_ref = scipy.linalg.lu_factor(A)
        assert np.array_equal(piv, piv_ref)
        np.testing.assert_allclose(LU, lu_ref, rtol=1e-12, atol=1e-13 * np.abs(lu_ref).max())
        x = orc.lu_solve(LU, piv, b)
        x_ref = scipy.linalg.lu_solve((lu_ref, piv_ref), b)
        np.testing.assert_allclose(x, x_ref, rtol=1e-11, atol=1e-12 * np.abs(x_ref).max())


def test_lu_zero_pivot(orc):
    A = np.array([[1.0, 2.0, 0.0], [3.0, 4.0, 0.0], [5.0, 6.0, 0.0]])
    rc, _, _ = orc.lu_factor(A)
    assert rc == -1
    rc, _, _ = orc.lu_factor(np.zeros((4, 4)))
    assert rc == -1


# ---------------------------------------------------------------------------------------------
# Backward Euler + Newton on closed-form problems
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("kf,K,dt", [(1e3, 2.0, 1e-4), (1e9, 0.3, 1e-6), (1e14, 5.0, 1e-6)])
def test_isomer_backward_euler_closed_form(orc, kf, K, dt):
    """A <=> B: one backward-Euler step has the exact solution
    Y_A = Y_eq + (Y_A0 - Y_eq)/(1 + (k_f + k_b) dt), Y_eq = k_b/(k_f + k_b), k_b = k_f/K.
    The system is linear, so Newton reaches it without halving and T does not move."""
    m = isomer_mech(kf, K)
    om = orc.OracleMech(m)
    rho = np.array([0.3, 0.05, 1.0])
    T = np.array([1500.0, 900.0, 2500.0])
    Y = np.array([[0.9, 0.2, 0.5], [0.1, 0.8, 0.5]])
    T1, Y1, st, lv, it = om.advance(rho, T, Y, dt)
    assert np.all(st == 0) and np.all(lv == 0)
    kb = kf / K
    yeq = kb / (kf + kb)
    yA = yeq + (Y[0] - yeq) / (1 + (kf + kb) * dt)
    np.testing.assert_allclose(Y1[0], yA, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Y1[0] + Y1[1], 1.0, rtol=0, atol=2e-16)
    np.testing.assert_allclose(T1, T, rtol=1e-14)


def test_isomer_first_order_convergence(orc):
    """2^L equal backward-Euler sub-steps converge to exp(-(k_f + k_b) t) at first order."""
    kf, K, dt = 1e6, 1.5, 2e-6
    m = isomer_mech(kf, K)
    om = orc.OracleMech(m)
    kb = kf / K
    yeq = kb / (kf + kb)
    y0 = 0.95
    exact = yeq + (y0 - yeq) * math.exp(-(kf + kb) * dt)
    errs = []
    for L in range(4, 10):
        _, Y1, st, lv, _ = om.advance(np.array([0.2]), np.array([1500.0]),
                                      np.array([[y0], [1 - y0]]), dt, L_forced=L)
        assert st[0] in (0, 1) and lv[0] == L
        errs.append(abs(Y1[0, 0] - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.1), ratios


def test_replay_equals_explicit_substeps(orc):
    """A forced level L is bitwise 2^L consecutive single steps of dt/2^L."""
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    st = cells(mech, 8, 21)
    dt, L = 1e-7, 2
    e0 = om.energy_batch(st.T, st.Y)
    Ta, Ya, sa, la, _ = om.advance(st.rho, st.T, st.Y, dt, e0=e0, L_forced=L)
    T, Y = st.T.copy(), st.Y.copy()
    ok = np.ones(st.n, bool)
    for _ in range(1 << L):
        T, Y, s, _, _ = om.advance(st.rho, T, Y, dt / (1 << L), e0=e0, L_forced=0)
        ok &= s < 2
    assert np.array_equal(sa < 2, ok)
    assert np.array_equal(Ta[ok], T[ok]) and np.array_equal(Ya[:, ok], Y[:, ok])


def test_equilibrium_is_fixed_point(orc):
    """A backward-Euler step from a detailed-balance state leaves it unchanged."""
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    for T, seed in ((1300.0, 4), (2600.0, 5)):
        rho, Y = _equilibrium_state(om, mech, T, seed)
        T1, Y1, st, lv, it = om.advance(np.array([rho]), np.array([T]), Y.reshape(-1, 1), 1e-6)
        assert st[0] == 0 and lv[0] == 0 and it[0] <= 2
        np.testing.assert_allclose(Y1[:, 0], Y, rtol=1e-12, atol=1e-25)
        assert abs(T1[0] - T) <= 1e-12 * T


# ---------------------------------------------------------------------------------------------
# Whole step: conservation, residual, temperature inversion, control
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,n", [("mech9", 64), ("mech36", 8)])
def test_whole_step_invariants(orc, name, n):
    """Element mass, total mass fraction and internal energy are conserved by a step."""
    mech = synth.mechanism(name)
    om = orc.OracleMech(mech)
    st = cells(mech, n, 31, 1.0 if name == "mech9" else 0.5)
    e0 = om.energy_batch(st.T, st.Y)
    T1, Y1, s, lv, it = om.advance(st.rho, st.T, st.Y, 1e-6)
    assert np.all(s < 2)
    elem_in = (mech.comp.T.astype(float) @ (st.Y / mech.M[:, None]))
    elem_out = (mech.comp.T.astype(float) @ (Y1 / mech.M[:, None]))
    np.testing.assert_allclose(elem_out, elem_in, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(Y1.sum(0), st.Y.sum(0), rtol=0, atol=1e-13)
    e1 = om.energy_batch(T1, Y1)
    np.testing.assert_allclose(e1, e0, rtol=1e-12, atol=1e-9 * np.abs(e0).max())


def test_newton_root_residual_long_double(orc):
    """The converged Newton iterate of a sub-step solves the backward-Euler equations
    G = x - x_prev - h f(x) = 0: re-evaluated in long double, every species row is at
    rounding level relative to its term scale and the temperature row within tolerance."""
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    st = cells(mech, 64, 41)
    h = 1e-6
    checked = 0
    for i in range(st.n):
        xp = np.r_[st.Y[:, i], st.T[i]]
        e0 = om.energy(st.Y[:, i], st.T[i])
        rc, x, it, xbe = om.be_substep(st.rho[i], e0, xp, h)
        if rc != 0:
            continue
        _, G = om.residual(st.rho[i], xp, xbe, h)
        S = om.term_scale(st.rho[i], st.Y[:, i], xbe, h)
        assert np.all(np.abs(G[:-1]) <= 1e-12 * S), (np.abs(G[:-1]) / S).max()
        assert abs(G[-1]) <= 1e-9 * xbe[-1]
        # the temperature inversion keeps Y and restores e(Y, T) = e0
        assert np.array_equal(x[:-1], xbe[:-1])
        assert abs(om.energy(x[:-1], x[-1]) - e0) <= 1e-12 * abs(e0) + 1e-6
        checked += 1
    assert checked >= 20


def test_temperature_inversion(orc):
    """e(Y, T_out) = e0 to 1e-13, from near and far starting points; no root -> failure."""
    mech = synth.mechanism("mech36")
    om = orc.OracleMech(mech)
    st = cells(mech, 5, 51, 0.5)
    for i in range(st.n):
        Y = st.Y[:, i]
        e0 = om.energy(Y, st.T[i])
        for T0 in (st.T[i] * 1.001, 250.0, 5900.0):
            rc, T = om.invert_T(Y, e0, T0)
            assert rc == 0
            assert abs(om.energy(Y, T) - e0) <= 1e-13 * abs(e0) + 1e-6
            assert abs(T - st.T[i]) <= 1e-11 * st.T[i]
        rc, _ = om.invert_T(Y, om.energy(Y, 6500.0), 3000.0)
        assert rc != 0


def test_control_paths(orc):
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    st = cells(mech, 16, 61)
    # k_max = 1 can never verify convergence away from equilibrium: every level fails and
    # the cell keeps its input state.
    o = orc.make_opts(k_max=1, L_max=4)
    T1, Y1, s, lv, it = om.advance(st.rho, st.T, st.Y, 1e-6, opts=o)
    assert np.all(s == 2) and np.all(lv == 4)
    assert np.array_equal(T1, st.T) and np.array_equal(Y1, st.Y)
    assert np.all(it == 5)  # one iteration per level 0..4
    # invalid inputs are rejected untouched
    T = st.T.copy()
    T[0] = np.nan
    T[1] = 100.0
    rho = st.rho.copy()
    rho[2] = -1.0
    T1, Y1, s, lv, it = om.advance(rho, T, st.Y, 1e-6)
    assert list(s[:3]) == [3, 3, 3] and np.all(s[3:] < 2)
    assert np.isnan(T1[0]) and T1[1] == 100.0 and np.array_equal(Y1[:, :3], st.Y[:, :3])


def test_adaptive_levels_reported(orc):
    """Cells that needed halving report status 1 and a level >= 1; the rest status 0, level 0."""
    mech = synth.mechanism("mech9")
    om = orc.OracleMech(mech)
    st = cells(mech, 128, 71)
    _, _, s, lv, it = om.advance(st.rho, st.T, st.Y, 1e-6)
    assert np.all((s == 0) == (lv == 0))
    assert np.all(it[s == 0] <= 10)
    assert (s == 1).sum() > 0 and (s == 0).sum() > 0


# ---------------------------------------------------------------------------------------------
# Point-implicit step (Sec. 3.2, Eq. "kinetics"): one linearised backward-Euler step over dt
# ---------------------------------------------------------------------------------------------

def test_point_implicit_isomer_is_exact_backward_euler(orc):
    """A <=> B is linear in Y with T fixed, so the single linearised step is the exact
    backward-Euler step x_A = x_eq + (x_A,n - x_eq) / (1 + (k_f + k_b) dt)."""
    kf, K, dt = 2e8, 0.7, 3e-6
    m = isomer_mech(kf, K)
    om = orc.OracleMech(m)
    Y = np.array([[0.85, 0.1], [0.15, 0.9]])
    rho, T = np.array([0.4, 0.02]), np.array([1200.0, 2400.0])
    T1, Y1, st, lv, it = om.advance(rho, T, Y, dt, opts=orc.make_opts(point_implicit=1))
    assert list(st) == [0, 0] and list(lv) == [0, 0] and list(it) == [1, 1]
    kb = kf / K
    yeq = kb / (kf + kb)
    np.testing.assert_allclose(Y1[0], yeq + (Y[0] - yeq) / (1 + (kf + kb) * dt), rtol=1e-13)
    np.testing.assert_allclose(T1, T, rtol=1e-13)


def test_point_implicit_is_one_linear_solve(orc):
    """On the 9-species mechanism, the point-implicit Y equals Y_n + dx with
    (I - dt J(x_n)) dx = dt f(x_n) solved by LAPACK (J and f from the pinned oracle routines);
    T is then set by the energy inversion, e(Y, T) = e0."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(17, 24, m.ns, 1.0)
    dt = 1e-7
    e0 = om.energy_batch(st.T, st.Y)
    T1, Y1, s1, l1, i1 = om.advance(st.rho, st.T, st.Y, dt, e0=e0, opts=orc.make_opts(point_implicit=1))
    assert np.all(l1 == 0) and np.all(i1 == 1)
    N = m.ns + 1
    for c in range(st.n):
        x = np.r_[st.Y[:, c], st.T[c]]
        f = om.rhs(st.rho[c], x)
        J = om.jacobian(st.rho[c], x)
        dx = scipy.linalg.solve(np.eye(N) - dt * J, dt * f)
        if s1[c] == 0:
            np.testing.assert_allclose(Y1[:, c], x[:-1] + dx[:-1], rtol=1e-10, atol=1e-14)
            assert abs(om.energy(Y1[:, c], T1[c]) - e0[c]) <= 1e-12 * abs(e0[c])
        else:
            assert s1[c] == 2 and np.array_equal(Y1[:, c], st.Y[:, c])
    assert np.mean(s1 == 0) > 0.5


def test_divergence_test_saves_iterations_and_keeps_invariants(orc):
    """Abandoning attempts whose update norm grows (diverge_ratio = 2, the default) changes the
    sub-step schedule but every accepted result is still a backward-Euler step: mass and
    element conservation and e(Y, T) = e0 hold, and fewer Newton iterations are spent than with
    the test disabled."""
    m = synth.mechanism("mech36")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(2, 40, m.ns, 0.5)
    e0 = om.energy_batch(st.T, st.Y)
    T1, Y1, s1, l1, i1 = om.advance(st.rho, st.T, st.Y, 1e-6, e0=e0)
    T0, Y0, s0, l0, i0 = om.advance(st.rho, st.T, st.Y, 1e-6, e0=e0, opts=orc.make_opts(diverge_ratio=0.0))
    assert np.all(s1 < 2) and np.all(s0 < 2)
    assert i1.sum() < 0.85 * i0.sum()
    comp = np.asarray(m.comp, dtype=float)
    M = np.asarray(m.M)
    for Y in (Y1, Y0):
        np.testing.assert_allclose(Y.sum(0), st.Y.sum(0), rtol=0, atol=1e-12)
        el0 = comp.T @ (st.Y / M[:, None])
        el1 = comp.T @ (Y / M[:, None])
        np.testing.assert_allclose(el1, el0, rtol=1e-11, atol=1e-14)
    for c in range(st.n):
        assert abs(om.energy(Y1[:, c], T1[c]) - e0[c]) <= 1e-12 * abs(e0[c])


# ---------------------------------------------------------------------------------------------
# Operator-split adapter (Sec. 2: the energy equation leaves out the formation energies, and
# the chemistry source must carry their change; operator-splitting equation)
# ---------------------------------------------------------------------------------------------

R_J = 8.31446261815324e3  # J/(kmol K), with molar masses in g/mol = kg/kmol


def test_sensible_energy_is_cv_integral(orc):
    """One species at T: E_sens / rho equals the integral of c_v from 298.15 K to T, computed
    by adaptive quadrature of the NASA-7 cp (independent of the closed-form energy)."""
    from scipy.integrate import quad
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    unit = np.eye(m.ns)
    for s in range(m.ns):
        cv = lambda T: R_J / m.M[s] * (om.thermo(T)[0][s] - 1.0)
        for T in (500.0, 1500.0, 2800.0, 4500.0):
            ref, _ = quad(cv, orc.T_REF, T, points=[m.T_mid[s]] if T > m.T_mid[s] else None,
                          epsabs=0.0, epsrel=1e-13, limit=200)
            rho = 0.37
            E = om.to_conserved(np.array([rho]), unit[s][:, None], np.array([om.energy(unit[s], T)]))[1][0]
            assert abs(E / rho - ref) <= 1e-11 * abs(ref), (s, T)


def test_conserved_round_trip(orc):
    """(rho, Y, T) -> (rho_s, E_sens) -> (rho, Y, T) on config 0's states: partial densities
    sum to rho and the inversion recovers T to 1e-12 relative."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(31, 200, m.ns, 1.0)
    e0 = om.energy_batch(st.T, st.Y)
    rho_s, E = om.to_conserved(st.rho, st.Y, e0)
    np.testing.assert_allclose(rho_s.sum(0), st.rho, rtol=1e-15)
    rho, Y, T, e1, ok = om.from_conserved(rho_s, E, T_guess=np.full(st.n, 2000.0))
    assert ok.all()
    np.testing.assert_allclose(rho, st.rho, rtol=1e-15)
    np.testing.assert_allclose(Y, st.Y, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(T, st.T, rtol=1e-12)
    np.testing.assert_allclose(e1, e0, rtol=1e-13)


def two_species_heat_release(dh_R):
    """A <=> B with equal constant cp/R = 3.5 and equal molar mass; B's formation enthalpy is
    lower by dh_R (K), so A -> B releases dh_R R per unit of moles converted."""
    a = nasa_const(3.5, 1000.0, 30.0)
    b = nasa_const(3.5, 1000.0 - dh_R, 28.0)
    return synth.mechanism_from_lists("heat", ("H",), [[2], [2]], [a, b],
                                      [dict(reac=[(0, 1)], prod=[(1, 1)], A=2e6, b=0.0, Ta=0.0)])


def test_conserved_constant_cp_closed_form(orc):
    """With constant cp, E_sens = sum rho_s c_v,s (T - T_ref); the inversion must return
    T = T_ref + E_sens / sum rho_s c_v,s."""
    m = two_species_heat_release(3000.0)
    om = orc.OracleMech(m)
    cv = R_J / m.M * (3.5 - 1.0)
    rho_s = np.array([[0.2, 0.01, 0.7], [0.05, 0.3, 0.0]])
    E = np.array([3.0e5, 2.5e6, 9.0e5])
    rho, Y, T, e0, ok = om.from_conserved(rho_s, E)
    assert ok.all()
    np.testing.assert_allclose(T, orc.T_REF + E / (cv @ rho_s), rtol=1e-12)


def test_formation_energy_source(orc):
    """Exothermic A -> B over one step from the conserved state: mass and the total energy
    E_sens + sum rho_s e_s(T_ref) are unchanged, E_sens rises by the formation energy released,
    (rho_A - rho_A') (e_A(T_ref) - e_B(T_ref)), and the new T is the constant-cp closed form."""
    dh = 3000.0
    m = two_species_heat_release(dh)
    om = orc.OracleMech(m)
    cv = R_J / m.M[0] * 2.5
    rho_s = np.array([[0.2, 0.9, 0.5], [0.0, 0.1, 0.5]])
    E = np.array([3.0e5, 1.2e6, 2.0e6])
    rho, Y, T, e0, ok = om.from_conserved(rho_s, E)
    T1, Y1, s1 = om.advance(rho, T, Y, 1e-6, e0=e0)[:3]
    assert np.all(s1 < 2)
    rho_s1, E1 = om.to_conserved(rho, Y1, e0)
    ef = om.formation_energies()
    np.testing.assert_allclose(ef[0] - ef[1], R_J / m.M[0] * dh, rtol=1e-12)
    np.testing.assert_allclose(rho_s1.sum(0), rho_s.sum(0), rtol=1e-14)
    np.testing.assert_allclose(E1 + ef @ rho_s1, E + ef @ rho_s, rtol=1e-13)
    released = (rho_s[0] - rho_s1[0]) * R_J / m.M[0] * dh
    assert np.all(released > 0)
    np.testing.assert_allclose(E1 - E, released, rtol=1e-9)
    np.testing.assert_allclose(T1, orc.T_REF + E1 / (rho * cv), rtol=1e-12)
