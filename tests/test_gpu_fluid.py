"""GPU parity of the fluid step (Sec. 3.1) and of the operator-split step (Sec. 2, Eq.
operator_splitting) against the FP64 oracles: the library's MP5 / HLLE / RK3 sweeps through the
C ABI against oracle/fluid_oracle.py on the same 2-D grids (periodic and transmissive), and one
split step (fluid step, then the chemistry sub-step through the conserved-variable adapter)
against the fluid oracle followed by the kinetics oracle.  Gate: 1e-10 of each conserved
variable's scale (its largest magnitude on the grid) per result."""
import numpy as np
import pytest

from paper_1110_4903_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1110_4903_amd import kin
    c = kin.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def fo():
    from oracle import fluid_oracle
    return fluid_oracle


def flow_state(fo, gas, nx, ny, seed, T_lo=900.0, T_hi=2600.0):
    """A hot pressure pulse in a sheared flow over a seeded mixture (primitive variables built
    here, the conserved state by the oracle's own conversion)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Yg = np.meshgrid(x, y)
    r2 = (X - 0.35) ** 2 + (Yg - 0.6) ** 2
    T = T_lo + (T_hi - T_lo) * np.exp(-r2 / 0.02)
    P = 1e5 * (1 + 1.5 * np.exp(-r2 / 0.01))
    Y = rng.dirichlet(np.ones(gas.ns), size=(ny, nx)).transpose(2, 0, 1)
    Rmix = (Y * gas.Rs[:, None, None]).sum(0)
    rho = P / (Rmix * T)
    u = 80.0 * np.sin(2 * np.pi * Yg)
    v = -60.0 * np.cos(2 * np.pi * X)
    W = np.concatenate([Y * rho[None], u[None], v[None], P[None]])
    return fo.to_conserved(gas, W)[0]


def var_scale(b, reduce=np.max):
    """Scale of each conserved variable over the grid (largest magnitude, or another reduction);
    the two momentum components share one (either may be zero everywhere)."""
    s = reduce(np.abs(b).reshape(b.shape[0], -1), axis=1)
    ns = b.shape[0] - 3
    s[ns] = s[ns + 1] = max(s[ns], s[ns + 1])
    return s


def scaled_diff(a, b):
    """max over cells of |a - b| / (the variable's scale), per variable."""
    return np.abs(a - b).reshape(b.shape[0], -1).max(1) / var_scale(b)


@pytest.mark.parametrize("bc", [0, 1])
def test_fluid_steps_against_oracle(ctx, fo, bc):
    """Two split steps (x then y, then y then x) of the 9-species mixture on a 40 x 33 grid
    (ragged against any tile), periodic or transmissive: every conserved variable of every cell
    within 1e-10 of its scale; the CFL step sizes agree to 1e-12."""
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    gas = fo.Gas(m)
    nx, ny, dx, dy = 40, 33, 1e-3 / 40, 1e-3 / 33
    Q = flow_state(fo, gas, nx, ny, 5)
    mid = ctx.mech_upload(m)
    fid = ctx.fluid_create(mid, nx, ny, dx, dy, bc)
    ctx.fluid_upload(fid, np.ascontiguousarray(Q))
    dt_g = ctx.fluid_max_dt(fid, 0.4)
    bcn = "periodic" if bc == 0 else "outflow"
    dt_o = fo.max_dt(gas, Q, dx, dy, 0.4)
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o, (dt_g, dt_o)
    Qo = Q.copy()
    for k in range(2):
        ctx.fluid_step(fid, dt_o, y_first=bool(k))
        Qo = fo.fluid_step(gas, Qo, dt_o, dx, dy, bcn, y_first=bool(k))
    Qg = ctx.fluid_download(fid)
    d = scaled_diff(Qg, Qo)
    print(f"\n[fluid bc={bcn}] dt={dt_o:.3e} max scaled diff per variable {np.array2string(d, precision=2)}", flush=True)
    assert np.all(d <= 1e-10), d
    assert np.abs(Qg - Q).max() > 0
    ctx.fluid_release(fid)
    ctx.mech_release(mid)


@pytest.mark.parametrize("which", ["gen14", "mech36"])
def test_fluid_step_other_register_classes(ctx, fo, which):
    """One fluid step (x then y) on a 24 x 20 periodic grid of a generated 14-species mixture
    (the kernels' 16-species register class) and of the 36-species mixture (face states
    streamed, no register class), against the fluid oracle: every conserved variable within
    1e-10 of its scale, the step sizes to 1e-12.  The 9-species tests take the 10-species
    class."""
    if which == "gen14":
        m = synth.make_mechanism(synth.MechRecipe("gen14", seed=714, n_elements=3, n_species=14, n_reactions=60,
                                                  frac_third_body=0.15, frac_irreversible=0.3))
    else:
        m = synth.mechanism("mech36")
    gas = fo.Gas(m)
    nx, ny = 24, 20
    dx, dy = 1e-3 / nx, 1e-3 / ny
    Q = flow_state(fo, gas, nx, ny, 11)
    mid = ctx.mech_upload(m)
    fid = ctx.fluid_create(mid, nx, ny, dx, dy, 0)
    ctx.fluid_upload(fid, np.ascontiguousarray(Q))
    dt_g = ctx.fluid_max_dt(fid, 0.4)
    dt_o = fo.max_dt(gas, Q, dx, dy, 0.4)
    assert abs(dt_g - dt_o) <= 1e-12 * dt_o, (dt_g, dt_o)
    ctx.fluid_step(fid, dt_o)
    Qo = fo.fluid_step(gas, Q, dt_o, dx, dy, "periodic")
    d = scaled_diff(ctx.fluid_download(fid), Qo)
    print(f"\n[fluid {which}] max scaled diff per variable {np.array2string(d, precision=2)}", flush=True)
    assert np.all(d <= 1e-10), d
    ctx.fluid_release(fid)
    ctx.mech_release(mid)


def test_shock_tube_on_gpu_against_oracle(ctx, fo):
    """Sod's tube in the 9-species mixture (uniform composition), transmissive, 256 x 2 cells,
    40 steps: the GPU and the oracle agree to 1e-10 of each variable's scale through the shock,
    contact and rarefaction."""
    m = synth.mechanism("mech9")
    gas = fo.Gas(m)
    nx, ny = 256, 2
    x = (np.arange(nx) + 0.5) / nx
    Yc = np.full(gas.ns, 1.0 / gas.ns)
    rho = np.where(x < 0.5, 1.0, 0.125)[None, :].repeat(ny, 0)
    P = np.where(x < 0.5, 1e5, 1e4)[None, :].repeat(ny, 0)
    W = np.concatenate([Yc[:, None, None] * rho[None], np.zeros((2, ny, nx)), P[None]])
    Q = fo.to_conserved(gas, W)[0]
    mid = ctx.mech_upload(m)
    fid = ctx.fluid_create(mid, nx, ny, 1.0 / nx, 1.0 / nx, 1)
    ctx.fluid_upload(fid, np.ascontiguousarray(Q))
    Qo = Q.copy()
    for k in range(40):
        dt = fo.max_dt(gas, Qo, 1.0 / nx, 1.0 / nx, 0.4)
        ctx.fluid_step(fid, dt, y_first=bool(k & 1))
        Qo = fo.fluid_step(gas, Qo, dt, 1.0 / nx, 1.0 / nx, "outflow", y_first=bool(k & 1))
    Qg = ctx.fluid_download(fid)
    d = scaled_diff(Qg, Qo)
    print(f"\n[shock tube] max scaled diff per variable {np.array2string(d, precision=2)}", flush=True)
    assert np.all(d <= 1e-10), d
    ctx.fluid_release(fid)
    ctx.mech_release(mid)


def test_split_step_against_oracles(ctx, orc, fo):
    """One operator-split step on a 32 x 24 grid of the 9-species mixture: the fluid step, then
    the chemistry sub-step on the same cells through the adapter, against the fluid oracle
    followed by the kinetics oracle's conversion, step and conversion back; partial densities
    and energy within 1e-10 of their scales, momenta untouched by the chemistry."""
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    gas = fo.Gas(m)
    om = orc.OracleMech(m)
    nx, ny, dx, dy = 32, 24, 1e-3 / 32, 1e-3 / 24
    Q = flow_state(fo, gas, nx, ny, 9, 1200.0, 2400.0)
    n, ns = nx * ny, m.ns
    mid = ctx.mech_upload(m)
    fid = ctx.fluid_create(mid, nx, ny, dx, dy, 0)
    ctx.fluid_upload(fid, np.ascontiguousarray(Q))
    dt = fo.max_dt(gas, Q, dx, dy, 0.4)
    st0 = synth.CellStates(np.ones(n), np.full(n, 1000.0), np.full((ns, n), 1.0 / ns))
    iid = ctx.state_upload(mid, st0.rho, st0.T, st0.Y)
    ctx.split_step(fid, iid, dt)
    Qg = ctx.fluid_download(fid)
    sched = ctx.download_schedule(iid)
    status = ctx.download(iid)[2]
    # the oracles: fluid step, then chemistry through the conversions
    Qf = fo.fluid_step(gas, Q, dt, dx, dy, "periodic")
    rho_s = Qf[:ns].reshape(ns, n)
    rho = rho_s.sum(0)
    KE = 0.5 * (Qf[ns] ** 2 + Qf[ns + 1] ** 2).reshape(n) / rho
    Es = Qf[ns + 2].reshape(n) - KE
    r, Y, T, e0, ok = om.from_conserved(rho_s, Es)
    assert ok.all()
    T1, Y1, s1, l1, i1, h1 = om.advance(r, T, Y, dt, e0=e0, with_sched=True)
    rs1, Es1 = om.to_conserved(r, Y1, e0)
    Qo = Qf.copy()
    Qo[:ns] = rs1.reshape(ns, ny, nx)
    Qo[ns + 2] = (Es1 + KE).reshape(ny, nx)
    same = (sched == h1) & (status == s1)
    d = scaled_diff(Qg, Qo)
    print(f"\n[split step] dt={dt:.3e} schedule matches {same.sum()}/{n}, max scaled diff "
          f"{np.array2string(d, precision=2)}", flush=True)
    assert same.sum() >= n - 2 and np.all(status < 2)
    assert np.all(d <= 1e-10), d
    ctx.instance_release(iid)
    ctx.fluid_release(fid)
    ctx.mech_release(mid)


def test_split_steps_cost_order_is_bitwise_neutral(ctx, fo):
    """Operator-split steps on a 512 x 512 grid (262144 cells, enough for the lane layout's cost
    order).  From the second step on, the chemistry is ordered by the previous step's iteration
    counts, which the reset from the fluid state keeps.  The same steps on a copy whose instance
    is reset before each step (so its counts are dropped and every step is ordered by the
    source-term estimate) give bitwise the same grid and the same state, status, level,
    iterations and schedule."""
    m = synth.mechanism("mech9")
    gas = fo.Gas(m)
    nx = ny = 512
    n, ns = nx * ny, m.ns
    Q = np.ascontiguousarray(flow_state(fo, gas, nx, ny, 5, 1200.0, 2400.0))
    mid = ctx.mech_upload(m)
    fa = ctx.fluid_create(mid, nx, ny, 1e-4, 1e-4, 0)
    fb = ctx.fluid_create(mid, nx, ny, 1e-4, 1e-4, 0)
    ctx.fluid_upload(fa, Q)
    ctx.fluid_upload(fb, Q)
    # both grids take the step-size query: it also refreshes the temperatures that start the
    # primitives' Newton, and those move the results by rounding
    dt = ctx.fluid_max_dt(fa, 0.4)
    assert ctx.fluid_max_dt(fb, 0.4) == dt
    st0 = synth.CellStates(np.ones(n), np.full(n, 1000.0), np.full((ns, n), 1.0 / ns))
    ia = ctx.state_upload(mid, st0.rho, st0.T, st0.Y)
    ib = ctx.state_upload(mid, st0.rho, st0.T, st0.Y)
    for k in range(3):
        ctx.split_step(fa, ia, dt, y_first=bool(k & 1))
        ctx.state_reset(ib, st0.rho, st0.T, st0.Y)
        ctx.split_step(fb, ib, dt, y_first=bool(k & 1))
    assert np.array_equal(ctx.fluid_download(fa), ctx.fluid_download(fb), equal_nan=True)
    for u, v in zip(ctx.download(ia) + (ctx.download_schedule(ia),), ctx.download(ib) + (ctx.download_schedule(ib),)):
        assert np.array_equal(u, v, equal_nan=True)
    assert np.all(ctx.download(ia)[2] < 2)
    for i in (ia, ib):
        ctx.instance_release(i)
    for f in (fa, fb):
        ctx.fluid_release(f)
    ctx.mech_release(mid)


def test_fluid_full_grid_conservation(ctx, fo):
    """The headline's 1024 x 1024 grid (band temperature field of the 9-species mixture, with a
    shear flow added), one periodic split convective step on the GPU: the totals of every partial
    density, both momenta and the energy are unchanged to 1e-12 of their scale, and the step size
    equals the oracle's CFL bound computed on the same state."""
    m, grid, _ = synth.workload_grid_mech9()
    gas = fo.Gas(m)
    nx = ny = 1024
    T = grid.T.reshape(ny, nx)
    Y = grid.Y.reshape(m.ns, ny, nx)
    P = np.full((ny, nx), 1e5)
    Rmix = (Y * gas.Rs[:, None, None]).sum(0)
    rho = P / (Rmix * T)
    yy = (np.arange(ny) + 0.5)[:, None] / ny
    W = np.concatenate([Y * rho[None], (50.0 * np.sin(2 * np.pi * yy) + 0 * T)[None], np.zeros((1, ny, nx)), P[None]])
    Q = fo.to_conserved(gas, W)[0]
    mid = ctx.mech_upload(m)
    fid = ctx.fluid_create(mid, nx, ny, 1e-4, 1e-4, 0)
    ctx.fluid_upload(fid, np.ascontiguousarray(Q))
    dt = ctx.fluid_max_dt(fid, 0.4)
    dt_o = fo.max_dt(gas, Q, 1e-4, 1e-4, 0.4)
    assert abs(dt - dt_o) <= 1e-12 * dt_o
    ctx.fluid_step(fid, dt)
    Qg = ctx.fluid_download(fid)
    tot0, tot1 = Q.reshape(Q.shape[0], -1).sum(1), Qg.reshape(Q.shape[0], -1).sum(1)
    scale = var_scale(Q, np.sum)
    print(f"\n[fluid 1024^2] dt={dt:.3e} conservation {np.array2string(np.abs(tot1 - tot0) / scale, precision=2)}", flush=True)
    assert np.all(np.abs(tot1 - tot0) <= 1e-12 * scale)
    assert np.all(np.isfinite(Qg))
    ctx.fluid_release(fid)
    ctx.mech_release(mid)


def test_grid_arguments_checked(ctx):
    """Bad grids are refused before any device work: a periodic direction of fewer than three
    cells (the stencil would wrap twice), non-positive spacings, an unknown boundary rule; a
    transmissive grid of one row is accepted."""
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    mid = ctx.mech_upload(m)
    for nx, ny, dx, bc in ((2, 8, 1e-3, 0), (8, 1, 1e-3, 0), (8, 8, 0.0, 1), (8, 8, 1e-3, 7)):
        with pytest.raises(kin.KinError) as e:
            ctx.fluid_create(mid, nx, ny, dx, 1e-3, bc)
        assert e.value.status == kin.EINVAL, (nx, ny, dx, bc)
    fid = ctx.fluid_create(mid, 8, 1, 1e-3, 1e-3, 1)
    ctx.fluid_release(fid)
    ctx.mech_release(mid)
