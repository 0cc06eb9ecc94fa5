"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the same
seeded inputs.  Gate per mass fraction and temperature: 1e-10 relative for the FP64 form, 1e-6
for the FP32-LU form (with the term-scale floor of tests/parity.py).  Every cell is compared:
a cell whose sub-step schedule (status, halving level, schedule hash) matches the oracle's own
is compared with the oracle's adaptive result, any other cell with the oracle following the
GPU's recorded schedule (tests/parity.check_every_cell).  Schedule mismatches are counted and
bounded; Newton iteration counts are reported, not compared (the FP32-LU form converges
linearly, and the FP64 form's last iteration can differ by one where an update sits at the
tolerance)."""
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


def run_gpu(ctx, mech, st, dt, prec=0, opts=None, e0=None, mech_id=None):
    from paper_1110_4903_amd import kin
    mid = mech_id if mech_id is not None else ctx.mech_upload(mech)
    iid = ctx.state_upload(mid, st.rho, st.T, st.Y, e0=e0)
    ctx.advance([iid], [dt], prec=prec, opts=opts)
    out = ctx.download(iid) + (ctx.download_schedule(iid),)
    ctx.instance_release(iid)
    if mech_id is None:
        ctx.mech_release(mid)
    return out


def run_oracle(orc, mech, st, dt, e0=None, **kw):
    om = orc.OracleMech(mech)
    return om, om.advance(st.rho, st.T, st.Y, dt, e0=e0, opts=orc.make_opts(**kw) if kw else None,
                          with_sched=True)


def report(name, s):
    print(f"\n[{name}] " + " ".join(f"{k}={v}" for k, v in s.items()), flush=True)


def every_cell(ctx, orc, m, st, dt, prec, rtol, opts=None, mech_id=None, orc_kw=None, max_mismatch=2):
    """Run the GPU and the oracle on the same cells and compare every cell (see check_every_cell);
    asserts the gate on every cell, no cell finished on one side and failed on the other, and at
    most max_mismatch schedule mismatches (a count, or a fraction of the cells when below 1)."""
    from tests.parity import check_every_cell
    mid = mech_id if mech_id is not None else ctx.mech_upload(m)
    gpu = run_gpu(ctx, m, st, dt, prec=prec, opts=opts, mech_id=mid)
    om, ref = run_oracle(orc, m, st, dt, **(orc_kw or {}))
    s = check_every_cell(ctx, orc, m, mid, st, dt, prec, gpu, ref, rtol, opts=opts,
                         orc_opts=orc.make_opts(**orc_kw) if orc_kw else None)
    if mech_id is None:
        ctx.mech_release(mid)
    bound = max_mismatch if max_mismatch >= 1 else max_mismatch * st.n
    assert s["unchecked"] == 0 and s["follow_fail"] == 0 and s["ok_vs_failed"] == 0, s
    assert s["fail_Y"] == 0 and s["fail_T"] == 0 and s["fail_Y_followed"] == 0 and s["fail_T_followed"] == 0, s
    assert s["status_mismatch"] + s["schedule_mismatch"] <= bound, s
    return s, gpu, ref


def test_isomer_closed_form_gpu(ctx):
    """A <=> B through the lane layout: the exact backward-Euler step."""
    from tests.test_oracle_pins import isomer_mech
    kf, K, dt = 1e9, 0.3, 1e-6
    m = isomer_mech(kf, K)
    st = synth.CellStates(np.array([0.3, 0.05, 1.0]), np.array([1500.0, 900.0, 2500.0]),
                          np.array([[0.9, 0.2, 0.5], [0.1, 0.8, 0.5]]))
    T1, Y1, s, lv, it = run_gpu(ctx, m, st, dt)[:5]
    assert np.all(s == 0)
    kb = kf / K
    yeq = kb / (kf + kb)
    yA = yeq + (st.Y[0] - yeq) / (1 + (kf + kb) * dt)
    np.testing.assert_allclose(Y1[0], yA, rtol=1e-13)
    np.testing.assert_allclose(T1, st.T, rtol=1e-13)


def test_mech9_small_fp64_lane(ctx, orc):
    """9 species / 38 reactions, 4096 cells, one step of 1e-6 s, FP64, lane layout."""
    m, st, dt = synth.workload_small_mech9()
    s, gpu, ref = every_cell(ctx, orc, m, st, dt, 0, 1e-10)
    report("mech9 4096 fp64", s)
    assert s["checked"] == st.n


def test_mech36_sample_fp64_wave(ctx, orc):
    """36 species / 308 reactions, 512 cells of the 2^18-cell input, FP64, wave layout."""
    m, st, dt = synth.workload_mech36(1 << 18)
    sub = st.subset(np.arange(0, 1 << 18, 512))
    s, gpu, ref = every_cell(ctx, orc, m, sub, dt, 0, 1e-10)
    report("mech36 512 fp64", s)
    assert s["checked"] == sub.n


def test_mech9_small_fp32lu(ctx, orc):
    """FP32-LU form against the FP64 oracle at 1e-6 per result, every one of the 4096 cells:
    FP32 Newton converges linearly, so some cells take another sub-step schedule than the
    oracle's own; those are compared with the oracle following the GPU's schedule."""
    from paper_1110_4903_amd import kin
    m, st, dt = synth.workload_small_mech9()
    s, gpu, ref = every_cell(ctx, orc, m, st, dt, kin.FP32_LU, 1e-6, max_mismatch=0.1)
    report("mech9 4096 fp32lu", s)
    assert s["checked"] == st.n and s["compared"] >= 0.9 * st.n


def test_mech36_sample_fp32lu(ctx, orc):
    """FP32-LU form of the 36-species mechanism, 256 cells of the 2^18-cell input, wave layout,
    every cell against the oracle at 1e-6."""
    from paper_1110_4903_amd import kin
    m, st, dt = synth.workload_mech36(1 << 18)
    sub = st.subset(np.arange(7, 1 << 18, 1024))
    s, gpu, ref = every_cell(ctx, orc, m, sub, dt, kin.FP32_LU, 1e-6, max_mismatch=0.1)
    report("mech36 256 fp32lu", s)
    assert s["checked"] == sub.n and s["compared"] >= 0.9 * sub.n


@pytest.mark.parametrize("prec,rtol", [(0, 1e-10), (1, 1e-6)])
def test_grid_multistep_sampled(ctx, orc, prec, rtol):
    """The 1024x1024 band grid (the headline input), three steps of 1e-6 s on the GPU over all
    cells in the benchmark's launch configuration (cost-ordered), in the FP64 and the FP32-LU
    form.  A strided sample of 1052 cells is checked two ways: against the oracle's own three
    adaptive steps (FP64: every sampled cell must take the oracle's schedules; FP32-LU: the
    agreement is reported), and, every sampled cell, against the oracle following the GPU's
    recorded schedules of the same three steps.  The recorded re-run of the sample reproduces the
    full-grid result bitwise."""
    from tests.parity import compare, gpu_traces, oracle_follow
    m, grid, dt = synth.workload_grid_mech9()
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload(mid, grid.rho, grid.T, grid.Y)
    for _ in range(3):
        ctx.advance([iid], [dt], prec=prec)
    gpu = ctx.download(iid) + (ctx.download_schedule(iid),)
    ctx.instance_release(iid)
    sample = np.arange(0, grid.n, 997)
    sub = grid.subset(sample)
    g = tuple(a[..., sample] for a in gpu)
    traces, reruns = gpu_traces(ctx, mid, sub, dt, prec, steps=3)
    ctx.mech_release(mid)
    for x, y in zip(reruns[-1], g):
        assert np.array_equal(x, y, equal_nan=True)
    om = orc.OracleMech(m)
    e0 = om.energy_batch(sub.T, sub.Y)
    T, Y = sub.T.copy(), sub.Y.copy()
    for _ in range(3):
        T, Y, s_, l_, i_, h_ = om.advance(sub.rho, T, Y, dt, e0=e0, with_sched=True)
    own = compare(g, (T, Y, s_, l_, i_, h_), sub.rho, sub.Y, 3 * dt, om, rtol)
    fol = oracle_follow(om, sub, dt, traces, e0=e0)
    assert np.array_equal(fol[5], g[5]) and np.array_equal(fol[2], g[2])
    s = compare(g, fol, sub.rho, sub.Y, 3 * dt, om, rtol)
    report(f"grid 3 steps sampled prec {prec} (own schedule)", own)
    report(f"grid 3 steps sampled prec {prec} (GPU schedule)", s)
    assert s["compared"] == sub.n and s["fail_Y"] == 0 and s["fail_T"] == 0
    if prec == 0:
        assert own["status_mismatch"] == 0 and own["fail_Y"] == 0 and own["fail_T"] == 0


def full_size_invariants(orc, m, st, T1, Y1, e0, status):
    """Properties every finished cell of a backward-Euler step at constant (rho, e) has, at any
    size: element amounts and the sum of mass fractions unchanged, and e(Y, T) = e0 (the
    temperature inversion), checked with the oracle's energy function on every cell."""
    om = orc.OracleMech(m)
    ok = status < 2
    comp = np.asarray(m.comp, dtype=float).T
    el0 = comp @ (st.Y[:, ok] / m.M[:, None])
    el1 = comp @ (Y1[:, ok] / m.M[:, None])
    scale = comp @ (np.abs(st.Y[:, ok]) / m.M[:, None])
    assert np.all(np.abs(el1 - el0) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(Y1[:, ok].sum(0) - st.Y[:, ok].sum(0)) <= 1e-12)
    e1 = om.energy_batch(T1[ok], Y1[:, ok])
    assert np.all(np.abs(e1 - e0[ok]) <= 1e-12 * np.abs(e0[ok]) + 1e-6)
    return int(ok.sum())


@pytest.mark.parametrize("prec,rtol", [(0, 1e-10), (1, 1e-6)])
def test_mech36_full_size_sampled(ctx, orc, prec, rtol):
    """All 2^18 cells of the 36-species input on the GPU in the launch configuration the
    benchmark times: every cell keeps its element amounts, sum of mass fractions and energy;
    1024 strided cells checked against the oracle (each through its own schedule, or the GPU's
    where they differ)."""
    from tests.parity import check_every_cell
    from paper_1110_4903_amd import kin
    m, st, dt = synth.workload_mech36(1 << 18)
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload(mid, st.rho, st.T, st.Y)
    ctx.advance([iid], [dt], prec=prec)
    gpu = ctx.download(iid) + (ctx.download_schedule(iid),)
    e0 = ctx.download_e0(iid)
    ctx.instance_release(iid)
    assert np.all(gpu[2] < 2)
    n_inv = full_size_invariants(orc, m, st, gpu[0], gpu[1], e0, gpu[2])
    sample = np.arange(3, 1 << 18, 256)
    sub = st.subset(sample)
    om, ref = run_oracle(orc, m, sub, dt)
    g = tuple(a[..., sample] for a in gpu)
    s = check_every_cell(ctx, orc, m, mid, sub, dt, prec, g, ref, rtol)
    ctx.mech_release(mid)
    s["invariant_cells"] = n_inv
    report(f"mech36 2^18 prec {prec}", s)
    assert s["checked"] == sub.n and s["follow_fail"] == 0 and s["ok_vs_failed"] == 0
    assert s["fail_Y"] == 0 and s["fail_T"] == 0 and s["fail_Y_followed"] == 0 and s["fail_T_followed"] == 0
    assert s["status_mismatch"] + s["schedule_mismatch"] <= (2 if prec == kin.FP64 else 0.1 * sub.n)


@pytest.mark.parametrize("prec", [0, 1])
def test_grid_ten_steps_invariants(ctx, orc, prec):
    """The headline run itself: all 2^20 cells of the band grid through the ten steps the
    benchmark times (cost-ordered after the first), in either form; every cell finishes every
    step and keeps its element amounts, sum of mass fractions and energy."""
    m, grid, dt = synth.workload_grid_mech9()
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload(mid, grid.rho, grid.T, grid.Y)
    for _ in range(10):
        ctx.advance([iid], [dt], prec=prec)
        assert np.all(ctx.download(iid)[2] < 2)
    T1, Y1, st1 = ctx.download(iid)[:3]
    e0 = ctx.download_e0(iid)
    ctx.instance_release(iid)
    ctx.mech_release(mid)
    n_inv = full_size_invariants(orc, m, grid, T1, Y1, e0, st1)
    report(f"grid 10 steps prec {prec}", dict(invariant_cells=n_inv))
    assert n_inv == grid.n


@pytest.mark.parametrize("n", [1, 63, 65, 1000])
def test_ragged_sizes_both_layouts(ctx, orc, n):
    """Cell counts that are not multiples of the wavefront, through both layouts, every cell."""
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    st = synth.uniform_cells(100 + n, n, m.ns, 1.0)
    mid = ctx.mech_upload(m)
    for layout in (kin.LAYOUT_LANE, kin.LAYOUT_WAVE):
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, 0, 1e-10, opts=kin.solver_opts(layout=layout), mech_id=mid)
        assert s["checked"] == st.n, (layout, s)
    ctx.mech_release(mid)


def test_bad_inputs_and_forced_failure(ctx, orc):
    """Non-finite or out-of-range inputs give status 3 and are left untouched; k_max = 1
    fails every cell at L_max with its state unchanged (checked on the oracle too)."""
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    st = synth.uniform_cells(61, 70, m.ns, 1.0)
    T = st.T.copy()
    T[0] = np.nan
    T[1] = 100.0
    rho = st.rho.copy()
    rho[2] = -1.0
    bad = synth.CellStates(rho, T, st.Y)
    for layout in (kin.LAYOUT_LANE, kin.LAYOUT_WAVE):
        Tg, Yg, sg, lg, ig = run_gpu(ctx, m, bad, 1e-6, opts=kin.solver_opts(layout=layout))[:5]
        assert list(sg[:3]) == [3, 3, 3] and np.all(sg[3:] < 2)
        assert np.isnan(Tg[0]) and Tg[1] == 100.0 and np.array_equal(Yg[:, :3], st.Y[:, :3])
        Tg, Yg, sg, lg, ig, hg = run_gpu(ctx, m, st, 1e-6, opts=kin.solver_opts(layout=layout, k_max=1, L_max=4))
        _, (To, Yo, so, lo, io, ho) = run_oracle(orc, m, st, 1e-6, k_max=1, L_max=4)
        assert np.array_equal(hg, ho)
        assert np.array_equal(sg, so) and np.array_equal(lg, lo) and np.array_equal(ig, io)
        assert np.all(sg == 2) and np.array_equal(Tg, st.T) and np.array_equal(Yg, st.Y)


def test_replay_level_matches_oracle(ctx, orc):
    """Forced level L (2^L equal sub-steps) through both layouts against the oracle replay."""
    from tests.parity import compare
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    st = synth.uniform_cells(71, 128, m.ns, 1.0)
    om, ref = run_oracle(orc, m, st, 1e-7)
    ref = om.advance(st.rho, st.T, st.Y, 1e-7, L_forced=3)
    for layout in (kin.LAYOUT_LANE, kin.LAYOUT_WAVE):
        gpu = run_gpu(ctx, m, st, 1e-7, opts=kin.solver_opts(layout=layout, L_forced=3))
        s = compare(gpu, ref, st.rho, st.Y, 1e-7, om, 1e-10)
        assert s["status_mismatch"] == 0 and s["level_mismatch"] == 0, s
        assert s["fail_Y"] == 0 and s["fail_T"] == 0, s


def test_e0_given_and_resume(ctx):
    """Checkpoint/resume: 4 steps equal 2 steps + download + re-upload (with e0) + 2 steps,
    bitwise, in the FP64 form."""
    m, st, dt = synth.workload_small_mech9(512)
    mid = ctx.mech_upload(m)
    a = ctx.state_upload(mid, st.rho, st.T, st.Y)
    for _ in range(4):
        ctx.advance([a], [dt])
    Ta, Ya = ctx.download(a)[:2]
    b = ctx.state_upload(mid, st.rho, st.T, st.Y)
    for _ in range(2):
        ctx.advance([b], [dt])
    Tb, Yb = ctx.download(b)[:2]
    e0 = ctx.download_e0(b)
    c = ctx.state_upload(mid, st.rho, Tb, Yb, e0=e0)
    for _ in range(2):
        ctx.advance([c], [dt])
    Tc, Yc = ctx.download(c)[:2]
    assert np.array_equal(Ta, Tc) and np.array_equal(Ya, Yc)
    for i in (a, b, c):
        ctx.instance_release(i)
    ctx.mech_release(mid)


@pytest.mark.parametrize("case", ["mech9-lane", "mech9-lane-fp32lu", "mech36-wave", "mech9-global"])
def test_cost_order_is_bitwise_neutral(ctx, case):
    """A single instance large enough (262144 cells in the lane layout, 32768 in the others)
    takes its cells in cost order: by the previous
    advance's iteration counts when they are current, and in the lane layout by the source
    term's temperature change on a first advance.  Both equal, bitwise (state, status, level,
    iterations, schedule), the same step in index order, taken through a batched launch (which
    never reorders).  A cell left out of, or repeated in, an order would show as a difference."""
    from paper_1110_4903_amd import kin
    name, layout = case.split("-")[:2]
    prec = 1 if case.endswith("fp32lu") else 0
    m = synth.mechanism(name)
    n = {"lane": 270000, "wave": 33000, "global": 40000}[layout]
    st = synth.uniform_cells(71, n, m.ns, 1.0 if name == "mech9" else 0.5)
    tiny = synth.uniform_cells(72, 64, m.ns, 0.5)
    dt = 1e-6
    mid = ctx.mech_upload(m)
    if layout == "global":
        ctx.set_layout(mid, kin.LAYOUT_GLOBAL, 64)

    def full(i):
        return ctx.download(i) + (ctx.download_schedule(i),)

    def same(x, y):
        for u, v in zip(x, y):
            assert np.array_equal(u, v, equal_nan=True)

    # first step: a alone (first-advance order in the lane layout) against index order
    a = ctx.state_upload(mid, st.rho, st.T, st.Y)
    c = ctx.state_upload(mid, st.rho, st.T, st.Y)
    d = ctx.state_upload(mid, tiny.rho, tiny.T, tiny.Y)
    ctx.advance([a], [dt], prec=prec)
    ctx.advance([c, d], [dt, dt], prec=prec)
    same(full(a), full(c))
    T1, Y1, _, _, it1 = ctx.download(a)[:5]
    bounds = [5, 10, 20, 40, 80, 160, 320]
    assert np.unique(np.digitize(it1, bounds)).size > 1, "the first step should give more than one cost class"
    # second step: a in the order of its counts; b (fresh, same state) and c (batched, index order)
    e0 = ctx.download_e0(a)
    b = ctx.state_upload(mid, st.rho, T1, Y1, e0=e0)
    ctx.advance([a], [dt], prec=prec)
    ctx.advance([b], [dt], prec=prec)
    ctx.advance([c, d], [dt, dt], prec=prec)
    same(full(a), full(b))
    same(full(a), full(c))
    report(f"cost order {case}", dict(cells=n, classes=np.bincount(np.digitize(it1, bounds), minlength=8).tolist()))
    for i in (a, b, c, d):
        ctx.instance_release(i)
    ctx.mech_release(mid)


def _batch_setup(ctx, insts):
    mids = {}
    ids, states = [], []
    for ins in insts:
        if ins.mech not in mids:
            mids[ins.mech] = ctx.mech_upload(synth.mechanism(ins.mech))
        st = ins.states()
        states.append(st)
        ids.append(ctx.state_upload(mids[ins.mech], st.rho, st.T, st.Y))
    return mids, ids, states


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_graph_equals_single_launches(ctx, prec):
    """An uneven batch (mech9 and mech36 instances of 1..3000 cells, one dt each) advanced in
    one call (one graph launch, one kernel per mechanism and layout, spans of up to 64
    instances) gives, bitwise, what advancing every instance alone gives.  70 instances, so
    the 9-species group needs two launches of its span table."""
    insts = synth.batch_instances(seed=11, n_inst=70, min_cells=1, max_cells=3000)
    mids, ids, states = _batch_setup(ctx, insts)
    dts = [ins.dt for ins in insts]
    ctx.advance(ids, dts, prec=prec)
    batched = [ctx.download(i) + (ctx.download_schedule(i),) for i in ids]
    # a second batched call replays the cached graph
    for i, st in zip(ids, states):
        ctx.state_reset(i, st.rho, st.T, st.Y)
    ctx.advance(ids, dts, prec=prec)
    again = [ctx.download(i) + (ctx.download_schedule(i),) for i in ids]
    for i, st in zip(ids, states):
        ctx.state_reset(i, st.rho, st.T, st.Y)
    for i, dt in zip(ids, dts):
        ctx.advance([i], [dt], prec=prec)
    single = [ctx.download(i) + (ctx.download_schedule(i),) for i in ids]
    for k, (a, b, c) in enumerate(zip(batched, again, single)):
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x, z, equal_nan=True), (k, insts[k])
            assert np.array_equal(y, z, equal_nan=True), (k, insts[k])
    for i in ids:
        ctx.instance_release(i)
    for m in mids.values():
        ctx.mech_release(m)


def test_batched_against_oracle(ctx, orc):
    """Every instance of a 24-instance uneven batch, advanced in one call, against the
    oracle per instance (FP64 gate)."""
    from tests.parity import compare
    insts = synth.batch_instances(seed=12, n_inst=24, min_cells=1, max_cells=400)
    mids, ids, states = _batch_setup(ctx, insts)
    ctx.advance(ids, [ins.dt for ins in insts])
    for ins, i, st in zip(insts, ids, states):
        gpu = ctx.download(i) + (ctx.download_schedule(i),)
        om, ref = run_oracle(orc, synth.mechanism(ins.mech), st, ins.dt)
        s = compare(gpu, ref, st.rho, st.Y, ins.dt, om, 1e-10)
        assert s["status_mismatch"] == 0 and s["fail_Y"] == 0 and s["fail_T"] == 0, (ins, s)
        assert s["schedule_mismatch"] <= max(1, ins.n_cells // 200), (ins, s)
        ctx.instance_release(i)
    for m in mids.values():
        ctx.mech_release(m)


def test_autotune_restores_state_and_persists(ctx, tmp_path):
    """The autotuner leaves the instance's state as it was, picks an admissible layout, and a
    new context reading its cache file applies the same choice at upload."""
    from paper_1110_4903_amd import kin
    cache = str(tmp_path / "tune.json")
    m, st, dt = synth.workload_small_mech9(8192)
    with kin.Context(0, tune_cache=cache) as c1:
        mid = c1.mech_upload(m)
        iid = c1.state_upload(mid, st.rho, st.T, st.Y)
        before = c1.download(iid)[:2]
        lay, blk, ms = c1.autotune(mid, iid, dt)
        after = c1.download(iid)[:2]
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        assert (lay, blk) in {(kin.LAYOUT_LANE, 64), (kin.LAYOUT_LANE, 128), (kin.LAYOUT_LANE, 256),
                              (kin.LAYOUT_WAVE, 1), (kin.LAYOUT_WAVE, 2), (kin.LAYOUT_WAVE, 4)}
        assert ms > 0
        print(f"\n[autotune mech9 8192] layout={lay} block={blk} {ms:.3f} ms", flush=True)
    with kin.Context(0, tune_cache=cache) as c2:
        mid = c2.mech_upload(m)
        assert c2.tuned(mid) == {(kin.FP64, kin.size_class(8192)): (lay, blk)}
        # the mechanism's own layout (other size classes) is unchanged
        assert c2.query_int(kin.Q_LAYOUT, mid) == kin.LAYOUT_LANE


def test_autotune_is_per_size_class(ctx, orc, tmp_path):
    """The autotuner's choice applies to launches of the size class it was tuned at.  Tuned at
    1024 cells the 9-species mechanism picks some layout for that class, and launches of 2^18
    cells still run the lane layout; the tuned small launch still matches the oracle."""
    from paper_1110_4903_amd import kin
    from tests.parity import compare
    m = synth.mechanism("mech9")
    small = synth.uniform_cells(81, 1024, m.ns, 1.0)
    with kin.Context(0, tune_cache=str(tmp_path / "t.json")) as c:
        mid = c.mech_upload(m)
        iid = c.state_upload(mid, small.rho, small.T, small.Y)
        lay, blk, ms = c.autotune(mid, iid, 1e-6)
        assert c.tuned(mid) == {(kin.FP64, 0): (lay, blk)}
        c.advance([iid], [1e-6])
        gpu = c.download(iid) + (c.download_schedule(iid),)
        om, ref = run_oracle(orc, m, small, 1e-6)
        s = compare(gpu, ref, small.rho, small.Y, 1e-6, om, 1e-10)
        assert s["status_mismatch"] == 0 and s["fail_Y"] == 0 and s["fail_T"] == 0, s
        print(f"\n[autotune mech9 1024] layout={lay} block={blk} {ms:.3f} ms", flush=True)
        c.instance_release(iid)


def test_point_implicit_both_layouts(ctx, orc):
    """The paper's point-implicit step (one linearised backward-Euler step over dt), FP64: mech9
    through both layouts and mech36 through the wave layout, against the oracle.  Gate: 1e-10
    relative plus the conditioning floor of a single linear solve, capped at 1e-6 |dx|
    (tests/parity.point_implicit_floor); cells whose floor would pass the cap (condition numbers
    beyond about 4e6) are compared instead by the componentwise backward error of the GPU's solve
    against the oracle's J and f in long double (tests/parity.point_implicit_residual, gate 1e-8:
    the oracle's own elimination reaches 1e-9 on these stiff matrices, and a 1e-6 relative error
    planted in one component of dx gives 1e-7), and counted.
    One iteration and level 0 everywhere.  The FP32-LU form is refused for this step (no Newton
    refinement)."""
    from tests.parity import compare, point_implicit_floor, point_implicit_residual
    from paper_1110_4903_amd import kin
    prec, rtol, eps = 0, 1e-10, np.finfo(np.float64).eps
    cases = [("mech9", synth.uniform_cells(23, 2000, 9, 1.0), 1e-7, kin.LAYOUT_LANE),
             ("mech9", synth.uniform_cells(23, 2000, 9, 1.0), 1e-7, kin.LAYOUT_WAVE),
             ("mech36", synth.uniform_cells(24, 300, 36, 0.5), 1e-8, kin.LAYOUT_WAVE)]
    for name, st, dt, layout in cases:
        m = synth.mechanism(name)
        gpu = run_gpu(ctx, m, st, dt, prec=prec, opts=kin.solver_opts(layout=layout, point_implicit=1))
        om, ref = run_oracle(orc, m, st, dt, point_implicit=1)
        fy, ft, over = point_implicit_floor(om, st.rho, st.Y, st.T, ref[1], ref[0], dt, eps)
        keep = np.flatnonzero(~over)
        s = compare(tuple(a[..., keep] for a in gpu), tuple(a[..., keep] for a in ref), st.rho[keep],
                    st.Y[:, keep], dt, om, rtol, extra=(fy[:, keep], ft[keep]))
        hard = np.flatnonzero(over & (gpu[2] < 2) & (ref[2] < 2))
        be = point_implicit_residual(om, st.rho[hard], st.Y[:, hard], st.T[hard], gpu[1][:, hard], dt)
        s.update(floor_capped_cells=int(over.sum()), backward_checked=int(hard.size),
                 max_backward_error=float(be.max()) if be.size else 0.0)
        report(f"point-implicit {name} layout={layout}", s)
        assert np.all(gpu[3] == 0) and np.all(gpu[4][gpu[2] < 3] == 1)
        assert np.array_equal(gpu[2], ref[2])
        assert s["fail_Y"] == 0 and s["fail_T"] == 0, s
        assert np.all(be <= 1e-8), be.max()
    m = synth.mechanism("mech9")
    st = synth.uniform_cells(25, 8, 9, 1.0)
    with pytest.raises(kin.KinError) as e:
        run_gpu(ctx, m, st, 1e-7, prec=kin.FP32_LU, opts=kin.solver_opts(point_implicit=1))
    assert e.value.status == kin.EINVAL


def test_divergence_test_off_matches_oracle(ctx, orc):
    """With the Newton divergence test disabled (diverge_ratio = 0) both layouts still follow
    the oracle (FP64 gate)."""
    from tests.parity import compare
    from paper_1110_4903_amd import kin
    for name, st, layout in (("mech9", synth.uniform_cells(31, 500, 9, 1.0), kin.LAYOUT_LANE),
                             ("mech36", synth.uniform_cells(32, 128, 36, 0.5), kin.LAYOUT_WAVE)):
        m = synth.mechanism(name)
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, 0, 1e-10, opts=kin.solver_opts(layout=layout, diverge_ratio=0.0),
                             orc_kw=dict(diverge_ratio=0.0))
        report(f"diverge off {name}", s)
        assert s["checked"] == st.n


@pytest.mark.parametrize("ns,nr,ne", [(20, 120, 3), (23, 140, 3), (28, 200, 4), (30, 200, 4), (45, 360, 4),
                                      (47, 380, 4), (60, 480, 4)])
def test_wave_layout_other_row_lengths(ctx, orc, ns, nr, ne):
    """Generated mechanisms whose padded Jacobian rows (24, 32, 48, 64 columns) select the other
    instantiations of the wave kernel, 128 cells, FP64 and FP32-LU, against the oracle.  The
    unknown counts N = Ns + 1 cover every remainder mod 4 (the FP64 elimination's panel width):
    24 and 48 end on a full panel with only b right of it, 31 on a three-column panel."""
    from tests.parity import compare
    from paper_1110_4903_amd import kin
    m = synth.make_mechanism(synth.MechRecipe(f"gen{ns}", seed=100 + ns, n_elements=ne, n_species=ns,
                                              n_reactions=nr, frac_third_body=0.15,
                                              frac_irreversible=0.3))
    st = synth.uniform_cells(200 + ns, 128, ns, 0.5)
    mid = ctx.mech_upload(m)
    for prec, rtol, bound in ((kin.FP64, 1e-10, 2), (kin.FP32_LU, 1e-6, 0.1)):
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, prec, rtol, mech_id=mid, max_mismatch=bound)
        report(f"gen{ns} prec {prec}", s)
        assert s["checked"] == st.n
    ctx.mech_release(mid)


@pytest.mark.gpu
def test_wave_layout_without_third_body_reactions(ctx, orc):
    """A 20-species mechanism with no third-body reaction on the wave layout (its dense
    third-body product is skipped), 128 cells, FP64 and FP32-LU, against the oracle."""
    from paper_1110_4903_amd import kin
    m = synth.make_mechanism(synth.MechRecipe("gen20_no_m", seed=420, n_elements=3, n_species=20,
                                              n_reactions=120, frac_third_body=0.0,
                                              frac_irreversible=0.3))
    assert m.ntb == 0
    st = synth.uniform_cells(520, 128, 20, 0.5)
    mid = ctx.mech_upload(m)
    assert ctx.query_int(kin.Q_LAYOUT, mid) == kin.LAYOUT_WAVE
    for prec, rtol, bound in ((kin.FP64, 1e-10, 2), (kin.FP32_LU, 1e-6, 0.1)):
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, prec, rtol, mech_id=mid, max_mismatch=bound)
        report(f"gen20 without third bodies prec {prec}", s)
        assert s["checked"] == st.n
    ctx.mech_release(mid)


@pytest.mark.parametrize("ns,nr,ne,block", [(15, 40, 3, 128), (11, 30, 3, 256)])
def test_lane_layout_largest_systems(ctx, orc, ns, nr, ne, block):
    """The lane layout at its largest systems: 15 species (a 16 x 16 Newton matrix in registers)
    at 128 threads per block, and 11 species at 256 threads, the largest block whose queue and
    start states fit 64 KiB of LDS; 300 cells, FP64 and FP32-LU, every cell against the oracle.
    256 threads for 15 species is refused (EINVAL)."""
    from paper_1110_4903_amd import kin
    m = synth.make_mechanism(synth.MechRecipe(f"gen{ns}", seed=300 + ns, n_elements=ne, n_species=ns,
                                              n_reactions=nr, frac_third_body=0.15,
                                              frac_irreversible=0.3))
    st = synth.uniform_cells(400 + ns, 300, ns, 0.5)
    mid = ctx.mech_upload(m)
    if ns == 15:
        with pytest.raises(kin.KinError) as e:
            ctx.set_layout(mid, kin.LAYOUT_LANE, 256)
        assert e.value.status == kin.EINVAL
    ctx.set_layout(mid, kin.LAYOUT_LANE, block)
    for prec, rtol, bound in ((kin.FP64, 1e-10, 3), (kin.FP32_LU, 1e-6, 0.1)):
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, prec, rtol, mech_id=mid, max_mismatch=bound)
        report(f"lane gen{ns} block {block} prec {prec}", s)
        assert s["checked"] == st.n
    ctx.mech_release(mid)


def both_sides_mech():
    """H, H2, O, OH, H2O, O2: a third-order reaction with H on both sides (3 H => H2 + H), a
    product with nu = 2, an irreversible reaction and a third-body reaction."""
    from tests.test_oracle_pins import nasa_const
    nas = [nasa_const(2.5, 2600.0, 14.0), nasa_const(3.5, 0.0, 16.0), nasa_const(2.5, 3000.0, 19.0),
           nasa_const(3.6, 450.0, 22.0), nasa_const(4.0, -2900.0, 23.0), nasa_const(3.5, 0.0, 25.0)]
    comp = [[1, 0], [2, 0], [0, 1], [1, 1], [2, 1], [0, 2]]
    rx = [dict(reac=[(0, 3)], prod=[(1, 1), (0, 1)], A=1e15, b=-0.5, Ta=0.0),
          dict(reac=[(2, 1), (4, 1)], prod=[(3, 2)], A=3e13, b=0.0, Ta=9000.0),
          dict(reac=[(1, 1), (5, 1)], prod=[(3, 2)], A=1e12, b=0.5, Ta=20000.0, reversible=False),
          dict(reac=[(0, 1), (3, 1)], prod=[(4, 1)], A=2e17, b=-1.0, Ta=0.0, tb=0),
          dict(reac=[(0, 1), (5, 1)], prod=[(3, 1), (2, 1)], A=2e14, b=0.0, Ta=8000.0)]
    return synth.mechanism_from_lists("bothsides", ("H", "O"), comp, nas, rx,
                                      eff=[[1.0, 2.5, 1.0, 1.0, 6.0, 1.0]])


def test_species_on_both_sides_both_layouts(ctx, orc):
    """A species on both sides of a reaction enters the wave layout's reactant and product
    slots separately; both layouts against the oracle, FP64."""
    from paper_1110_4903_amd import kin
    m = both_sides_mech()
    st = synth.uniform_cells(77, 300, m.ns, 1.0)
    mid = ctx.mech_upload(m)
    for layout in (kin.LAYOUT_LANE, kin.LAYOUT_WAVE):
        s, _, ref = every_cell(ctx, orc, m, st, 1e-6, 0, 1e-10, opts=kin.solver_opts(layout=layout), mech_id=mid)
        report(f"both sides layout {layout}", s)
        assert np.all(ref[2] < 2) and s["checked"] == st.n, (layout, s)
    ctx.mech_release(mid)


def test_conserved_inversion_across_range_switch(ctx, orc):
    """The adapter's temperature inversion where the cells' temperatures (600-2500 K) lie on both
    sides of the species' NASA-7 range switch and the Newton starts on the other side of it: an
    upload without guesses (start 1500 K), then a reset with guesses of 2400 K for the cells
    below 1000 K and 700 K for the others.  T within 1e-12 of the oracle's inversion both times,
    so the Newton's coefficient sums are redone correctly when T crosses a switch."""
    m = synth.mechanism("mech9")
    om = orc.OracleMech(m)
    st = synth.uniform_cells(43, 512, m.ns, 1.0, T_range=(600.0, 2500.0))
    e0 = om.energy_batch(st.T, st.Y)
    rho_s, E = om.to_conserved(st.rho, st.Y, e0)
    T = om.from_conserved(rho_s, E)[2]
    assert np.all(np.abs(T - st.T) <= 1e-9 * st.T)
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload_conserved(mid, rho_s, E)
    np.testing.assert_allclose(ctx.download(iid)[0], T, rtol=1e-12)
    guess = np.where(st.T < 1000.0, 2400.0, 700.0)
    ctx.state_reset_conserved(iid, rho_s, E, T_guess=guess)
    np.testing.assert_allclose(ctx.download(iid)[0], T, rtol=1e-12)
    ctx.instance_release(iid)
    ctx.mech_release(mid)

@pytest.mark.parametrize("name", ["mech9", "mech36"])
def test_conserved_adapter_against_oracle(ctx, orc, name):
    """Operator-split adapter: partial densities and sensible energy in, one step of 1e-6 s,
    partial densities and sensible energy out, against the oracle's same pipeline (FP64, 1e-10
    relative on the scale of the energy terms); device and host destinations agree bitwise.
    Cells with no density, or with an energy beyond 6000 K, come out as bad input."""
    import torch
    from tests.parity import compare
    m = synth.mechanism(name)
    om = orc.OracleMech(m)
    st = synth.uniform_cells(41, 256, m.ns, 1.0 if name == "mech9" else 0.5)
    dt = 1e-6
    e0 = om.energy_batch(st.T, st.Y)
    rho_s, E = om.to_conserved(st.rho, st.Y, e0)
    rho_s[:, 5] = 0.0            # no density
    E[7] = 1e3 * abs(E[7]) + 1e9  # no temperature in [200, 6000] K
    with np.errstate(invalid="ignore", divide="ignore"):
        rho, Y, T, e0o, ok = om.from_conserved(rho_s, E)
    assert not ok[7]
    mid = ctx.mech_upload(m)
    iid = ctx.state_upload_conserved(mid, rho_s, E)
    T_up = ctx.download(iid)[0]
    good = np.ones(st.n, bool)
    good[[5, 7]] = False
    np.testing.assert_allclose(T_up[good], T[good], rtol=1e-12)
    assert np.isnan(T_up[7])
    ctx.advance([iid], [dt])
    gpu = ctx.download(iid) + (ctx.download_schedule(iid),)
    g_rho_s, g_E = ctx.download_conserved(iid)
    d_rho_s = torch.empty((m.ns, st.n), dtype=torch.float64, device="cuda")
    d_E = torch.empty(st.n, dtype=torch.float64, device="cuda")
    ctx.download_conserved_device(iid, d_rho_s, d_E)
    torch.cuda.synchronize()
    assert np.array_equal(d_rho_s.cpu().numpy(), g_rho_s, equal_nan=True)
    assert np.array_equal(d_E.cpu().numpy(), g_E, equal_nan=True)
    ctx.instance_release(iid)
    ctx.mech_release(mid)
    assert gpu[2][5] == 3 and gpu[2][7] == 3
    T_in = np.where(good, T, st.T)
    Y_in = np.where(good[None, :], Y, st.Y)
    rho_in = np.where(good, rho, st.rho)
    ref = om.advance(rho_in, T_in, Y_in, dt, e0=np.where(good, e0o, e0), with_sched=True)
    s = compare(tuple(a[..., good] for a in gpu), tuple(a[..., good] for a in ref), rho_in[good],
                Y_in[:, good], dt, om, 1e-10)
    report(f"{name} adapter", s)
    assert s["status_mismatch"] == 0 and s["schedule_mismatch"] <= 2 and s["fail_Y"] == 0 and s["fail_T"] == 0
    r_rho_s, r_E = om.to_conserved(rho_in, ref[1], np.where(good, e0o, e0))
    same = good & (gpu[5] == ref[5])
    ef = om.formation_energies()
    scale = np.abs(r_E) + rho_in * (np.abs(ef) @ np.abs(ref[1]))
    assert np.all(np.abs(g_E[same] - r_E[same]) <= 1e-10 * scale[same])
    np.testing.assert_allclose(g_rho_s[:, same], r_rho_s[:, same], rtol=1e-10, atol=1e-14 * rho_in.max())


def big_mech(ns, nr):
    """Generated mechanism beyond the wave layout's 63 species (5 elements)."""
    return synth.make_mechanism(synth.MechRecipe(f"gen{ns}", seed=1000 + ns, n_elements=5, n_species=ns,
                                                 n_reactions=nr, frac_third_body=0.15,
                                                 frac_irreversible=0.3))


@pytest.mark.parametrize("case", ["mech9", "mech36", "gen100"])
def test_global_layout_against_oracle(ctx, orc, case):
    """The global-memory layout (one wavefront per cell, the cell's matrix column-major in HBM):
    the 9- and 36-species
    mechanisms forced onto it, and a 100-species mechanism that selects it by itself, FP64 and
    FP32-LU, against the oracle."""
    from tests.parity import compare
    from paper_1110_4903_amd import kin
    if case == "gen100":
        m, n, alpha = big_mech(100, 600), 64, 0.5
    else:
        m, n, alpha = synth.mechanism(case), 128, 1.0 if case == "mech9" else 0.5
    st = synth.uniform_cells(500 + m.ns, n, m.ns, alpha)
    mid = ctx.mech_upload(m)
    if case == "gen100":
        assert ctx.query_int(kin.Q_LAYOUT, mid) == kin.LAYOUT_GLOBAL
    opts = kin.solver_opts(layout=kin.LAYOUT_GLOBAL)
    for prec, rtol, bound in ((kin.FP64, 1e-10, 2), (kin.FP32_LU, 1e-6, 0.1)):
        s, _, _ = every_cell(ctx, orc, m, st, 1e-6, prec, rtol, opts=opts, mech_id=mid, max_mismatch=bound)
        report(f"global {case} prec {prec}", s)
        assert s["checked"] == st.n
    ctx.mech_release(mid)


def test_batched_graph_with_global_layout(ctx):
    """A batch mixing a 70-species mechanism (global-memory layout, two instances sharing one
    launch and the graph's workspace) with mech36 (wave layout) equals, bitwise, advancing
    each instance alone; a second call replays the cached graph."""
    from paper_1110_4903_amd import kin
    big = big_mech(70, 400)
    m36 = synth.mechanism("mech36")
    mb, m3 = ctx.mech_upload(big), ctx.mech_upload(m36)
    assert ctx.query_int(kin.Q_LAYOUT, mb) == kin.LAYOUT_GLOBAL
    cases = [(mb, big, synth.uniform_cells(61, 70, big.ns, 0.5), 1e-6),
             (mb, big, synth.uniform_cells(62, 33, big.ns, 0.5), 3e-7),
             (m3, m36, synth.uniform_cells(63, 100, m36.ns, 0.5), 1e-6)]
    ids = [ctx.state_upload(mid, st.rho, st.T, st.Y) for mid, _, st, _ in cases]
    dts = [dt for *_, dt in cases]
    runs = []
    for _ in range(2):
        for i, (_, _, st, _) in zip(ids, cases):
            ctx.state_reset(i, st.rho, st.T, st.Y)
        ctx.advance(ids, dts)
        runs.append([ctx.download(i) + (ctx.download_schedule(i),) for i in ids])
    for i, (_, _, st, _) in zip(ids, cases):
        ctx.state_reset(i, st.rho, st.T, st.Y)
    for i, dt in zip(ids, dts):
        ctx.advance([i], [dt])
    single = [ctx.download(i) + (ctx.download_schedule(i),) for i in ids]
    for run in runs:
        for k, (a, c) in enumerate(zip(run, single)):
            for x, z in zip(a, c):
                assert np.array_equal(x, z, equal_nan=True), k
    assert all(np.all(s[2] < 2) for s in single)
    for i in ids:
        ctx.instance_release(i)
    ctx.mech_release(mb)
    ctx.mech_release(m3)


def test_kernel_times_recorded_per_advance():
    """KIN_CTX_TIME_KERNELS: one duration per single-instance advance, in launch order, each
    positive and within the host's wall time around its advance; the list empties on reading;
    a context without the flag records nothing.  These durations are the benchmark roofline's
    kernel time."""
    import time
    import torch
    from paper_1110_4903_amd import kin
    m = synth.mechanism("mech9")
    st = synth.uniform_cells(71, 20000, 9, 1.0)
    for flag in (True, False):
        c = kin.Context(0, time_kernels=flag)
        try:
            mid = c.mech_upload(m)
            iid = c.state_upload(mid, st.rho, st.T, st.Y)
            c.advance([iid], [1e-6])
            torch.cuda.synchronize()
            c.kernel_times()
            walls = []
            for dt in (1e-7, 1e-6, 4e-6):
                t0 = time.perf_counter()
                c.advance([iid], [dt])
                torch.cuda.synchronize()
                walls.append(1e3 * (time.perf_counter() - t0))
            kt = c.kernel_times()
            if flag:
                assert len(kt) == 3, kt
                assert all(0.0 < k <= w for k, w in zip(kt, walls)), (kt, walls)
                assert c.kernel_times() == []
            else:
                assert kt == []
        finally:
            c.close()
