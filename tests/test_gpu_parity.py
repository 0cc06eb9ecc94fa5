"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the same
seeded inputs.  Gate: 1e-10 relative per mass fraction and temperature for the FP64 form (with
the term-scale floor of tests/parity.py), identical per-cell status, halving level and Newton
iteration count."""
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
    out = ctx.download(iid)
    ctx.instance_release(iid)
    if mech_id is None:
        ctx.mech_release(mid)
    return out


def run_oracle(orc, mech, st, dt, e0=None, **kw):
    om = orc.OracleMech(mech)
    return om, om.advance(st.rho, st.T, st.Y, dt, e0=e0, opts=orc.make_opts(**kw) if kw else None)


def report(name, s):
    print(f"\n[{name}] " + " ".join(f"{k}={v}" for k, v in s.items()), flush=True)


def test_isomer_closed_form_gpu(ctx):
    """A <=> B through the lane layout: the exact backward-Euler step."""
    from tests.test_oracle_pins import isomer_mech
    kf, K, dt = 1e9, 0.3, 1e-6
    m = isomer_mech(kf, K)
    st = synth.CellStates(np.array([0.3, 0.05, 1.0]), np.array([1500.0, 900.0, 2500.0]),
                          np.array([[0.9, 0.2, 0.5], [0.1, 0.8, 0.5]]))
    T1, Y1, s, lv, it = run_gpu(ctx, m, st, dt)
    assert np.all(s == 0)
    kb = kf / K
    yeq = kb / (kf + kb)
    yA = yeq + (st.Y[0] - yeq) / (1 + (kf + kb) * dt)
    np.testing.assert_allclose(Y1[0], yA, rtol=1e-13)
    np.testing.assert_allclose(T1, st.T, rtol=1e-13)


def test_mech9_small_fp64_lane(ctx, orc):
    """9 species / 38 reactions, 4096 cells, one step of 1e-6 s, FP64, lane layout."""
    from tests.parity import compare
    m, st, dt = synth.workload_small_mech9()
    gpu = run_gpu(ctx, m, st, dt)
    om, ref = run_oracle(orc, m, st, dt)
    s = compare(gpu, ref, st.rho, st.Y, dt, om, 1e-10)
    report("mech9 4096 fp64", s)
    assert s["status_mismatch"] == 0 and s["level_mismatch"] <= 2
    assert s["fail_Y"] == 0 and s["fail_T"] == 0


def test_mech36_sample_fp64_wave(ctx, orc):
    """36 species / 308 reactions, 512 cells of the 2^18-cell input, FP64, wave layout."""
    from tests.parity import compare
    m, st, dt = synth.workload_mech36(1 << 18)
    sub = st.subset(np.arange(0, 1 << 18, 512))
    gpu = run_gpu(ctx, m, sub, dt)
    om, ref = run_oracle(orc, m, sub, dt)
    s = compare(gpu, ref, sub.rho, sub.Y, dt, om, 1e-10)
    report("mech36 512 fp64", s)
    assert s["status_mismatch"] == 0 and s["level_mismatch"] <= 2
    assert s["fail_Y"] == 0 and s["fail_T"] == 0
