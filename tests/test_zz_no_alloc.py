"""kin_advance_noalloc (the advance that allocates nothing: fixed device memory for its work
counters and the global layout's matrices) against kin_advance, bitwise, through the C ABI:
two calls in a row, the second with a smaller input, then the refusal of a call beyond its
limit.  The two entry points share their kernels; what differs is where the counters and the
workspace live and that the noalloc call launches without a graph."""
import numpy as np
import pytest

from paper_1110_4903_amd import synth

pytestmark = pytest.mark.gpu


def _big_mech(ns, nr):
    return synth.make_mechanism(synth.MechRecipe(f"gen{ns}", seed=1000 + ns, n_elements=5, n_species=ns,
                                                 n_reactions=nr, frac_third_body=0.15,
                                                 frac_irreversible=0.3))


def _full(ctx, i):
    return ctx.download(i) + (ctx.download_schedule(i),)


def _same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y, equal_nan=True), (what, k)


def test_noalloc_advance_equals_advance():
    import torch
    from paper_1110_4903_amd import kin
    with kin.Context(0) as ctx:
        mechs = {"gen100": _big_mech(100, 600), "mech9": synth.mechanism("mech9"),
                 "mech36": synth.mechanism("mech36")}
        mids = {k: ctx.mech_upload(m) for k, m in mechs.items()}
        assert ctx.query_int(kin.Q_LAYOUT, mids["gen100"]) == kin.LAYOUT_GLOBAL
        assert ctx.query_int(kin.Q_LAYOUT, mids["mech9"]) == kin.LAYOUT_LANE
        assert ctx.query_int(kin.Q_LAYOUT, mids["mech36"]) == kin.LAYOUT_WAVE
        calls = [
            # (mechanism, cells, dt, state seed, Dirichlet alpha) per instance
            [("gen100", 300, 1e-6, 11, 0.5), ("mech9", 3000, 1e-6, 12, 1.0), ("mech36", 200, 5e-7, 13, 0.5),
             ("gen100", 70, 3e-7, 14, 0.5)],
            [("gen100", 40, 1e-6, 15, 0.5)],
        ]
        for prec in (kin.FP64, kin.FP32_LU):
            for c, insts in enumerate(calls):
                sts = [synth.uniform_cells(seed, n, mechs[name].ns, alpha) for name, n, _, seed, alpha in insts]
                dts = [dt for _, _, dt, _, _ in insts]
                a = [ctx.state_upload(mids[name], st.rho, st.T, st.Y) for (name, *_), st in zip(insts, sts)]
                b = [ctx.state_upload(mids[name], st.rho, st.T, st.Y) for (name, *_), st in zip(insts, sts)]
                print(f"\n[noalloc] prec={prec} call {c}: {[(i[0], i[1]) for i in insts]}", flush=True)
                ctx.advance(a, dts, prec=prec)
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                ctx.advance_noalloc(b, dts, prec=prec)
                torch.cuda.synchronize()
                free1 = torch.cuda.mem_get_info()[0]
                for k, (ia, ib) in enumerate(zip(a, b)):
                    ra, rb = _full(ctx, ia), _full(ctx, ib)
                    _same(ra, rb, (prec, c, insts[k]))
                    assert np.all(rb[2] < 2), (prec, c, insts[k])
                # a second advance of the same instances: noalloc again against advance again; the
                # device's free memory does not move across the second noalloc call (the first may
                # see the runtime set up the launch stream's own resources)
                ctx.advance(a, dts, prec=prec)
                torch.cuda.synchronize()
                free2 = torch.cuda.mem_get_info()[0]
                ctx.advance_noalloc(b, dts, prec=prec)
                torch.cuda.synchronize()
                free3 = torch.cuda.mem_get_info()[0]
                print(f"[noalloc] free memory change: first call {free1 - free0} B, second call {free3 - free2} B",
                      flush=True)
                assert free2 - free3 < (2 << 20), (free2, free3)
                for k, (ia, ib) in enumerate(zip(a, b)):
                    _same(_full(ctx, ia), _full(ctx, ib), (prec, c, insts[k], "second step"))
                for i in a + b:
                    ctx.instance_release(i)
        # beyond the limit: 65 instances are refused before anything is launched
        st = synth.uniform_cells(16, 8, 9, 1.0)
        ids = [ctx.state_upload(mids["mech9"], st.rho, st.T, st.Y) for _ in range(65)]
        with pytest.raises(kin.KinError) as e:
            ctx.advance_noalloc(ids, [1e-6] * 65)
        assert e.value.status == kin.EINVAL and "at most 64" in str(e.value)
        ctx.advance_noalloc(ids[:64], [1e-6] * 64)
        ref = ctx.download(ids[64])
        ctx.advance([ids[64]], [1e-6])
        got = [ctx.download(i) for i in (ids[0], ids[64])]
        _same(got[0], got[1], "64 instances")
        assert not np.array_equal(ref[0], got[1][0])
        for i in ids:
            ctx.instance_release(i)
        for m in mids.values():
            ctx.mech_release(m)
