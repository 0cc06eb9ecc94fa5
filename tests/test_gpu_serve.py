"""Serving on the GPU: every request's result is the same in the mix as alone (bitwise, both
forms, layouts fixed per mechanism), admission holds the device pool within the budget, and the
pool returns to one free block after the run."""
import numpy as np
import pytest

from paper_1110_4903_amd import serve, synth

pytestmark = pytest.mark.gpu


def _setup(budget):
    from paper_1110_4903_amd import kin
    ctx = kin.Context(0, hbm_budget=budget)
    mids = {name: ctx.mech_upload(synth.mechanism(name)) for name in ("mech9", "mech36")}
    return ctx, mids


def _jobs(seed, n):
    # small requests so the test stays short: sizes log-normal around 600 cells
    reqs = synth.serving_requests(seed, n, rate_per_s=2000.0, median_cells=600, sigma_ln=1.0,
                                  cells_range=(1, 4000))
    return reqs, serve.make_jobs(reqs)


@pytest.mark.parametrize("prec,reserve,chunk,nstreams", [(0, 0, None, None), (1, 0, None, None), (1, 32, None, 2),
                                                        (0, 32, 700, 2)])
def test_alone_equals_mix(prec, reserve, chunk, nstreams):
    """chunk: requests above that many cells are served as parts (joined afterwards); nstreams:
    streams per request class shared by the slots (None: one per slot)."""
    budget = 8 << 20
    ctx, mids = _setup(budget)
    try:
        reqs, jobs = _jobs(40 + prec, 24)
        be = serve.KinBackend(ctx, mids, prec, n_slots=6, reserve_cu=reserve, n_streams=nstreams)
        for j, r in zip(jobs, reqs):
            be.prepare(j, r.inst.states(), max_chunk=chunk)
        rep = serve.run(jobs, be, budget, 6, max_chunk=chunk)
        s = rep.summary()
        print(f"\n[serve mix prec={prec} reserve={reserve} chunk={chunk} streams={nstreams}] " + " ".join(f"{k}={v}" for k, v in s.items()),
              flush=True)
        assert s["rejected"] == 0 and s["requests"] == len(jobs)
        assert rep.max_bytes_in_use <= budget and ctx.bytes_in_use() == 0
        assert ctx.largest_free() == budget
        assert rep.max_in_flight > 1, "no two requests overlapped"
        if chunk:
            assert any(j.n_cells > chunk for j in jobs)
        mixed = {r.rid: tuple(np.copy(a) for a in r.result) for r in rep.records}
        # each request alone and unsplit, in a fresh loop with one slot and no other traffic
        for j, r in zip(jobs, reqs):
            j.arrival = 0.0
            if chunk:
                be.prepare(j, r.inst.states())
            rep1 = serve.run([j], be, budget, 1)
            alone = rep1.records[0].result
            for a, b in zip(alone, mixed[j.rid]):
                assert np.array_equal(a, b), (j.rid, j.mech, j.n_cells)
        be.close()
    finally:
        ctx.close()


def test_pool_budget_and_coalescing():
    from paper_1110_4903_amd import kin
    budget = 4 << 20
    ctx, mids = _setup(budget)
    try:
        st = synth.uniform_cells(5, 2000, 9, 1.0)
        fp = ctx.footprint(mids["mech9"], 2000)
        ids = []
        with pytest.raises(kin.KinError) as e:
            while True:
                ids.append(ctx.state_upload(mids["mech9"], st.rho, st.T, st.Y))
        assert e.value.status == kin.ENOMEM and len(ids) == budget // fp
        assert ctx.bytes_in_use() == len(ids) * fp
        for i in ids[::2]:
            ctx.instance_release(i)
        for i in ids[1::2]:
            ctx.instance_release(i)
        assert ctx.bytes_in_use() == 0 and ctx.largest_free() == budget
    finally:
        ctx.close()
