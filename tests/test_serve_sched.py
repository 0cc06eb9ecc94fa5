"""The serving loop's host logic on a simulated device and clock (CPU only): admission never
exceeds the HBM budget or the slot count, requests start in arrival order and all finish,
oversized requests are rejected, and latencies are accounted from arrival to completion."""
import numpy as np
import pytest

from paper_1110_4903_amd import serve, synth


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def idle(self, next_arrival, backend):
        nxt = [x for x in (next_arrival, backend.next_completion()) if x is not None]
        assert nxt, "loop idles with nothing left to wait for"
        self.t = max(self.t, min(nxt))


class SimBackend:
    """Each request occupies bytes_per_cell * n bytes and finishes n / rate seconds after it
    starts; device memory is tracked independently of the loop's own accounting."""

    def __init__(self, clock, rate, bytes_per_cell, capacity):
        self.clock, self.rate, self.bpc, self.capacity = clock, rate, bytes_per_cell, capacity
        self.used = 0
        self.peak = 0
        self.running = {}

    def footprint(self, job):
        return self.bpc[job.mech] * job.n_cells

    def start(self, job, slot):
        fp = self.footprint(job)
        assert slot not in self.running
        if self.used + fp > self.capacity:
            return False
        self.used += fp
        self.peak = max(self.peak, self.used)
        self.running[slot] = (job, fp, self.clock.now() + job.n_cells / self.rate)
        return True

    def done(self, slot):
        return self.running[slot][2] <= self.clock.now()

    def finish(self, slot):
        job, fp, _ = self.running.pop(slot)
        self.used -= fp
        return job.rid

    def next_completion(self):
        return min((r[2] for r in self.running.values()), default=None)


def _jobs(seed, n, rate):
    return serve.make_jobs(synth.serving_requests(seed, n, rate))


BPC = {"mech9": 100, "mech36": 330}


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_budget_slots_and_order(seed):
    jobs = _jobs(seed, 300, 40.0)
    budget = 30_000_000
    clk = SimClock()
    be = SimBackend(clk, 1.0e6, BPC, budget)
    rep = serve.run(jobs, be, budget, 8, clk)
    assert len(rep.records) == len(jobs)
    assert rep.max_bytes_in_use <= budget and be.peak <= budget
    assert rep.max_in_flight <= 8
    # first come, first served: starts follow arrivals
    assert rep.start_order == sorted(rep.start_order)
    assert all(r.done >= r.admitted >= r.arrival for r in rep.records)
    assert be.used == 0 and not be.running


def test_admission_binds_and_rejects_oversized():
    jobs = [serve.Job(0, 0.0, "mech9", 1000, 1e-6), serve.Job(1, 0.0, "mech9", 1000, 1e-6),
            serve.Job(2, 0.0, "mech36", 100000, 1e-6), serve.Job(3, 0.0, "mech9", 500, 1e-6)]
    clk = SimClock()
    be = SimBackend(clk, 1000.0, BPC, 150_000)
    rep = serve.run(jobs, be, 150_000, 4, clk)
    rec = {r.rid: r for r in rep.records}
    assert rec[2].rejected and not rec[0].rejected
    # job 1 waits for job 0's memory: 1000 + 1000 cells x 100 B exceed 150 kB
    assert rec[0].done == pytest.approx(1.0) and rec[1].admitted == pytest.approx(1.0)
    assert rec[1].done == pytest.approx(2.0)
    # job 3 (50 kB) is behind job 1 in the queue and fits beside it
    assert rec[3].admitted == pytest.approx(1.0) and rec[3].done == pytest.approx(1.5)


def test_latency_accounting_single_slot():
    """One slot, service n/rate: the k-th latency is the Lindley recursion of the queue."""
    rng = np.random.default_rng(0)
    arr = np.cumsum(rng.exponential(1.0, 50))
    n = rng.integers(100, 2000, 50)
    jobs = [serve.Job(k, float(a), "mech9", int(c), 1e-6) for k, (a, c) in enumerate(zip(arr, n))]
    clk = SimClock()
    be = SimBackend(clk, 1000.0, BPC, 10**9)
    rep = serve.run(jobs, be, 10**9, 1, clk)
    free_at = 0.0
    want = []
    for a, c in zip(arr, n):
        start = max(a, free_at)
        free_at = start + c / 1000.0
        want.append(free_at - a)
    got = [r.latency for r in sorted(rep.records, key=lambda r: r.rid)]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    s = rep.summary()
    assert s["p50_ms"] == pytest.approx(1e3 * serve.percentile(want, 50))
    assert s["p99_ms"] == pytest.approx(1e3 * max(want))


def test_percentile_nearest_rank():
    x = list(range(1, 101))
    assert serve.percentile(x, 50) == 50 and serve.percentile(x, 99) == 99 and serve.percentile(x, 100) == 100
    assert serve.percentile([3.0], 99) == 3.0


class PartBackend(SimBackend):
    """SimBackend whose results name the cells each part covered; join() checks their order."""

    def finish(self, slot):
        part, fp, _ = self.running.pop(slot)
        self.used -= fp
        return (part.rid, part.index, part.offset, part.n_cells)

    def join(self, job, results):
        assert [r[1] for r in results] == list(range(len(results)))
        assert results[0][2] == 0 and sum(r[3] for r in results) == job.n_cells
        assert all(a[2] + a[3] == b[2] for a, b in zip(results, results[1:]))
        return job.rid


@pytest.mark.parametrize("n,chunk", [(1, 4), (10, 4), (12, 4), (100000, 65536), (7, None), (7, 7)])
def test_split_covers_the_cells(n, chunk):
    job = serve.Job(0, 0.0, "mech9", n, 1e-6)
    parts = serve.split(job, chunk)
    assert parts[0].offset == 0 and sum(p.n_cells for p in parts) == n
    assert all(a.offset + a.n_cells == b.offset for a, b in zip(parts, parts[1:]))
    assert [p.index for p in parts] == list(range(len(parts)))
    if chunk:
        sizes = [p.n_cells for p in parts]
        assert max(sizes) <= chunk and max(sizes) - min(sizes) <= 1
        assert len(parts) == -(-n // chunk)


@pytest.mark.parametrize("seed", [7, 8])
def test_split_requests_budget_order_and_joining(seed):
    """Requests above 20k cells go as parts: budget and slots hold, requests start in arrival
    order with their parts in order, every request is joined from all its parts in cell order."""
    jobs = _jobs(seed, 200, 40.0)
    budget = 30_000_000
    clk = SimClock()
    be = PartBackend(clk, 1.0e6, BPC, budget)
    rep = serve.run(jobs, be, budget, 8, clk, max_chunk=20000)
    assert len(rep.records) == len(jobs)
    # a split request's result comes from join(); an unsplit one's is its single part's
    assert all(r.result == (r.rid if r.n_cells > 20000 else (r.rid, 0, 0, r.n_cells)) for r in rep.records)
    assert rep.max_bytes_in_use <= budget and be.peak <= budget and rep.max_in_flight <= 8
    assert rep.start_order == sorted(rep.start_order)
    assert all(r.done >= r.admitted >= r.arrival for r in rep.records)
    assert be.used == 0 and not be.running
    assert any(j.n_cells > 20000 for j in jobs)


def test_split_single_slot_keeps_latencies():
    """With one slot the parts of a request run back to back, so splitting changes no latency
    (service times add up): the records equal those of the unsplit run."""
    rng = np.random.default_rng(3)
    arr = np.cumsum(rng.exponential(1.0, 40))
    n = rng.integers(100, 5000, 40)
    mk = lambda: [serve.Job(k, float(a), "mech9", int(c), 1e-6) for k, (a, c) in enumerate(zip(arr, n))]
    out = []
    for chunk in (None, 700):
        clk = SimClock()
        rep = serve.run(mk(), PartBackend(clk, 1000.0, BPC, 10**9), 10**9, 1, clk, max_chunk=chunk)
        out.append(sorted((r.rid, r.admitted, r.done) for r in rep.records))
    for (r0, a0, d0), (r1, a1, d1) in zip(*out):
        assert r0 == r1 and a0 == pytest.approx(a1, abs=1e-9) and d0 == pytest.approx(d1, abs=1e-9)


def test_split_request_runs_its_parts_side_by_side():
    """A lone request of 4 parts on 4 free slots: the parts start together and the request is
    done after a quarter of its unsplit service time; wait and size statistics are reported."""
    clk = SimClock()
    rep = serve.run([serve.Job(0, 0.0, "mech9", 4000, 1e-6)], PartBackend(clk, 1000.0, BPC, 10**9), 10**9, 4,
                    clk, max_chunk=1000)
    r = rep.records[0]
    assert r.done == pytest.approx(1.0) and r.wait == 0.0 and rep.max_in_flight == 4
    s = rep.summary()
    assert s["wait_p99_ms"] == 0.0 and s["cells_lt16k_n"] == 1 and s["cells_lt16k_p99_ms"] == pytest.approx(1e3)
