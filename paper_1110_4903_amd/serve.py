"""Serving loop: continuous batching of chemistry solves of uneven size on one GPU.

Requests (a mechanism, a cell count, a dt and the cells' state in host memory) arrive over
time.  The loop keeps every mechanism resident on the device, queues arrivals in order and
admits the queue's head as soon as a slot is free and its HBM footprint fits the budget
(strict first-come-first-served, so no request waits behind a later one).  An admitted request
is uploaded, advanced and downloaded in stream order on its slot's stream, so the work of
requests admitted while others run overlaps on the device.  Its latency runs from arrival to
the moment the loop sees its results in host memory.

The loop itself knows nothing of HIP: a backend starts, polls and finishes requests, and a
clock gives the time.  KinBackend drives libkin; the tests also drive the loop with a
simulated backend and clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Job:
    rid: int
    arrival: float      # s since the start of the run
    mech: str
    n_cells: int
    dt: float
    state: object = None  # backend-specific inputs


@dataclasses.dataclass
class Part:
    """Cells [offset, offset + n_cells) of a job: the unit that is admitted and launched."""
    job: Job
    index: int
    offset: int
    n_cells: int

    @property
    def rid(self) -> int:
        return self.job.rid

    @property
    def mech(self) -> str:
        return self.job.mech

    @property
    def dt(self) -> float:
        return self.job.dt


def split(job: Job, max_chunk: Optional[int]) -> List[Part]:
    """A job as parts of at most max_chunk cells (one part when max_chunk is None)."""
    if not max_chunk or job.n_cells <= max_chunk:
        return [Part(job, 0, 0, job.n_cells)]
    k = -(-job.n_cells // max_chunk)
    base, extra = divmod(job.n_cells, k)  # k parts of nearly equal size, the larger ones first
    parts, off = [], 0
    for i in range(k):
        n = base + (1 if i < extra else 0)
        parts.append(Part(job, i, off, n))
        off += n
    return parts


@dataclasses.dataclass
class Record:
    rid: int
    mech: str
    n_cells: int
    arrival: float
    admitted: float
    done: float
    result: object = None
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def wait(self) -> float:
        """Queueing delay: arrival to the admission of the request's first part."""
        return self.admitted - self.arrival


@dataclasses.dataclass
class Report:
    records: List[Record]
    max_bytes_in_use: int
    max_in_flight: int
    start_order: List[int]
    wall_s: float

    def summary(self) -> dict:
        ok = [r for r in self.records if not r.rejected]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        cells = sum(r.n_cells for r in ok)
        first = min((r.arrival for r in ok), default=0.0)
        last = max((r.done for r in ok), default=0.0)
        span = max(last - first, 1e-12)
        out = dict(requests=len(ok), rejected=len(self.records) - len(ok), cells=cells,
                   cells_per_s=cells / span, p50_ms=1e3 * percentile(lat, 50),
                   p99_ms=1e3 * percentile(lat, 99), mean_ms=1e3 * float(lat.mean()),
                   max_in_flight=self.max_in_flight, max_bytes_in_use=self.max_bytes_in_use,
                   span_s=span)
        out["wait_p50_ms"] = 1e3 * percentile([r.wait for r in ok], 50)
        out["wait_p99_ms"] = 1e3 * percentile([r.wait for r in ok], 99)
        for mech in sorted({r.mech for r in ok}):
            lm = [r.latency for r in ok if r.mech == mech]
            out[f"{mech}_p50_ms"] = 1e3 * percentile(lm, 50)
            out[f"{mech}_p99_ms"] = 1e3 * percentile(lm, 99)
        # by request size: the tail of the small requests is the loop's responsiveness; that of
        # the large ones is mostly their own service time
        for name, lo, hi in SIZE_BUCKETS:
            lb = [r.latency for r in ok if lo <= r.n_cells < hi]
            if lb:
                out[f"cells_{name}_n"] = len(lb)
                out[f"cells_{name}_p50_ms"] = 1e3 * percentile(lb, 50)
                out[f"cells_{name}_p99_ms"] = 1e3 * percentile(lb, 99)
        return out


SIZE_BUCKETS = (("lt16k", 0, 16384), ("16k_128k", 16384, 131072), ("ge128k", 131072, 1 << 62))


def percentile(x, q) -> float:
    """Nearest-rank percentile (the smallest sample with at least q% of samples at or below)."""
    s = np.sort(np.asarray(x, dtype=float))
    if s.size == 0:
        return float("nan")
    k = max(int(np.ceil(q / 100.0 * s.size)) - 1, 0)
    return float(s[k])


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, next_arrival: Optional[float], backend) -> None:
        # nothing to do this round: yield briefly, but never sleep past the next arrival
        d = 50e-6 if next_arrival is None else min(50e-6, max(next_arrival - self.now(), 0.0))
        if d > 0:
            time.sleep(d)


def run(jobs: List[Job], backend, budget: int, n_slots: int, clock=None,
        max_chunk: Optional[int] = None) -> Report:
    """Serve `jobs` (sorted by arrival).  backend: footprint(part) -> bytes, start(part, slot)
    -> bool (False: no room on the device now, retry later), done(slot) -> bool, finish(slot)
    -> the part's result, and optionally join(job, [part results]) -> the job's result.  A job
    of more than max_chunk cells is queued as parts of at most max_chunk cells (split()), which
    are admitted and launched independently, in order; the job is done when its last part is.
    A job with a part whose footprint exceeds the whole budget is rejected."""
    clock = clock or WallClock()
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    queue: collections.deque = collections.deque()
    free = list(range(n_slots - 1, -1, -1))
    inflight: Dict[int, tuple] = {}
    used = 0
    records: List[Record] = []
    order: List[int] = []
    max_used = max_fl = 0
    left: Dict[int, int] = {}        # rid -> parts not finished
    first: Dict[int, float] = {}     # rid -> admission of its first part
    results: Dict[int, list] = {}
    rejected = set()
    t_start = clock.now()
    while pending or queue or inflight:
        now = clock.now()
        while pending and pending[0].arrival <= now:
            job = pending.popleft()
            parts = split(job, max_chunk)
            left[job.rid] = len(parts)
            results[job.rid] = [None] * len(parts)
            queue.extend(parts)
        progressed = False
        for slot in list(inflight):
            if backend.done(slot):
                part, fp, t_adm = inflight.pop(slot)
                results[part.rid][part.index] = backend.finish(slot)
                used -= fp
                free.append(slot)
                progressed = True
                left[part.rid] -= 1
                if left[part.rid] == 0:
                    job = part.job
                    res = results.pop(job.rid)
                    res = res[0] if len(res) == 1 else (backend.join(job, res) if hasattr(backend, "join") else res)
                    records.append(Record(job.rid, job.mech, job.n_cells, job.arrival, first.pop(job.rid),
                                          clock.now(), res))
        while queue and free:
            part = queue[0]
            if part.rid in rejected:
                queue.popleft()
                continue
            fp = backend.footprint(part)
            if fp > budget:
                queue.popleft()
                rejected.add(part.rid)
                t = clock.now()
                job = part.job
                records.append(Record(job.rid, job.mech, job.n_cells, job.arrival, t, t, None, rejected=True))
                progressed = True
                continue
            if used + fp > budget:
                break
            slot = free.pop()
            if not backend.start(part, slot):
                free.append(slot)
                if not inflight:
                    raise RuntimeError(f"request {part.rid} fits the budget but the device has no room "
                                       "for it with nothing in flight")
                break
            queue.popleft()
            used += fp
            t = clock.now()
            inflight[slot] = (part, fp, t)
            if part.index == 0:
                first[part.rid] = t
                order.append(part.rid)
            max_used = max(max_used, used)
            max_fl = max(max_fl, len(inflight))
            progressed = True
        if not progressed:
            clock.idle(pending[0].arrival if pending else None, backend)
    return Report(records, max_used, max_fl, order, clock.now() - t_start)


class KinBackend:
    """Requests through libkin: one stream per slot; upload from pinned host memory, advance
    and download in stream order; completion seen through an event on the slot's stream.

    reserve_cu > 0: requests of the mechanisms in `heavy` (long launches) run on streams whose
    kernels are confined to the first num_cu - reserve_cu compute units, so the remaining units
    stay available to the other requests, which would otherwise wait for units to drain.

    n_streams: streams per class (light, heavy) shared round-robin by the slots; by default one
    per slot.  The device runs a few hardware queues per process (four by default), and a
    kernel waits behind whatever precedes it in its queue: with two light and two heavy streams
    the light requests never queue behind a heavy launch.
    """

    def __init__(self, ctx, mech_ids: Dict[str, int], prec: int, n_slots: int, opts=None,
                 reserve_cu: int = 0, heavy=("mech36",), n_streams: Optional[int] = None):
        import torch
        from . import kin
        self.torch = torch
        self.ctx, self.mids, self.prec, self.opts = ctx, mech_ids, prec, opts
        ns = n_streams or n_slots
        self.streams = [torch.cuda.Stream() for _ in range(ns)]
        self.events = [torch.cuda.Event() for _ in range(n_slots)]
        self.heavy = set(heavy)
        self._raw = []
        self.heavy_streams = None
        if reserve_cu > 0:
            ncu = ctx.query_int(kin.Q_NUM_CU)
            if not 0 < reserve_cu < ncu:
                raise ValueError(f"reserve_cu must be in 1..{ncu - 1}")
            self._raw = [ctx.stream_create(0, ncu - reserve_cu) for _ in range(ns)]
            self.heavy_streams = [torch.cuda.ExternalStream(h) for h in self._raw]
        self.slot: Dict[int, tuple] = {}
        self._ns = {name: ctx.mech_ns[mid] for name, mid in mech_ids.items()}
        self._fp: Dict[tuple, int] = {}

    def close(self):
        self.torch.cuda.synchronize()
        for h in self._raw:
            self.ctx.stream_destroy(h)
        self._raw = []
        self.heavy_streams = None

    def prepare(self, job: Job, st, max_chunk: Optional[int] = None) -> None:
        """Pinned host copies of a request's inputs and room for its outputs, per part (the
        same max_chunk as the loop's)."""
        torch = self.torch
        pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        ns = self._ns[job.mech]
        parts = []
        for p in split(job, max_chunk):
            c = slice(p.offset, p.offset + p.n_cells)
            parts.append(dict(rho=pin(st.rho[c]), T=pin(st.T[c]), Y=pin(st.Y[:, c]),
                              T_out=torch.empty(p.n_cells, dtype=torch.float64, pin_memory=True),
                              Y_out=torch.empty((ns, p.n_cells), dtype=torch.float64, pin_memory=True),
                              status=torch.empty(p.n_cells, dtype=torch.int32, pin_memory=True)))
        job.state = parts

    def footprint(self, part: Part) -> int:
        key = (part.mech, part.n_cells)
        if key not in self._fp:
            self._fp[key] = self.ctx.footprint(self.mids[part.mech], part.n_cells, self.prec)
        return self._fp[key]

    def start(self, part: Part, slot: int) -> bool:
        from . import kin
        s = self.streams[slot % len(self.streams)]
        if self.heavy_streams is not None and part.mech in self.heavy:
            s = self.heavy_streams[slot % len(self.heavy_streams)]
        d = part.job.state[part.index]
        try:
            iid = self.ctx.state_upload(self.mids[part.mech], d["rho"], d["T"], d["Y"], stream=s)
        except kin.KinError as e:
            if e.status == kin.ENOMEM:
                return False
            raise
        self.ctx.advance([iid], [part.dt], prec=self.prec, opts=self.opts, stream=s)
        self.ctx.download_device(iid, d["T_out"], d["Y_out"], status=d["status"], stream=s)
        self.events[slot].record(s)
        self.slot[slot] = (part, iid)
        return True

    def done(self, slot: int) -> bool:
        return self.events[slot].query()

    def finish(self, slot: int):
        part, iid = self.slot.pop(slot)
        self.ctx.instance_release(iid)
        d = part.job.state[part.index]
        return d["T_out"].numpy(), d["Y_out"].numpy(), d["status"].numpy()

    def join(self, job: Job, results):
        """A split request's result: its parts' outputs side by side, in cell order."""
        return (np.concatenate([r[0] for r in results]), np.concatenate([r[1] for r in results], axis=1),
                np.concatenate([r[2] for r in results]))


def make_jobs(requests, time_scale: float = 1.0) -> List[Job]:
    """Jobs from synth.Request records (arrival times multiplied by time_scale)."""
    return [Job(k, r.arrival * time_scale, r.inst.mech, r.inst.n_cells, r.inst.dt) for k, r in enumerate(requests)]
