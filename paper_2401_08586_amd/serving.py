"""Serving loop: neighbour-search requests from many concurrent simulations on one GPU.

Each simulation keeps its particles, its CSR outputs and its sorted cell structure
resident in HBM between time steps; a request asks for one step (the particles move by the
simulation's displacement, then the structure is updated and searched). Requests are
served continuously: whenever one of the stream slots is free, the oldest queued request
whose simulation is idle starts on it, so requests that arrive while others run are
admitted as slots and memory free up, and their work overlaps on the device. The first
step of a resident simulation builds its structure; every later step is the incremental
update (the displacement applied on the device and only migrating particles re-binned)
plus count and fill, replayed from the HIP graph its structure captured (one launch per
request). With per_sim=False the requests of a slot are instead batched (up to a particle
budget) into one library batch call (move, then a full build + search) on a structure per
slot. Simulations are admitted into HBM by a byte budget, by default the device's free
memory (re-read before every admission) less a reserve: before a request runs, idle
simulations are evicted (positions to pinned host memory, outputs and cell structure
freed) in least-recently-used order until it fits.

The scheduler (`Scheduler`) is host logic only and is tested on the CPU; `Server` drives
the library through the binding in `nnps.py`. Every search runs in the HIP library; the
simulation's own work between steps, drawing its displacement (uniform per component,
reflected at the box), is a few elementwise torch operations on the slot's stream,
ordered before the sim's next step by an event.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Request:
    sim: int
    arrival: float                 # seconds after the run's start
    issued: float | None = None    # host time the batch holding it was launched (s)
    done_ms: float | None = None   # device completion time (ms after the run's start)
    device_ms: float = 0.0         # device time of its batch (events around the step)
    nnz: int = 0
    batch: int = -1
    step: int = -1

    @property
    def latency_ms(self) -> float:
        return self.done_ms - 1e3 * self.arrival

    @property
    def queue_ms(self) -> float:
        """Arrival to launch: waiting for a slot, for its simulation's previous step, or
        for the scheduler loop to see it."""
        return 1e3 * (self.issued - self.arrival)


class Scheduler:
    """Queue, batch formation and HBM admission (host logic, no device calls).

    sizes[s] = particles of simulation s; nbytes[s] = its resident footprint in bytes
    (positions + CSR outputs). At most one request per simulation is in flight; later
    requests of a busy simulation wait in arrival order."""

    def __init__(self, sizes, nbytes, budget_bytes: float = math.inf, max_batch_particles: int = 1 << 23,
                 groups=None):
        self.sizes = list(sizes)
        # requests of one batch share a group (the library batches sets of one dimension)
        self.groups = list(groups) if groups is not None else [0] * len(self.sizes)
        self.nbytes = list(nbytes)
        self.budget = budget_bytes
        self.max_batch = max_batch_particles
        self.queue: collections.deque[Request] = collections.deque()
        self.busy: set[int] = set()
        self.resident: collections.OrderedDict[int, None] = collections.OrderedDict()  # LRU order
        self.evictions = 0
        self.admissions = 0

    def push(self, req: Request):
        self.queue.append(req)

    def pending(self) -> int:
        return len(self.queue)

    def resident_bytes(self) -> int:
        return sum(self.nbytes[s] for s in self.resident)

    def next_batch(self) -> list[Request]:
        """Requests for the next batch, in arrival order: each idle simulation's oldest
        request of the first eligible request's group, until the particle budget is
        reached (the first one always fits)."""
        chosen: list[Request] = []
        taken: set[int] = set()
        total = 0
        keep: collections.deque[Request] = collections.deque()
        while self.queue:
            r = self.queue.popleft()
            if (r.sim in self.busy or r.sim in taken
                    or (chosen and self.groups[r.sim] != self.groups[chosen[0].sim])
                    or (chosen and total + self.sizes[r.sim] > self.max_batch)):
                keep.append(r)
                continue
            chosen.append(r)
            taken.add(r.sim)
            total += self.sizes[r.sim]
        self.queue = keep
        return chosen

    def admit(self, sims) -> tuple[list[int], list[int]]:
        """Make `sims` resident within the budget. Returns (to_admit, to_evict): idle
        resident simulations outside `sims` are evicted least recently used first. A batch
        larger than the budget on its own is still admitted, with everything else evicted."""
        need = [s for s in sims if s not in self.resident]
        want = sum(self.nbytes[s] for s in need)
        evict: list[int] = []
        have = self.resident_bytes()
        for s in list(self.resident):
            if have + want <= self.budget:
                break
            if s in sims or s in self.busy:
                continue
            evict.append(s)
            have -= self.nbytes[s]
        for s in evict:
            del self.resident[s]
        for s in sims:
            self.resident[s] = None
            self.resident.move_to_end(s)
        self.evictions += len(evict)
        self.admissions += len(need)
        return need, evict

    def start(self, sims):
        self.busy.update(sims)

    def finish(self, sims):
        self.busy.difference_update(sims)


def poisson_arrivals(rate: float, count: int, nsims: int, seed: int = 0, start: float = 0.0):
    """`count` arrivals of a Poisson process of `rate` per second, each for a simulation
    drawn uniformly; returns [(time_s, sim)] in time order."""
    rng = np.random.default_rng(seed)
    t = start + np.cumsum(rng.exponential(1.0 / rate, size=count))
    sims = rng.integers(0, nsims, size=count)
    return [(float(a), int(b)) for a, b in zip(t, sims)]


def percentile(values, q):
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))


class Server:
    """Runs the request loop on one GPU. `sims` are workloads.ParticleSet; `slots` is the
    number of batches that may be on the device at once (one stream each)."""

    def __init__(self, sims, slots: int = 4, budget_bytes: float | None = None, max_batch_particles: int = 1 << 23,
                 seed: int = 4, frac: float = 0.05, headroom: float = 1.1, ctx=None, keep_results: bool = False,
                 per_sim: bool = True, reserve_bytes: float = 2 << 30, use_update: bool = True):
        import torch
        from . import nnps
        self.torch = torch
        self.nnps = nnps
        self.ctx = ctx or nnps.Context(0)
        self.own_ctx = ctx is None
        self.sims = sims
        self.seed = seed
        self.frac = frac
        self.headroom = headroom
        self.keep_results = keep_results
        self.results = {}  # (sim, step) -> (pos, row_ptr, col, dist) copies when keep_results
        # per_sim: every resident simulation keeps its own cell structure, and each step is
        # one replay of that structure's captured graph; otherwise the requests of a slot
        # are batched into one library batch call on the slot's structure
        self.per_sim = per_sim
        # per_sim: steps after a simulation's first one update its structure incrementally
        self.use_update = use_update and per_sim
        # budget_bytes None: free device memory, re-read before each admission, less a reserve
        self.auto_budget = budget_bytes is None
        self.reserve = reserve_bytes
        self.cells = [None] * len(sims)
        self.built = [False] * len(sims)   # the simulation's own structure holds its last step
        n = len(sims)
        self.step = [0] * n
        self.pos = [None] * n       # device positions (resident) or None
        self.host = [None] * n      # pinned host positions while evicted
        self.rp = [None] * n
        self.col = [None] * n
        self.dist = [None] * n
        self.cap = [0] * n
        self.ready = [None] * n     # event: positions of the next step are in place
        self.gen = {}               # per-simulation device generator (reseeded every step)
        self.disp = {}              # per-simulation displacement buffer of the motion
        self.pending = [False] * n  # a displacement is drawn but not yet applied
        self.box = [(torch.tensor(ps.lo, dtype=torch.float64, device="cuda"),
                     torch.tensor(ps.hi, dtype=torch.float64, device="cuda")) for ps in sims]
        # initial capacity estimate per simulation from one search of its starting positions
        cells = self.ctx.cells()
        for s, ps in enumerate(sims):
            self.host[s] = torch.from_numpy(np.ascontiguousarray(ps.pos)).pin_memory()
            pos = self.host[s].cuda()
            rp, col, _, _ = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=self.ctx, cells=cells)
            self.cap[s] = int(col.numel() * headroom) + 4096
            del pos, rp, col
        cells.close()
        nbytes = [self._footprint(s) for s in range(len(sims))]
        self.sched = Scheduler([ps.n for ps in sims], nbytes, math.inf if budget_bytes is None else budget_bytes,
                               1 if per_sim else max_batch_particles, groups=[ps.dim for ps in sims])
        self.slots = []
        for _ in range(slots):
            c = self.ctx.cells()
            self.slots.append({"stream": torch.cuda.Stream(), "cells": c, "batch": None, "done": None})
        self.batches = 0
        torch.cuda.synchronize()

    # -- resident state ------------------------------------------------------------------
    def _footprint(self, s):
        """Device bytes a resident simulation holds: positions and the motion's displacement
        buffer, CSR outputs and, per simulation, its cell structure (about 200 bytes per particle plus the dense-cell
        lists' 16 bytes per stencil entry, 3^d per particle)."""
        ps = self.sims[s]
        b = 2 * ps.n * ps.dim * 8 + (ps.n + 1) * 8 + self.cap[s] * 8
        if self.per_sim:
            b += ps.n * (200 + 16 * 3 ** ps.dim)
        return b

    def _free_budget(self):
        """Bytes the resident simulations may hold: what they hold now plus the device's free
        memory (the driver's, and blocks torch's allocator has cached but not handed out)
        less the reserve."""
        torch = self.torch
        free, _ = torch.cuda.mem_get_info()
        cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
        return self.sched.resident_bytes() + free + cached - self.reserve

    def _admit(self, s, stream):
        torch = self.torch
        ps = self.sims[s]
        with torch.cuda.stream(stream):
            self.pos[s] = self.host[s].to("cuda", non_blocking=True)
            self.rp[s] = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
            self.col[s] = torch.empty(self.cap[s], dtype=torch.int32, device="cuda")
            self.dist[s] = torch.empty(self.cap[s], dtype=torch.float32, device="cuda")
        self.host[s] = None
        self.built[s] = False
        if self.per_sim:
            self.cells[s] = self.ctx.cells()
            self.cells[s].set_graphs(True)

    def _evict(self, s):
        torch = self.torch
        # an idle simulation: its last step (and motion) finished; wait for that motion
        if self.ready[s] is not None:
            self.ready[s].synchronize()
        self._apply(s, torch.cuda.current_stream())  # a drawn displacement goes with the positions
        torch.cuda.current_stream().synchronize()
        host = torch.empty(self.pos[s].shape, dtype=torch.float64, pin_memory=True)
        host.copy_(self.pos[s])
        self.host[s] = host
        self.pos[s] = self.rp[s] = self.col[s] = self.dist[s] = None
        self.disp.pop(s, None)
        self.ready[s] = None
        self.built[s] = False
        if self.cells[s] is not None:
            self.cells[s].close()
            self.cells[s] = None

    def _apply(self, s, stream):
        """Apply a drawn displacement to the positions as the library's update does (paths
        that rebuild instead of updating): p + d, or p - d for a component where p + d would
        leave the box."""
        if self.pending[s]:
            torch = self.torch
            lo, hi = self.box[s]
            with torch.cuda.stream(stream):
                p, d = self.pos[s], self.disp[s]
                q = p + d
                p.copy_(torch.where((q >= lo) & (q <= hi), q, p - d))
            self.pending[s] = False

    def _move(self, s, stream):
        """The simulation's time step: a displacement U(-frac dx, +frac dx) per component,
        dx = radius / 2.4 (seeded per simulation and step; one device launch). The next
        step's update applies it, reflecting a component that would leave the box (the
        rebuild paths apply it the same way first)."""
        torch = self.torch
        ps = self.sims[s]
        g = self.gen.get(s)
        if g is None:
            g = self.gen[s] = torch.Generator(device="cuda")
        g.manual_seed(self.seed * 1_000_003 + s * 65_537 + self.step[s])
        a = self.frac * ps.radius / 2.4
        with torch.cuda.stream(stream):
            p = self.pos[s]
            d = self.disp.get(s)
            if d is None or d.shape != p.shape:
                d = self.disp[s] = torch.empty_like(p)
            d.uniform_(-a, a, generator=g)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.pending[s] = True
        self.ready[s] = ev

    # -- the loop -------------------------------------------------------------------------
    def _launch(self, slot, reqs, t0):
        torch, nnps = self.torch, self.nnps
        stream = slot["stream"]
        sims = [r.sim for r in reqs]
        if self.auto_budget:
            self.sched.budget = self._free_budget()
        admit, evict = self.sched.admit(sims)
        for s in evict:
            self._evict(s)
        for s in admit:
            self._admit(s, stream)
        for s in sims:
            if self.ready[s] is not None:
                stream.wait_event(self.ready[s])
        sets = [(self.pos[s], self.sims[s].lo, self.sims[s].hi, self.sims[s].cell_size, self.sims[s].radius)
                for s in sims]
        cells = self.cells[sims[0]] if self.per_sim else slot["cells"]
        outs = ([self.rp[s] for s in sims], [self.col[s] for s in sims], [self.dist[s] for s in sims])
        with torch.cuda.stream(stream):
            begin = torch.cuda.Event(enable_timing=True)
            begin.record(stream)
            if self.use_update and self.built[sims[0]]:
                s0 = sims[0]
                cells.batch_update_step(*outs, disp=[self.disp[s0] if self.pending[s0] else None], stream=stream)
                self.pending[s0] = False
            else:
                for s in sims:
                    self._apply(s, stream)
                cells.batch_step(sets, *outs, stream=stream)
                if self.per_sim:
                    self.built[sims[0]] = True
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
            cells.batch_nnz_enqueue(stream=stream)
        slot["used"] = cells
        now = time.perf_counter() - t0
        for r in reqs:
            r.issued = now
            r.batch = self.batches
            r.step = self.step[r.sim]
        self.sched.start(sims)
        slot["batch"] = reqs
        slot["done"] = done
        slot["begin"] = begin
        self.batches += 1

    def _finish(self, slot, ref):
        torch, nnps = self.torch, self.nnps
        reqs = slot["batch"]
        stream = slot["stream"]
        done_ms = ref.elapsed_time(slot["done"])
        device_ms = slot["begin"].elapsed_time(slot["done"])
        nnz, code = slot["used"].batch_nnz_fetch(check=False)
        sims = [r.sim for r in reqs]
        redo = []
        for r, k in zip(reqs, nnz):
            s = r.sim
            if k > self.cap[s]:
                redo.append(r)
                continue
            r.nnz = int(k)
            r.done_ms = done_ms
            r.device_ms = device_ms
            if self.keep_results:  # copies ordered before the motion on the same stream
                with torch.cuda.stream(stream):
                    self.results[(s, self.step[s])] = (self.pos[s].clone(), self.rp[s].clone(),
                                                       self.col[s][:k].clone(), self.dist[s][:k].clone())
            self.step[s] += 1
            self._move(s, stream)
        if code not in (nnps.NNPS_OK, nnps.NNPS_ECAPACITY):
            raise nnps.NnpsError(code, "serving batch")
        for r in redo:  # outputs too small: grow them and run that step again (rebuilt) first
            s = r.sim
            self.built[s] = False
            self.cap[s] = int(nnz[sims.index(s)] * self.headroom) + 4096
            self.sched.nbytes[s] = self._footprint(s)
            with torch.cuda.stream(stream):
                self.col[s] = torch.empty(self.cap[s], dtype=torch.int32, device="cuda")
                self.dist[s] = torch.empty(self.cap[s], dtype=torch.float32, device="cuda")
            self.sched.queue.appendleft(r)
        self.sched.finish(sims)
        slot["batch"] = None
        slot["done"] = None

    def run(self, arrivals, closed_loop: int = 0):
        """Serve `arrivals` ([(time_s, sim)], time order). With closed_loop = k > 0 the
        arrivals are ignored and every simulation always has a request waiting (each
        completion immediately issues the next) until k requests have completed: the
        saturated rate. Returns the completed requests."""
        torch = self.torch
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        ref.synchronize()
        t0 = time.perf_counter()
        done: list[Request] = []
        arr = collections.deque(arrivals)
        if closed_loop:
            for s in range(len(self.sims)):
                self.sched.push(Request(s, 0.0))
        total = closed_loop if closed_loop else len(arrivals)
        while len(done) < total:
            now = time.perf_counter() - t0
            while arr and not closed_loop and arr[0][0] <= now:
                a, s = arr.popleft()
                self.sched.push(Request(s, a))
            progressed = False
            for slot in self.slots:
                if slot["batch"] is not None and slot["done"].query():
                    reqs = slot["batch"]
                    self._finish(slot, ref)
                    finished = [r for r in reqs if r.done_ms is not None]
                    done.extend(finished)
                    if closed_loop:
                        for r in finished:  # each completion issues that simulation's next step
                            if len(done) + self.sched.pending() + len(self.sched.busy) < total:
                                self.sched.push(Request(r.sim, time.perf_counter() - t0))
                    progressed = True
            for slot in self.slots:
                if slot["batch"] is None and self.sched.pending():
                    reqs = self.sched.next_batch()
                    if reqs:
                        self._launch(slot, reqs, t0)
                        progressed = True
            if not progressed:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        return done

    def counters(self) -> dict:
        """Admissions and evictions so far, and the budget last used."""
        return {"admissions": self.sched.admissions, "evictions": self.sched.evictions,
                "budget_bytes": None if math.isinf(self.sched.budget) else float(self.sched.budget),
                "auto_budget": self.auto_budget}

    def close(self):
        for slot in self.slots:
            slot["cells"].close()
        for c in self.cells:
            if c is not None:
                c.close()
        if self.own_ctx:
            self.ctx.close()


def summarize(done, warmup: int = 0):
    """p50/p99 latency (ms, arrival -> CSR ready), throughput and counts over the requests
    after the first `warmup` completions (in arrival order)."""
    reqs = sorted(done, key=lambda r: r.arrival)[warmup:]
    if not reqs:
        return {}
    lat = [r.latency_ms for r in reqs]
    t_first = min(r.arrival for r in reqs) * 1e3
    t_last = max(r.done_ms for r in reqs)
    pairs = sum(r.nnz for r in reqs)
    span_s = max((t_last - t_first) * 1e-3, 1e-9)
    qw = [r.queue_ms for r in reqs]
    dev = [r.device_ms for r in reqs]
    # the tail: requests at or above the p99 latency, their mean queue wait and device time
    p99 = percentile(lat, 99)
    tail = [r for r in reqs if r.latency_ms >= p99]
    return {"requests": len(reqs), "p50_ms": percentile(lat, 50), "p99_ms": p99,
            "mean_ms": float(np.mean(lat)), "max_ms": float(np.max(lat)),
            "gpairs_per_s": pairs / span_s / 1e9, "requests_per_s": len(reqs) / span_s,
            "batches": len({r.batch for r in reqs}),
            "mean_batch": len(reqs) / max(len({r.batch for r in reqs}), 1),
            "queue_p50_ms": percentile(qw, 50), "queue_p99_ms": percentile(qw, 99),
            "device_p50_ms": percentile(dev, 50), "device_p99_ms": percentile(dev, 99),
            "tail_queue_ms": float(np.mean([r.queue_ms for r in tail])),
            "tail_device_ms": float(np.mean([r.device_ms for r in tail]))}
