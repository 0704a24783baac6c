"""Continuous-batching service for ensembles of independent single-level simulations.

Requests (lattice size N, step count, precision, seed, arrival time) arrive over time.
The server keeps every admitted job's state resident in HBM, admits queued jobs in
arrival order while their arenas fit the memory budget, and advances all resident jobs
together: one batched launch per kernel per step for each precision (sh_batch_advance),
so jobs that arrive while others run overlap on the device.  Finished jobs release
their memory at once, which lets waiting jobs in.  Each job's result is bit-identical
to running it alone.

``serve`` runs a request list against the wall clock and returns per-job timings;
``serve_fifo`` runs the same list one job at a time (the baseline, run for real).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import shamr


@dataclass
class Job:
    jid: int
    n: int
    steps: int
    prec: int
    seed: int
    arrival: float
    U0: np.ndarray = field(repr=False, default=None)
    beta: int = 2
    h: object = field(repr=False, default=None)
    nbytes: int = 0
    done_steps: int = 0
    t_admit: float = None
    t_join: float = None
    t_done: float = None
    result: np.ndarray = field(repr=False, default=None)
    staged: object = field(repr=False, default=None)
    ready: object = field(repr=False, default=None)
    out: object = field(repr=False, default=None)

    @property
    def cell_stages(self) -> int:
        return self.n ** 3 * 4 * self.steps


def make_hierarchy(job: Job, stream):
    h = shamr.Hierarchy(job.n, float(job.n), 0.25, 0.1, 1.0, 2.0, job.beta, max_level=0, prec=job.prec,
                        stream=stream)
    box = [(0, 0, 0, job.n - 1, job.n - 1, job.n - 1)]
    h.set_layout(0, box)
    h.write_dense(0, job.U0)
    h.fill_ghosts(0)
    return h


def arena_bytes(job: Job) -> int:
    p = shamr.sh_params(job.n, float(job.n), 0.25, 0.1, 1.0, 2.0, job.beta, 0, 8, 64, 2, job.prec, 4, 1, 1, 0, 0.0, 0)
    b = np.array([0, 0, 0, job.n - 1, job.n - 1, job.n - 1], np.int32)
    import ctypes
    return int(shamr.load().sh_arena_bytes(ctypes.byref(p), 0, 1, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))


class Pool:
    """Hierarchies of finished jobs, kept for later jobs of the same lattice size,
    precision and potential exponent: a reused hierarchy needs no device allocation, only
    its new initial state and its step counter set back to 0."""

    def __init__(self):
        self.idle = collections.defaultdict(list)
        self.all = []

    @staticmethod
    def key(job: Job):
        return (job.n, job.prec, job.beta)

    def take(self, job: Job, stream):
        """A hierarchy for ``job`` on ``stream`` holding its initial state (queued there)."""
        import torch
        free = self.idle[self.key(job)]
        if free:
            h = free.pop()
            h.set_stream(stream)
        else:
            h = shamr.Hierarchy(job.n, float(job.n), 0.25, 0.1, 1.0, 2.0, job.beta, max_level=0, prec=job.prec,
                                stream=stream)
            h.set_layout(0, [(0, 0, 0, job.n - 1, job.n - 1, job.n - 1)])
            self.all.append(h)
        with torch.cuda.stream(stream):
            src = torch.from_numpy(np.ascontiguousarray(job.U0).reshape(-1)).pin_memory()
            job.staged = src.to("cuda", non_blocking=True)
        # the counter first: it decides which state slot holds U_n
        h.restart()
        h.write_device(0, job.staged)
        h.fill_ghosts(0)
        return h

    def give_back(self, job: Job):
        self.idle[self.key(job)].append(job.h)
        job.h = None

    def close(self):
        for h in self.all:
            h.close()
        self.all = []
        self.idle.clear()


def serve(jobs, budget_bytes: int, stream=None, keep_results=(), inflight: int = 4, log=None,
          poison=None, graph_steps: int = 16, pool=None):
    """Run ``jobs`` (sorted by arrival, seconds from start) under continuous batching.

    Jobs are admitted in arrival order while their arenas fit ``budget_bytes`` and set up
    on a stream of their own (a finished job's hierarchy of the same class reused when one
    is free), so the running batch never waits for an admission; a job joins the batch
    once its set-up has run.  All resident jobs of one precision advance together, one
    batched launch per kernel per step, recorded as a graph of ``graph_steps`` steps while
    every stepping job has that many steps left (single steps after that); a job alone in
    its precision steps on its own hierarchy instead, with a graph recorded once per pooled
    hierarchy.  A job that arrives while nothing is resident or being set up is set up
    on the batch stream itself and joins at once.  A change of members rewrites the batch tables in stream order
    (sh_batch_update), and a finished job is noticed from its step count and released once
    the stream has passed its last step, so neither drains the GPU.  ``keep_results``: job ids whose final state is copied out;
    ``poison``: optional callable(job) -> bool marking jobs whose state is set to NaN at
    admission (failure-isolation checks).  Returns the jobs and the wall time from the
    start to the last completion; each job gets t_admit (set-up queued), t_join (in the
    batch) and t_done (its last step seen complete)."""
    import torch
    stream = stream or torch.cuda.Stream()
    side = torch.cuda.Stream()
    own_pool = pool is None
    pool = pool or Pool()
    use_graphs = graph_steps > 1
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    queue = collections.deque()
    staging, resident, retiring = [], [], []
    used = 0
    batches, graphs, graveyard = {}, {}, []
    solo_graphs = {}
    members = {}
    dirty = set()
    events = collections.deque()
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    def retire_ready():
        nonlocal used
        for r in list(retiring):
            j, ev = r
            if ev.query():
                j.t_done = now()
                if j.out is not None:
                    j.result = j.out.cpu().numpy().reshape(j.U0.shape)
                    j.out = None
                pool.give_back(j)
                used -= j.nbytes
                retiring.remove(r)
        for g in list(graveyard):
            if g[1].query():
                g[0].close()
                graveyard.remove(g)

    while pending or queue or staging or resident or retiring:
        t = now()
        while pending and pending[0].arrival <= t:
            queue.append(pending.popleft())
        while queue and used + queue[0].nbytes <= budget_bytes:
            j = queue.popleft()
            j.out = None
            # with nothing resident the batch stream is idle: set the job up there, so it
            # joins without waiting for a side-stream event
            direct = not (resident or staging)
            j.h = pool.take(j, stream if direct else side)
            if poison is not None and poison(j):
                with torch.cuda.stream(stream if direct else side):
                    j.staged = torch.full((j.U0.size,), float("nan"), dtype=torch.float64, device="cuda")
                j.h.write_device(0, j.staged)
                j.h.fill_ghosts(0)
            j.t_admit = now()
            used += j.nbytes
            if direct:
                j.staged = None
                j.t_join = j.t_admit
                resident.append(j)
                dirty.add(j.prec)
                continue
            j.ready = torch.cuda.Event()
            j.ready.record(side)
            staging.append(j)
        if queue and not (staging or resident or retiring):
            raise RuntimeError(f"job {queue[0].jid} needs {queue[0].nbytes} bytes, more than the budget")
        for j in list(staging):
            if j.ready.query():
                j.h.set_stream(stream)
                j.staged = None
                j.t_join = now()
                staging.remove(j)
                resident.append(j)
                dirty.add(j.prec)
        retire_ready()
        if not resident:
            if pending or staging or retiring:
                wait = 0.0005 if (staging or retiring) else max(0.0, min(0.01, pending[0].arrival - now()))
                time.sleep(wait)
            continue
        for p in sorted(dirty):
            hs = [j.h for j in resident if j.prec == p]
            for key in [k for k in graphs if k[0] == p]:
                ev = torch.cuda.Event()
                ev.record(stream)
                graveyard.append((graphs.pop(key), ev))
            members[p] = hs
            if not hs:
                continue
            if p in batches:
                batches[p].update(hs)
            else:
                batches[p] = shamr.Batch(hs)
        dirty.clear()
        # a graph of graph_steps steps while every resident job has that many left, else
        # single steps (recording shorter graphs would cost more than it saves)
        left = min(j.steps - j.done_steps for j in resident)
        nstep = graph_steps if use_graphs and left >= graph_steps else 1
        for p, b in batches.items():
            hs = members.get(p)
            if not hs:
                continue
            if len(hs) == 1:
                # a job alone in its class steps on its own hierarchy, whose recorded
                # graph outlives the job (pooled hierarchies are reused)
                h = hs[0]
                if nstep > 1:
                    g = solo_graphs.get(id(h))
                    if g is None:
                        with h.capture() as c:
                            for _ in range(nstep):
                                h.advance(0)
                        g = solo_graphs[id(h)] = c.graph
                    g.launch()
                else:
                    h.advance(0)
            elif nstep > 1:
                g = graphs.get((p, nstep))
                if g is None:
                    g = graphs[(p, nstep)] = b.capture(nstep)
                g.launch()
            else:
                b.advance()
        ev = torch.cuda.Event()
        ev.record(stream)
        events.append(ev)
        while len(events) > inflight:
            events.popleft().synchronize()
        for j in list(resident):
            j.done_steps += nstep
            if j.done_steps == j.steps:
                if j.jid in keep_results:
                    j.out = j.h.read_device(0)
                done_ev = torch.cuda.Event()
                done_ev.record(stream)
                retiring.append((j, done_ev))
                resident.remove(j)
                dirty.add(j.prec)
        if log is not None and dirty:
            log(f"t={now():.2f}s resident {len(resident)}, staging {len(staging)}, queued {len(queue)}, "
                f"pending {len(pending)}")
    stream.synchronize()
    retire_ready()
    wall = max((j.t_done for j in jobs), default=now())
    for g in list(graphs.values()) + list(solo_graphs.values()):
        g.close()
    for g, _ in graveyard:
        g.close()
    for b in batches.values():
        b.close()
    if own_pool:
        pool.close()
    return jobs, wall


def serve_fifo(jobs, stream=None, keep_results=(), graph_steps: int = 16, pool=None):
    """The one-at-a-time server, run for real: jobs in arrival order, each set up (pooled
    hierarchies as in ``serve``), stepped alone to its end (graphs of ``graph_steps``
    steps, recorded once per hierarchy) and finished before the next starts.  Returns the
    jobs (t_admit = start of its set-up, t_done = its last step complete) and the wall
    time to the last completion."""
    import torch
    stream = stream or torch.cuda.Stream()
    own_pool = pool is None
    pool = pool or Pool()
    graphs = {}
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    for j in sorted(jobs, key=lambda j: j.arrival):
        wait = j.arrival - now()
        if wait > 0:
            time.sleep(wait)
        j.t_admit = now()
        j.h = pool.take(j, stream)
        j.t_join = j.t_admit
        key = id(j.h)
        full, rest = divmod(j.steps, graph_steps) if graph_steps > 1 else (0, j.steps)
        if full:
            if key not in graphs:
                with j.h.capture() as c:
                    for _ in range(graph_steps):
                        j.h.advance(0)
                graphs[key] = c.graph
            for _ in range(full):
                graphs[key].launch()
        for _ in range(rest):
            j.h.advance(0)
        j.done_steps = j.steps
        out = j.h.read_device(0) if j.jid in keep_results else None
        stream.synchronize()
        j.t_done = now()
        j.staged = None
        if out is not None:
            j.result = out.cpu().numpy().reshape(j.U0.shape)
        pool.give_back(j)
    wall = max((j.t_done for j in jobs), default=now())
    for g in graphs.values():
        g.close()
    if own_pool:
        pool.close()
    return jobs, wall


def solo_runtime(job: Job, stream=None, keep: bool = False):
    """Run one job alone (eager level steps); returns (seconds, final state or None)."""
    import torch
    stream = stream or torch.cuda.current_stream()
    h = make_hierarchy(job, stream)
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(job.steps):
        h.advance(0)
    stream.synchronize()
    dt = time.perf_counter() - t0
    res = h.read_dense(0) if keep else None
    h.close()
    return dt, res


def make_requests(njobs: int = 256, rate: float = 4.0, sizes=(32, 48, 64, 96, 128), steps=(200, 1000),
                  seed: int = 42, beta: int = 2):
    """Poisson arrivals; N uniform over ``sizes``; steps uniform in [lo, hi]; FP32/FP64 1:1."""
    from synth import random_state
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(njobs):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        st = int(rng.integers(steps[0], steps[1] + 1))
        prec = shamr.SH_F32 if rng.random() < 0.5 else shamr.SH_F64
        jobs.append(Job(jid=j, n=n, steps=st, prec=prec, seed=1000 + j, arrival=t, beta=beta))
    for j in jobs:
        j.U0 = random_state(j.n, float(j.n), j.seed)
        j.nbytes = arena_bytes(j)
    return jobs


def _reset(jobs, arrivals=None):
    for k, j in enumerate(jobs):
        j.h = None
        j.done_steps = 0
        j.t_admit = j.t_join = j.t_done = None
        j.result = None
        if arrivals is not None:
            j.arrival = arrivals[k]


def _report(jobs, wall):
    lat = np.array([j.t_done - j.arrival for j in jobs])
    work = sum(j.cell_stages for j in jobs)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "wall_s": wall, "cell_updates_per_s": work / wall}


def bench_serving(njobs: int = 256, budget_gb: float = 200.0, log=print, verify: int = 4,
                  saturated_rate: float = 32.0):
    """The ensemble-serving measurement: continuous batching against a one-at-a-time FIFO
    server, both run for real on the same jobs and arrival times (set-up included), at the
    nominal Poisson rate (4 jobs/s) and with the same jobs arriving ``saturated_rate``/4
    times faster.  The budget is in units of 1e9 bytes."""
    import torch
    from synth import random_state
    log(f"generating {njobs} requests")
    jobs = make_requests(njobs)
    budget = int(budget_gb * 1e9)
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(7)
    check = set(int(i) for i in rng.choice(njobs, size=min(verify, njobs), replace=False))
    log("warm-up: every kernel once per precision and size class")
    with torch.cuda.stream(stream):
        for n in (32, 48, 64, 96, 128):
            for p in (shamr.SH_F32, shamr.SH_F64):
                w = Job(jid=-1, n=n, steps=3, prec=p, seed=0, arrival=0.0, U0=random_state(n, float(n), 0))
                solo_runtime(w, stream)
    nominal_arrivals = [j.arrival for j in jobs]
    out = {}
    results = {}
    for label, scale in (("nominal", 1.0), ("saturated", 4.0 / saturated_rate)):
        arrivals = [a * scale for a in nominal_arrivals]
        _reset(jobs, arrivals)
        log(f"one at a time, {label} rate")
        _, wall = serve_fifo(jobs, stream=stream, keep_results=check)
        fifo = _report(jobs, wall)
        results[("fifo", label)] = {i: jobs[i].result for i in check}
        _reset(jobs, arrivals)
        log(f"continuous batching, {label} rate")
        _, wall = serve(jobs, budget, stream=stream, keep_results=check)
        batched = _report(jobs, wall)
        results[("batched", label)] = {i: jobs[i].result for i in check}
        out[label] = {"batched": batched, "one_at_a_time": fifo}
    same = all(np.array_equal(results[("fifo", "nominal")][i], results[(k, lab)][i], equal_nan=True)
               for i in check for k in ("fifo", "batched") for lab in ("nominal", "saturated"))
    work = sum(j.cell_stages for j in jobs)
    return {
        "metric": "p50/p99 ensemble-job latency and throughput, continuous batching vs one at a time",
        "unit": "s",
        "value": out["nominal"]["batched"]["p99_s"],
        "n_gpus": 1,
        "data": "synthetic",
        "higher_is_better": False,
        "config": {"workload": f"{njobs} single-level jobs, Poisson arrivals 4/s, N in {{32,48,64,96,128}}, "
                               "steps in [200, 1000], FP32/FP64 1:1, HBM budget 200 GB (1e9 bytes)", "seed": 42},
        **out["nominal"],
        "saturated": {"rate_per_s": saturated_rate, **out["saturated"]},
        "total_cell_stage_updates": work,
        "alone_vs_mix_bitwise": bool(same),
        "verified_jobs": sorted(check),
    }
