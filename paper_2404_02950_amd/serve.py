"""Continuous-batching service for ensembles of independent single-level simulations.

Requests (lattice size N, step count, precision, seed, arrival time) arrive over time.
The server keeps every admitted job's state resident in HBM, admits queued jobs in
arrival order while their arenas fit the memory budget, and advances all resident jobs
together: one batched launch per kernel per step for each precision (sh_batch_advance),
so jobs that arrive while others run overlap on the device.  Finished jobs release
their memory at once, which lets waiting jobs in.  Each job's result is bit-identical
to running it alone.

``serve`` runs a request list against the wall clock and returns per-job timings;
``fifo_timeline`` gives the one-at-a-time baseline from measured solo run times.
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
    t_done: float = None
    result: np.ndarray = field(repr=False, default=None)

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


def serve(jobs, budget_bytes: int, stream=None, keep_results=(), inflight: int = 4, log=None,
          poison=None, graph_steps: int = 16):
    """Run ``jobs`` (sorted by arrival, seconds from start) under continuous batching.

    ``keep_results``: job ids whose final state is read back (in ``Job.result``).
    ``poison``: optional callable(job) -> bool marking jobs whose state is overwritten
    with NaN after admission (failure-isolation checks).  ``graph_steps``: up to this many
    batch steps (a power of two, never past the first job to finish) are recorded once as
    a HIP graph and replayed with one launch, which takes the per-step host work out of
    the loop (1: no graphs; graphs need a stream other than the default one).  Returns the
    jobs and the wall time from the first arrival to the last completion.
    """
    import torch
    stream = stream or torch.cuda.current_stream()
    use_graphs = graph_steps > 1 and stream.cuda_stream != 0
    graphs = {}
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    queue = collections.deque()
    resident = []
    used = 0
    batches = {}
    dirty = True
    events = collections.deque()
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    while pending or queue or resident:
        t = now()
        while pending and pending[0].arrival <= t:
            queue.append(pending.popleft())
        while queue and used + queue[0].nbytes <= budget_bytes:
            j = queue.popleft()
            j.h = make_hierarchy(j, stream)
            if poison is not None and poison(j):
                bad = np.full_like(j.U0, np.nan)
                j.h.write_dense(0, bad)
                j.h.fill_ghosts(0)
            j.t_admit = now()
            used += j.nbytes
            resident.append(j)
            dirty = True
        if queue and not resident:
            raise RuntimeError(f"job {queue[0].jid} needs {queue[0].nbytes} bytes, more than the budget")
        if not resident:
            if pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival - now())))
            continue
        if dirty:
            stream.synchronize()  # recorded steps may still run on the old batch tables
            for g in graphs.values():
                g.close()
            graphs = {}
            for b in batches.values():
                b.close()
            groups = collections.defaultdict(list)
            for j in resident:
                groups[j.prec].append(j.h)
            batches = {p: shamr.Batch(hs) for p, hs in groups.items()}
            dirty = False
        nstep = 1
        if use_graphs:
            left = min(j.steps - j.done_steps for j in resident)
            while nstep * 2 <= min(graph_steps, left):
                nstep *= 2
        if nstep > 1:
            for p, b in batches.items():
                g = graphs.get((p, nstep))
                if g is None:
                    g = graphs[(p, nstep)] = b.capture(nstep)
                g.launch()
        else:
            for b in batches.values():
                b.advance()
        ev = torch.cuda.Event()
        ev.record(stream)
        events.append(ev)
        if len(events) > inflight:
            events.popleft().synchronize()
        finished = []
        for j in resident:
            j.done_steps += nstep
            if j.done_steps == j.steps:
                finished.append(j)
        if finished:
            stream.synchronize()
            events.clear()
            t = now()
            for j in finished:
                j.t_done = t
                if j.jid in keep_results:
                    j.result = j.h.read_dense(0)
                resident.remove(j)
                used -= j.nbytes
            for g in graphs.values():
                g.close()
            graphs = {}
            for b in batches.values():
                b.close()
            batches = {}
            for j in finished:
                j.h.close()
                j.h = None
            dirty = True
            if log is not None:
                log(f"t={t:.2f}s finished {[j.jid for j in finished]}, resident {len(resident)}, "
                    f"queued {len(queue)}, pending {len(pending)}")
    stream.synchronize()
    for g in graphs.values():
        g.close()
    for b in batches.values():
        b.close()
    return jobs, now()


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


def fifo_timeline(jobs, solo):
    """One-at-a-time FIFO server: start = max(arrival, previous finish)."""
    t = 0.0
    lat = {}
    for j in sorted(jobs, key=lambda j: j.arrival):
        start = max(j.arrival, t)
        t = start + solo[j.jid]
        lat[j.jid] = t - j.arrival
    return lat, t


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
        j.t_admit = j.t_done = None
        j.result = None
        if arrivals is not None:
            j.arrival = arrivals[k]


def _latency_report(jobs, solo, wall, stream, budget_gb, check):
    lat_fifo, fifo_end = fifo_timeline(jobs, solo)
    lat = np.array([j.t_done - j.arrival for j in jobs])
    lf = np.array([lat_fifo[j.jid] for j in jobs])
    work = sum(j.cell_stages for j in jobs)
    return {
        "batched": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                    "wall_s": wall, "cell_updates_per_s": work / wall},
        "one_at_a_time": {"p50_s": float(np.percentile(lf, 50)), "p99_s": float(np.percentile(lf, 99)),
                          "wall_s": fifo_end, "cell_updates_per_s": work / fifo_end},
    }


def bench_serving(njobs: int = 256, budget_gb: float = 200.0, log=print, verify: int = 4,
                  saturated_rate: float = 32.0):
    """The ensemble-serving measurement: continuous batching vs one-at-a-time FIFO, at the
    nominal Poisson rate (4 jobs/s) and with the same jobs arriving ``saturated_rate``/4
    times faster, where a one-at-a-time server cannot keep up."""
    import torch
    log(f"generating {njobs} requests")
    jobs = make_requests(njobs)
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(7)
    check = set(int(i) for i in rng.choice(njobs, size=min(verify, njobs), replace=False))
    log("solo run times (one-at-a-time baseline)")
    solo, solo_res = {}, {}
    with torch.cuda.stream(stream):
        # warm up the kernels once per precision and size class
        for n in (32, 48, 64, 96, 128):
            for p in (shamr.SH_F32, shamr.SH_F64):
                from synth import random_state
                w = Job(jid=-1, n=n, steps=3, prec=p, seed=0, arrival=0.0, U0=random_state(n, float(n), 0))
                solo_runtime(w, stream)
        for j in jobs:
            solo[j.jid], res = solo_runtime(j, stream, keep=j.jid in check)
            if res is not None:
                solo_res[j.jid] = res
        log("continuous batching, nominal rate")
        _, wall = serve(jobs, int(budget_gb * 2**30), stream=stream, keep_results=check)
        nominal = _latency_report(jobs, solo, wall, stream, budget_gb, check)
        same = all(np.array_equal(solo_res[i], jobs[i].result, equal_nan=True) for i in check)
        scale = 4.0 / saturated_rate
        nominal_arrivals = [j.arrival for j in jobs]
        _reset(jobs, [a * scale for a in nominal_arrivals])
        log(f"continuous batching, {saturated_rate:g} jobs/s")
        _, wall = serve(jobs, int(budget_gb * 2**30), stream=stream, keep_results=check)
        sat = _latency_report(jobs, solo, wall, stream, budget_gb, check)
        same = same and all(np.array_equal(solo_res[i], jobs[i].result, equal_nan=True) for i in check)
        _reset(jobs, [a * scale for a in nominal_arrivals])
        log(f"continuous batching, {saturated_rate:g} jobs/s, every step launched from the host")
        _, wall = serve(jobs, int(budget_gb * 2**30), stream=stream, keep_results=check, graph_steps=1)
        sat_nograph = _latency_report(jobs, solo, wall, stream, budget_gb, check)["batched"]
        same = same and all(np.array_equal(solo_res[i], jobs[i].result, equal_nan=True) for i in check)
    work = sum(j.cell_stages for j in jobs)
    return {
        "metric": "p50/p99 ensemble-job latency and throughput, continuous batching vs one at a time",
        "unit": "s",
        "value": nominal["batched"]["p99_s"],
        "n_gpus": 1,
        "data": "synthetic",
        "higher_is_better": False,
        "config": {"workload": f"{njobs} single-level jobs, Poisson arrivals 4/s, N in {{32,48,64,96,128}}, "
                               "steps in [200, 1000], FP32/FP64 1:1, HBM budget 200 GB", "seed": 42},
        **nominal,
        "gpu_busy_one_at_a_time_s": float(sum(solo.values())),
        "saturated": {"rate_per_s": saturated_rate, **sat, "batched_without_graphs": sat_nograph},
        "total_cell_stage_updates": work,
        "alone_vs_mix_bitwise": bool(same),
        "verified_jobs": sorted(check),
    }
