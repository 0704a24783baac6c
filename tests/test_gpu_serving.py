"""Batched stepping across independent simulations and the continuous-batching server.

Each job's result must be the same bit for bit alone and in the mix (the kernels are
gather-only per box and every job carries its own step counter and time), admission
must respect the memory budget, and a job whose state is all NaN must not disturb the
others."""
import numpy as np
import pytest

from oracle.level import run_single_level
from synth import random_state

pytestmark = pytest.mark.gpu

shamr = pytest.importorskip("paper_2404_02950_amd.shamr")
from paper_2404_02950_amd import serve  # noqa: E402
from gpu_util import assert_bitwise  # noqa: E402


def _job(jid, n, steps, prec, arrival=0.0, beta=0):
    j = serve.Job(jid=jid, n=n, steps=steps, prec=prec, seed=100 + jid, arrival=arrival, beta=beta)
    j.U0 = random_state(n, float(n), j.seed)
    j.nbytes = serve.arena_bytes(j)
    return j


def test_batch_step_equals_solo_and_oracle():
    import torch
    stream = torch.cuda.Stream()
    jobs = [_job(0, 32, 7, shamr.SH_F64), _job(1, 48, 7, shamr.SH_F64), _job(2, 64, 7, shamr.SH_F64),
            _job(3, 40, 7, shamr.SH_F64)]
    hs = [serve.make_hierarchy(j, stream) for j in jobs]
    b = shamr.Batch(hs)
    for _ in range(7):
        b.advance()
    b.close()
    for j, h in zip(jobs, hs):
        _, solo = serve.solo_runtime(j, stream, keep=True)
        got = h.read_dense(0)
        assert_bitwise(got, solo, f"job {j.jid} batched vs alone")
        assert h.level_info(0)["k"] == 7
        h.close()
    ref = run_single_level(jobs[1].U0, 7, 0.1, 0.25, 1.0, beta=0)
    assert_bitwise(serve.solo_runtime(jobs[1], stream, keep=True)[1], ref, "48^3 job vs oracle")


def test_server_budget_admission_and_alone_vs_mix():
    import torch
    stream = torch.cuda.Stream()
    specs = [(32, 30, shamr.SH_F64), (64, 12, shamr.SH_F32), (48, 20, shamr.SH_F64), (32, 25, shamr.SH_F32),
             (64, 9, shamr.SH_F64), (48, 14, shamr.SH_F32)]
    jobs = [_job(i, n, st, p, arrival=0.01 * i) for i, (n, st, p) in enumerate(specs)]
    budget = max(j.nbytes for j in jobs) * 2 + 1      # at most two of the larger jobs at once
    done, wall = serve.serve(jobs, budget, stream=stream, keep_results={j.jid for j in jobs})
    assert all(j.t_done is not None for j in done)
    # admission in arrival order, never more resident bytes than the budget
    events = sorted([(j.t_admit, j.nbytes) for j in done] + [(j.t_done, -j.nbytes) for j in done])
    used = 0
    for _, d in events:
        used += d
        assert used <= budget
    assert [j.jid for j in sorted(done, key=lambda j: j.t_admit)] == list(range(len(jobs)))
    for j in done:
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(j.result, solo, f"job {j.jid} in the mix vs alone")


def test_nan_job_is_isolated():
    import torch
    stream = torch.cuda.Stream()
    jobs = [_job(i, n, 10, shamr.SH_F64, arrival=0.0) for i, n in enumerate((32, 48, 32, 64))]
    done, _ = serve.serve(jobs, 1 << 40, stream=stream, keep_results={0, 1, 2, 3}, poison=lambda j: j.jid == 2)
    assert np.all(np.isnan(done[2].result))
    for j in done:
        if j.jid == 2:
            continue
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(j.result, solo, f"job {j.jid} next to a NaN job")


def test_batch_update_keeps_every_job_exact():
    # members change between steps (sh_batch_update rewrites the tables in stream order):
    # every job still ends bit for bit where it would alone
    import torch
    stream = torch.cuda.Stream()
    jobs = [_job(i, n, 9, shamr.SH_F64) for i, n in enumerate((32, 48, 64, 32))]
    hs = [serve.make_hierarchy(j, stream) for j in jobs]
    b = shamr.Batch(hs[:2])
    for _ in range(3):
        b.advance()
    b.update(hs)                       # two more join
    for _ in range(3):
        b.advance()
    b.update([hs[1], hs[2], hs[3]])    # the first leaves
    for _ in range(3):
        b.advance()
    b.update([hs[2], hs[3]])
    for _ in range(3):
        b.advance()
    b.close()
    steps = {0: 6, 1: 9, 2: 9, 3: 9}
    for j, h in zip(jobs, hs):
        j.steps = steps[j.jid]
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(h.read_dense(0), solo, f"job {j.jid}")
        assert h.level_info(0)["k"] == steps[j.jid]
        h.close()


def test_pooled_hierarchies_and_the_one_at_a_time_server():
    # one class of jobs under a budget of one job: every job after the first reuses the
    # previous job's hierarchy (new state written on the device, counter set back to 0);
    # the batched and the one-at-a-time servers give every job its solo result
    import torch
    stream = torch.cuda.Stream()
    jobs = [_job(i, 48, 5 + 3 * i, shamr.SH_F32, arrival=0.002 * i) for i in range(5)]
    budget = jobs[0].nbytes
    keep = {j.jid for j in jobs}
    pool = serve.Pool()
    done, _ = serve.serve(jobs, budget, stream=stream, keep_results=keep, pool=pool)
    assert len(pool.all) == 1, "one hierarchy served every job"
    batched = {j.jid: j.result for j in done}
    serve._reset(jobs)
    done, _ = serve.serve_fifo(jobs, stream=stream, keep_results=keep, graph_steps=4)
    for j in done:
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(batched[j.jid], solo, f"job {j.jid} batched")
        assert_bitwise(j.result, solo, f"job {j.jid} one at a time")
        assert j.t_done >= j.t_admit >= j.arrival
    pool.close()




def test_a_job_arriving_to_an_idle_server_is_set_up_on_the_batch_stream():
    # nothing resident: the job is set up where it will step and joins at once; later
    # arrivals that find it running go through the side stream; all results are solo
    import torch
    stream = torch.cuda.Stream()
    jobs = [_job(0, 64, 40, shamr.SH_F64, arrival=0.0), _job(1, 32, 12, shamr.SH_F32, arrival=0.0),
            _job(2, 48, 20, shamr.SH_F64, arrival=0.0)]
    done, _ = serve.serve(jobs, 1 << 40, stream=stream, keep_results={0, 1, 2})
    by = {j.jid: j for j in done}
    assert by[0].t_join == by[0].t_admit
    for j in done:
        _, solo = serve.solo_runtime(j, stream, keep=True)
        assert_bitwise(j.result, solo, f"job {j.jid}")
