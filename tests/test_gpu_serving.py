"""GPU tests of batched stepping and of the serving loop (continuous batching).

Every job's spike raster must be identical whether the job runs alone on the
plain path, alone in a batch, or in a mix of uneven jobs admitted at
different times (the multi-job kernels implement the same definitions; the
history is sorted when read).
"""
import sys

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def snn():
    from paper_1803_08833_amd import snn as S

    S.lib()
    import torch

    assert torch.cuda.is_available()
    return S


def mix(n, seed=9):
    r = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        g = int(r.choice([1, 2, 3, 4]))
        kind = W.GAUSS if i % 2 == 0 else W.EXP
        rng = float(r.uniform(1.0, 2.0) if kind == W.GAUSS else r.uniform(2.0, 6.0))
        jobs.append(dict(net=W.make(g, g, kind, rng, 600, 500 + i, ext_rate_hz=float(r.uniform(2.0, 3.0))),
                         steps=int(r.integers(60, 400))))
    return jobs


def mixed_schedules(n, seed=13):
    """Jobs the batched kernels treat differently: F32 records (binned),
    8-bit codes and more than 20 delay buckets (both delivered directly)."""
    r = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        g = int(r.choice([1, 2, 3]))
        over = dict(ext_rate_hz=float(r.uniform(2.0, 3.0)))
        if i % 3 == 1:
            over["record"] = W.REC_CODE8
        elif i % 3 == 2:
            over["d_max"] = 28
        jobs.append(dict(net=W.make(g, g, W.EXP, float(r.uniform(2.0, 5.0)), 500, 700 + i, **over),
                         steps=int(r.integers(80, 300))))
    return jobs


def alone(snn, job):
    with snn.Net(job["net"], hist_cap=1 << 22) as g:
        g.build_synapses()
        g.step(job["steps"])
        return g.read_spikes(), g.stats()


def test_batch_equals_alone(snn):
    jobs = mix(16)
    say("case: 16 uneven jobs in one batch vs each alone")
    ref = [alone(snn, j) for j in jobs]
    got = [None] * len(jobs)
    with snn.Batch(32 << 30, 1 << 20) as b:
        slot_job = {}
        for i, j in enumerate(jobs[:10]):
            s = b.admit(j["net"], j["steps"])
            assert s is not None
            slot_job[s] = i
        pending = list(range(10, len(jobs)))
        while slot_job or pending:
            b.step(37)
            for s in b.poll():
                i = slot_job.pop(s)
                st = b.job_stats(s)
                assert st["rec_events"] == ref[i][1]["rec_events"]
                assert st["ext_events"] == ref[i][1]["ext_events"]
                got[i] = b.read_spikes(s)
            while pending:   # late admissions join the running batch
                s = b.admit(jobs[pending[0]]["net"], jobs[pending[0]]["steps"])
                if s is None:
                    break
                slot_job[s] = pending.pop(0)
    for i, (r, _) in enumerate(ref):
        assert got[i] is not None
        assert len(r) > 0
        np.testing.assert_array_equal(got[i], r, err_msg=f"job {i}")


def test_single_job_batch_equals_alone(snn):
    job = mix(1, seed=3)[0]
    ref, _ = alone(snn, job)
    with snn.Batch(8 << 30, 1 << 20) as b:
        s = b.admit(job["net"], job["steps"])
        while not b.poll():
            b.step(64)
        np.testing.assert_array_equal(b.read_spikes(s), ref)


def test_admission_by_budget(snn):
    """A job that could never fit (footprint above the whole budget, or more
    neurons than the batch's capacity) is refused for good (SNN_E_INVAL); one
    that does not fit beside the running jobs is refused for now (None) and
    admitted once they have finished."""
    jobs = mix(3, seed=5)
    with snn.Batch(1 << 20, 1 << 20) as b:   # 1 MiB: nothing can ever fit
        with pytest.raises(snn.SNNError, match="budget"):
            b.admit(jobs[0]["net"], 50)
    with snn.Batch(6 << 30, 4096) as b:      # neuron capacity of four 1024-neuron blocks
        big = W.make(2, 2, W.EXP, 3.0, 300, 1)   # 4960 neurons: five blocks
        with pytest.raises(snn.SNNError, match="capacity"):
            b.admit(big, 50)
        small = W.make(1, 1, W.EXP, 3.0, 300, 2)   # 1240 neurons: two blocks
        s = b.admit(small, 20)
        assert s is not None
        s2 = b.admit(dict(small, seed=3), 20)      # two blocks more: still fits
        assert s2 is not None
        assert b.admit(dict(small, seed=4), 20) is None   # not beside the two running jobs
        used, n = b.usage()
        assert n == 2 and used > 0
        done = []
        while len(done) < 2:
            b.step(10)
            done += b.poll()
        b.read_spikes(s)
        b.read_spikes(s2)
        assert b.usage() == (0, 0)
        s3 = b.admit(dict(small, seed=4), 20)       # room again
        assert s3 is not None
        while not b.poll():
            b.step(10)
        b.read_spikes(s3)


def test_serving_loop_matches_plain(snn):
    from paper_1803_08833_amd import serve

    jobs = mix(20, seed=11)
    arrivals = serve.poisson_arrivals(len(jobs), rate_per_s=40.0, seed=2)
    say("case: served stream of 20 jobs, continuous batching vs one at a time")
    rb = serve.serve_batched(jobs, arrivals, hbm_budget=32 << 30, max_neurons=1 << 20, chunk_ms=25,
                             keep_spikes=True)
    rp = serve.serve_plain(jobs, arrivals, keep_spikes=True)
    for i in range(len(jobs)):
        np.testing.assert_array_equal(rb["rasters"][i], rp["rasters"][i], err_msg=f"job {i}")
    assert np.all(np.isfinite(rb["latency"])) and np.all(rb["latency"] > 0)
    np.testing.assert_array_equal(rb["events"], rp["events"])
    say("batched", serve.summary(rb, jobs))
    say("plain", serve.summary(rp, jobs))


def test_batch_mixes_binned_and_direct_jobs(snn):
    """Binned F32 jobs, 8-bit-code jobs and jobs with 28 delay buckets (direct
    delivery in the batch) share the batch: every raster equals the job run
    alone."""
    jobs = mixed_schedules(9)
    say("case: 9 jobs mixing binned and direct batch schedules")
    ref = [alone(snn, j) for j in jobs]
    got = {}
    with snn.Batch(16 << 30, 1 << 20) as b:
        slots = {b.admit(j["net"], j["steps"]): i for i, j in enumerate(jobs)}
        assert None not in slots
        while len(got) < len(jobs):
            b.step(41)
            for s in b.poll():
                i = slots[s]
                assert b.job_stats(s)["rec_events"] == ref[i][1]["rec_events"]
                got[i] = b.read_spikes(s)
    for i, (r, _) in enumerate(ref):
        assert len(r) > 0
        np.testing.assert_array_equal(got[i], r, err_msg=f"job {i}")
