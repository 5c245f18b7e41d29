"""Batched multi-job stepping against the FP64 oracle, at the job sizes of
the served workload (grids up to 16x16 modules, 1100 synapses per neuron,
Gaussian and exponential laws, 8-byte and 8-bit-code records), all jobs in one
batch so that the batched kernels' bin windows span several jobs.

* One-step jobs: after the job's only step, every neuron's state, the spike
  set and the external event count equal the oracle's step 0, and the charge
  queued for sampled targets equals the oracle's column sums of the GPU's
  spike set.
* Longer jobs (33-70 steps, through the start-up transient, binned and direct
  steps): after the job's last step the charge in flight for sampled targets
  equals the oracle's column sums over the job's own spike sets of the last
  d_max steps, and the raster is the one the job gives stepped alone.
"""
import sys

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W
from parity_helpers import compare_state, pending_charge, ring_pending

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


# (grid, law, range, record, steps); seeds 2,000,000 + index
JOBS = [
    (16, W.EXP, 4.0, W.REC_F32, 1),
    (12, W.GAUSS, 1.5, W.REC_CODE8, 1),
    (16, W.GAUSS, 1.0, W.REC_F32, 45),
    (12, W.EXP, 3.0, W.REC_F32, 60),
    (16, W.EXP, 6.0, W.REC_CODE8, 33),
    (12, W.GAUSS, 2.0, W.REC_CODE8, 50),
    (8, W.EXP, 2.0, W.REC_F32, 70),
    (4, W.GAUSS, 1.2, W.REC_F32, 64),
    (2, W.EXP, 5.0, W.REC_F32, 40),
]


def _jobs():
    out = []
    for i, (g, law, rng, rec, steps) in enumerate(JOBS):
        net = W.make(g, g, law, rng, 1100, 2_000_000 + i, record=rec, ext_rate_hz=2.05)
        out.append(dict(net=net, steps=steps))
    return out


@pytest.fixture(scope="module")
def batch_run(snn):
    """Run every job in one batch; keep each finished job's state, ring and
    raster."""
    jobs = _jobs()
    n_all = sum(W.n_neurons(j["net"]) for j in jobs)
    say(f"case: {len(jobs)} jobs (grids up to 16x16, {n_all} neurons) in one batch")
    res = {}
    with snn.Batch(96 << 30, n_all + 4096) as b:
        slot_job = {}
        for i, j in enumerate(jobs):
            s = b.admit(j["net"], j["steps"])
            assert s is not None, f"job {i} not admitted"
            slot_job[s] = i
        while slot_job:
            b.step(7)
            for s in b.poll():
                i = slot_job.pop(s)
                V, Wf, R, ring = b.read_state(s)
                st = b.job_stats(s)
                res[i] = dict(V=V, W=Wf, R=R, ring=ring, stats=st, raster=b.read_spikes(s))
    return jobs, res


def test_one_step_jobs_match_oracle_step0(snn, oracle_mod, batch_run):
    jobs, res = batch_run
    for i, j in enumerate(jobs):
        if j["steps"] != 1:
            continue
        net = j["net"]
        say(f"job {i}: {net['gx']}x{net['gy']} step 0 against the oracle")
        o = oracle_mod.Net(net)
        o.step(1)
        Vo, Wo, Ro = o.state()
        s0 = o.spikes()[:, 1]
        r = res[i]
        gsp = r["raster"][:, 1]
        assert np.all(r["raster"][:, 0] == 0)
        diff = np.setxor1d(gsp, s0)          # fp32 and fp64 within rounding of V_th
        assert diff.size <= 2
        ok = np.setdiff1d(np.arange(W.n_neurons(net)), diff)
        compare_state(net, (r["V"][ok], r["W"][ok], r["R"][ok]), (Vo[ok], Wo[ok], Ro[ok]), 0)
        assert r["stats"]["ext_events"] == o.stats()["ext_events"]
        assert r["stats"]["spikes"] == gsp.size
        rng = np.random.default_rng(100 + i)
        pres = np.sort(gsp).astype(np.uint32)
        for t in rng.integers(0, W.n_neurons(net), 12):
            want = oracle_mod.col_input(net, int(t), pres)
            got = r["ring"][net["d_min"]:net["d_max"] + 1, t].astype(np.int64)
            np.testing.assert_array_equal(got, want, err_msg=f"job {i} target {t}")


def test_longer_jobs_in_flight_charge(snn, oracle_mod, batch_run):
    jobs, res = batch_run
    for i, j in enumerate(jobs):
        if j["steps"] == 1:
            continue
        net, T = j["net"], j["steps"]
        r = res[i]
        raster = r["raster"]
        counts = np.bincount(raster[:, 0].astype(np.int64), minlength=T)
        assert counts.size == T and r["stats"]["t"] == T
        say(f"job {i}: {net['gx']}x{net['gy']} {T} steps, spikes per step max {counts.max()}, "
            f"recent {counts[-net['d_max']:].sum()}")
        N = W.n_neurons(net)
        rng = np.random.default_rng(200 + i)
        for t in list(rng.integers(0, N, 10)) + [0, N - 1]:
            want = pending_charge(oracle_mod, net, raster, T, int(t))
            np.testing.assert_array_equal(ring_pending(r["ring"], net, T, int(t)), want,
                                          err_msg=f"job {i} target {t}")


def test_batched_rasters_equal_alone(snn, batch_run):
    jobs, res = batch_run
    for i in (2, 4, 6):
        j = jobs[i]
        with snn.Net(j["net"], hist_cap=1 << 22) as g:
            g.build_synapses()
            g.step(j["steps"])
            np.testing.assert_array_equal(res[i]["raster"], g.read_spikes(), err_msg=f"job {i}")
            np.testing.assert_array_equal(res[i]["ring"], g.read_ring(), err_msg=f"job {i}")
