"""Host-side pieces of the serving benchmark: the seeded job stream, the
arrival process and the latency summary (no GPU)."""
import numpy as np
import pytest

from paper_1803_08833_amd import serve
from paper_1803_08833_amd import workloads as W


def test_serving_stream_composition():
    jobs = W.serving_stream(512, seed=4)
    assert len(jobs) == 512
    kinds = [j["net"]["kernel"] for j in jobs]
    assert kinds.count(W.GAUSS) == 256 and kinds.count(W.EXP) == 256
    grids = {(j["net"]["gx"], j["net"]["gy"]) for j in jobs}
    assert grids <= {(g, g) for g in (2, 4, 8, 12, 16)} and len(grids) == 5
    for j in jobs:
        assert 500 <= j["steps"] <= 5000
        lo, hi = (1.0, 2.0) if j["net"]["kernel"] == W.GAUSS else (2.0, 6.0)
        assert lo <= j["net"]["range"] <= hi
    seeds = [j["net"]["seed"] for j in jobs]
    assert seeds == list(range(1_000_000, 1_000_512))
    # same seed, same stream; different seed, different order
    assert W.serving_stream(512, seed=4) == jobs
    assert [j["net"]["kernel"] for j in W.serving_stream(512, seed=5)] != kinds


def test_poisson_arrivals_rate_and_order():
    a = serve.poisson_arrivals(20000, rate_per_s=8.0, seed=3)
    assert np.all(np.diff(a) > 0)
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(gaps.mean() - 1 / 8.0) < 0.01 * (1 / 8.0) * 3
    # exponential gaps: coefficient of variation ~ 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_summary_percentiles_and_rates():
    jobs = [dict(net={}, steps=1000), dict(net={}, steps=3000)]
    res = serve.Result(latency=np.array([0.5, 1.5]), events=np.array([10, 30]), wall=2.0)
    s = serve.summary(res, jobs)
    assert s["jobs"] == 2 and s["jobs_per_s"] == 1.0
    assert s["p50_s"] == 1.0
    assert abs(s["p99_s"] - (0.5 + 0.99 * 1.0)) < 1e-12
    assert s["events_per_s"] == 20.0
    assert s["sim_s_per_wall_s"] == 2.0


class _FakeBatch:
    """Host stand-in for snn.Batch with the library's admission rules: a job
    whose neurons exceed the batch's capacity is refused for good (SNNError,
    SNN_E_INVAL); one that does not fit beside the running jobs gets None."""

    def __init__(self, cap_neurons, *a, **k):
        self.cap = cap_neurons
        self.used = 0
        self.running = {}     # slot -> [neurons, steps left]
        self.next_slot = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        pass

    def admit(self, net, steps):
        if net["n"] > self.cap:
            from paper_1803_08833_amd import snn
            raise snn.SNNError(-1, "job larger than the batch's neuron capacity")
        if self.used + net["n"] > self.cap:
            return None
        s = self.next_slot
        self.next_slot += 1
        self.running[s] = [net["n"], steps]
        self.used += net["n"]
        return s

    def step(self, chunk):
        for v in self.running.values():
            v[1] -= chunk

    def poll(self):
        return [s for s, v in self.running.items() if v[1] <= 0]

    def job_stats(self, slot):
        return {"rec_events": 1}

    def read_spikes(self, slot):
        n, _ = self.running.pop(slot)
        self.used -= n
        return np.zeros((0, 2), dtype=np.uint32)


def test_never_fitting_job_fails_and_does_not_block(monkeypatch):
    """A job that can never be admitted is recorded as failed and the jobs
    queued behind it are still served (it used to stay at the head of the
    queue and stall the loop)."""
    from paper_1803_08833_amd import snn

    monkeypatch.setattr(snn, "Batch", lambda budget, neurons, stream=None: _FakeBatch(neurons))
    monkeypatch.setattr(snn, "current_stream_handle", lambda: None)
    jobs = [dict(net=dict(n=n), steps=s) for n, s in ((10, 100), (500, 100), (60, 200), (40, 50), (30, 50))]
    res = serve.serve_batched(jobs, np.zeros(len(jobs)), hbm_budget=0, max_neurons=100, chunk_ms=50)
    assert [j for j, _ in res["failed"]] == [1]
    assert np.isnan(res["latency"][1])
    assert not np.isnan(np.delete(res["latency"], 1)).any()
    s = serve.summary(res, jobs)
    assert s["failed"] == 1
    assert s["sim_s_per_wall_s"] == pytest.approx((100 + 200 + 50 + 50) * 1e-3 / res["wall"])
