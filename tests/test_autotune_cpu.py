"""CPU checks of the autotuner's host logic (no device work)."""
from paper_1803_08833_amd import workloads as W


def test_key_ignores_seed_and_separates_workloads():
    from paper_1803_08833_amd import autotune

    a = W.workload("grid24_exp")["net"]
    assert autotune.key(a) == autotune.key(dict(a, seed=99))
    assert autotune.key(a) != autotune.key(W.workload("grid24_gauss")["net"])


def test_candidates_cover_both_schedules():
    from paper_1803_08833_amd import autotune, snn

    c = autotune.candidates(dict(bin_threshold=1000, binned_ok=1))
    modes = {o[snn.OPT_DELIVER_MODE] for o in c}
    assert modes == {0, 1}
    assert all(o.get(snn.OPT_BIN_THRESHOLD, 1) >= 0 for o in c)
    assert {o[snn.OPT_DELIVER_MODE] for o in autotune.candidates(dict(bin_threshold=0, binned_ok=0))} == {0}
    assert {o[snn.OPT_DELIVER_MODE] for o in autotune.candidates(dict(bin_threshold=9, binned_ok=2))} == {0, 2}


def test_batch_candidates_default_first_and_distinct():
    from paper_1803_08833_amd import autotune, snn

    c = autotune.batch_candidates()
    assert c[0] == dict(chunk_ms=50, options={snn.OPT_SCATTER_BLOCKS: 256, snn.OPT_DELIVER_MODE: 1,
                                              snn.OPT_BIN_THRESHOLD_PPM: 0})
    assert len({repr(x) for x in c}) == len(c)
    assert {x["chunk_ms"] for x in c} == {25, 50, 100}
    assert {x["options"][snn.OPT_DELIVER_MODE] for x in c} == {0, 1}


def test_batch_key_ignores_seeds_drives_and_durations():
    from paper_1803_08833_amd import autotune

    jobs = W.serving_stream(8, seed=4)
    other = [dict(net=dict(j["net"], seed=j["net"]["seed"] + 1, ext_rate_hz=9.0), steps=j["steps"] + 5)
             for j in jobs]
    assert autotune.batch_key(jobs) == autotune.batch_key(other)
    assert autotune.batch_key(jobs) == autotune.batch_key(jobs[::-1])
    assert autotune.batch_key(jobs) != autotune.batch_key(jobs[:-1])


def test_tune_batch_keeps_fastest_finalist_and_caches(tmp_path, monkeypatch):
    """The tuner's bookkeeping with a stand-in server whose wall time depends
    on the schedule: every candidate is tried, the finalists twice, the one
    with the best mean wins and is cached under the mix's key."""
    import numpy as np

    from paper_1803_08833_amd import autotune, serve

    wall = {25: 3.0, 50: 2.0, 100: 1.0}
    calls = []

    def fake(jobs, arrivals, hbm_budget, max_neurons, schedule=None, **kw):
        calls.append(schedule)
        w = wall[schedule["chunk_ms"]] + 0.01 * schedule["options"][autotune.snn.OPT_DELIVER_MODE]
        return serve.Result(latency=np.ones(len(jobs)), events=np.zeros(len(jobs), np.int64), wall=w,
                            rasters=[None] * len(jobs), failed=[])

    monkeypatch.setattr(serve, "serve_batched", fake)
    jobs = W.serving_stream(4, seed=1)
    cache = str(tmp_path / "t.json")
    res = autotune.tune_batch(jobs, 1 << 30, 1 << 20, finalists=2, cache=cache)
    n = len(autotune.batch_candidates())
    assert len(calls) == n + 2
    assert res["schedule"]["chunk_ms"] == 100
    assert res["schedule"]["options"][str(autotune.snn.OPT_DELIVER_MODE)] == 0
    assert len(res["trials"]) == n
    assert autotune.load_batch(jobs, cache) == res["schedule"]
    assert autotune.load_batch(jobs[:2], cache) is None
