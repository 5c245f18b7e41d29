"""GPU test of the schedule autotuner: it times every candidate on the same
(reset) workload, applies and caches the fastest, and the tuned network gives
the same raster as the untuned one."""
import os

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_picks_applies_and_caches(tmp_path):
    from paper_1803_08833_amd import autotune, snn

    net = W.workload("grid4_gauss", seed=44)["net"]
    with snn.Net(net) as ref:
        ref.build_synapses()
        ref.step(300)
        want = ref.read_spikes()
    cache = str(tmp_path / "tune.json")
    with snn.Net(net) as g:
        g.build_synapses()
        res = autotune.tune(g, warmup=20, steps=60, cache=cache)
        assert len(res["trials"]) >= 3
        assert res["ms_per_step"] == min(t["ms_per_step"] for t in res["trials"])
        assert g.stats()["t"] == 0
        g.step(300)
        np.testing.assert_array_equal(g.read_spikes(), want)
    assert os.path.exists(cache)
    with snn.Net(net) as h:
        h.build_synapses()
        assert autotune.load(h, cache)
        h.step(300)
        np.testing.assert_array_equal(h.read_spikes(), want)


def test_batch_autotune_and_schedules_give_same_rasters(tmp_path):
    """The batch autotuner serves the same closed loop under each candidate
    schedule and keeps the fastest; rasters under the most different
    schedules equal the one-job-at-a-time server's."""
    from paper_1803_08833_amd import autotune, serve, snn

    jobs = W.serving_stream(8, seed=7)
    for j in jobs:
        j["steps"] = min(j["steps"], 400)
    cands = [dict(chunk_ms=50, options={snn.OPT_SCATTER_BLOCKS: 256, snn.OPT_DELIVER_MODE: 1}),
             dict(chunk_ms=25, options={snn.OPT_SCATTER_BLOCKS: 512, snn.OPT_DELIVER_MODE: 1,
                                        snn.OPT_BIN_THRESHOLD_PPM: 5000}),
             dict(chunk_ms=100, options={snn.OPT_DELIVER_MODE: 0})]
    res = autotune.tune_batch(jobs, 32 << 30, 4 << 20, candidates=cands, finalists=2,
                              cache=str(tmp_path / "b.json"))
    assert res["schedule"] in [dict(chunk_ms=c["chunk_ms"], options={str(k): v for k, v in c["options"].items()})
                               for c in cands]
    assert all(len(t["jobs_per_s"]) >= 1 for t in res["trials"])
    z = np.zeros(len(jobs))
    want = serve.serve_plain(jobs, z, keep_spikes=True)["rasters"]
    for c in cands[1:] + [res["schedule"]]:
        got = serve.serve_batched(jobs, z, 32 << 30, 4 << 20, keep_spikes=True, schedule=c)
        assert not got["failed"]
        for i in range(len(jobs)):
            np.testing.assert_array_equal(got["rasters"][i], want[i], err_msg=f"job {i} under {c}")


def test_batch_set_option_rejects_bad_values():
    from paper_1803_08833_amd import snn

    with snn.Batch(1 << 30, 1 << 20) as b:
        for opt, v in ((snn.OPT_SCATTER_BLOCKS, 8), (snn.OPT_SCATTER_BLOCKS, 5000), (snn.OPT_DELIVER_MODE, 2),
                       (snn.OPT_BIN_THRESHOLD_PPM, -1), (snn.OPT_GRAPH_CHUNK, 10)):
            with pytest.raises(snn.SNNError):
                b.set_option(opt, v)
        b.set_option(snn.OPT_SCATTER_BLOCKS, 512)
        b.set_option(snn.OPT_DELIVER_MODE, 0)
        b.set_option(snn.OPT_BIN_THRESHOLD_PPM, 1000)
