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
