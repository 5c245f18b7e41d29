"""The allocation-free lock-step call (snn_step_forced_noalloc) against the
ordinary one (snn_step_forced), through the C ABI: twin networks fed the same
forced spike sets give bit-identical state, delay ring, spike history and
counters after every call, on two calls in a row where the second has the
smaller input (a larger network with many forced spikes, then a smaller one
with few), and over a longer lock-step run; sizes beyond the static array's
maximum are refused before any device work."""
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


def _same(a, b):
    for x, y in zip(a.read_state(), b.read_state()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.read_ring(), b.read_ring())
    np.testing.assert_array_equal(a.read_spikes(), b.read_spikes())
    sa, sb = a.stats(), b.stats()
    for k in ("t", "spikes", "rec_events", "ext_events", "disagree"):
        assert sa[k] == sb[k], k


def test_two_calls_second_smaller(snn):
    big = W.make(4, 2, W.EXP, 3.0, 400, 61)       # 9,920 neurons
    small = W.make(2, 1, W.GAUSS, 1.0, 300, 62, n_exc=400, n_inh=100)   # 1,000 neurons
    say("case: no-alloc lock-step, large call then smaller call")
    rng = np.random.default_rng(3)
    with snn.Net(big) as a, snn.Net(big) as b, snn.Net(small) as c, snn.Net(small) as d:
        for g in (a, b, c, d):
            g.build_synapses()
        ids_big = np.sort(rng.choice(a.N, 3000, replace=False)).astype(np.uint32)
        a.step_forced(ids_big)
        b.step_forced_noalloc(ids_big)
        _same(a, b)
        ids_small = np.array([0, 5, 999, 500], dtype=np.uint32)   # unordered, fewer ids
        c.step_forced(ids_small)
        d.step_forced_noalloc(ids_small)
        _same(c, d)
        # the big network's flags from the first call must not leak into a
        # second call on it with fewer ids
        a.step_forced(ids_big[:7])
        b.step_forced_noalloc(ids_big[:7])
        _same(a, b)
        # an empty forced set
        c.step_forced([])
        d.step_forced_noalloc([])
        _same(c, d)


def test_lockstep_run_matches(snn, oracle_mod):
    net = W.make(2, 2, W.GAUSS, 1.0, 500, 63, n_exc=400, n_inh=100)
    say("case: no-alloc lock-step over 120 oracle steps")
    o = oracle_mod.Net(net).build()
    with snn.Net(net) as a, snn.Net(net) as b:
        a.build_synapses()
        b.build_synapses()
        for t in range(120):
            o.step(1)
            sp = o.spikes()
            ids = sp[sp[:, 0] == t, 1]
            a.step_forced(ids)
            b.step_forced_noalloc(ids)
            if t % 20 == 0 or t == 119:
                _same(a, b)
        np.testing.assert_array_equal(b.read_ring(), o.ring())
        np.testing.assert_array_equal(b.read_spikes(), o.spikes())


def test_limits_refused(snn):
    net = W.make(1, 1, W.GAUSS, 1.0, 0, 64, n_exc=8, n_inh=8)
    with snn.Net(net) as g:
        g.build_synapses()
        with pytest.raises(snn.SNNError, match="2\\^20"):
            g.step_forced_noalloc(np.zeros((1 << 20) + 1, dtype=np.uint32))
        with pytest.raises(snn.SNNError, match="out of range"):
            g.step_forced_noalloc([16])
        assert g.stats()["t"] == 0
        g.step_forced_noalloc([3])
        assert g.stats()["t"] == 1
