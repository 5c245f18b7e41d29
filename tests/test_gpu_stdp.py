"""GPU parity of spike-timing plasticity (Sec. II; Sec. II.A steps 1 and 4;
the long-term application every period) against the FP64 oracle, through the
C ABI.  The weights are integers (2^-16 mV) on both sides, so every check of
records and ring is bit-exact.

* Lock-step: the GPU is fed the oracle's spike set each step (direct, binned
  and two-level-free schedules); after every period's end all records
  (targets and weights) equal the oracle's, the delay ring is bit-exact (the
  changed weights are the ones delivered), state within tolerance.
* Free run with graph-replayed steps that stop at each period's end: a second
  network and the oracle, fed the first network's own raster, end with the
  same records.
* Full size (24x24 exponential, 786 M synapses): after one period of free
  running, the weight change of sampled synapses of sampled rows equals the
  oracle's pair sums over the GPU's own raster, clipped.
* Refusals: 8-bit codes, the exact solver, batches, too large w_max,
  per-launch timing; a history that overflows is reported.
"""
import sys

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W
from parity_helpers import compare_state

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


def _plastic(**over):
    net = W.make(2, 1, W.EXP, 2.0, 300, 41, n_exc=400, n_inh=100, ext_rate_hz=3.5, stdp=1, a_plus=0.01,
                 a_minus=0.0105, tau_plus=20.0, tau_minus=20.0, w_max=0.6, ltp_period=100)
    net.update(over)
    return net


@pytest.mark.parametrize("mode,thr", [(0, None), (1, 0), (1, None)])
def test_lockstep_weights_bit_exact(snn, oracle_mod, mode, thr):
    net = _plastic()
    say(f"case: plastic lock-step, delivery mode {mode}, threshold {thr}")
    o = oracle_mod.Net(net).build()
    _, _, c0 = o.csr()
    changed = 0
    with snn.Net(net) as g:
        g.build_synapses()
        g.set_option(snn.OPT_DELIVER_MODE, mode)
        if thr is not None:
            g.set_option(snn.OPT_BIN_THRESHOLD, thr)
        assert g.stats()["deliver_mode"] == mode
        for t in range(420):
            o.step(1)
            sp = o.spikes()
            g.step_forced(sp[sp[:, 0] == t, 1])
            if (t + 1) % 100 == 0 or t % 50 == 7:
                np.testing.assert_array_equal(g.read_ring(), o.ring(), err_msg=f"ring at step {t}")
                compare_state(net, g.read_state(), o.state(), t)
            if (t + 1) % 100 == 0:
                rl, be, rc = g.export_rows(0, g.N)
                rp, bo, ro = o.csr()
                np.testing.assert_array_equal(rl, np.diff(rp.astype(np.int64)))
                np.testing.assert_array_equal(rc, ro, err_msg=f"records after the period ending at {t}")
                changed += int((ro.view(np.uint32)[1::2] != c0.view(np.uint32)[1::2]).sum())
        np.testing.assert_array_equal(g.read_spikes(), o.spikes())
    say(f"weights changed (summed over periods): {changed}")
    assert changed > 1000


def test_free_run_graphs_stop_at_period_ends(snn, oracle_mod):
    net = _plastic(ltp_period=90)
    say("case: plastic free run with graphs (chunk 64, period 90)")
    with snn.Net(net) as a:
        a.build_synapses()
        a.set_option(snn.OPT_GRAPH_CHUNK, 64)
        a.step(200)          # calls that cross period ends (90, 180, ...) inside them
        a.step(170)
        a.step(80)           # and one that ends on one (450)
        raster = a.read_spikes()
        ra = a.export_rows(0, a.N)
        T = a.stats()["t"]
    assert T == 450 and raster.shape[0] > 1000
    o = oracle_mod.Net(net).build()
    with snn.Net(net) as b:
        b.build_synapses()
        for t in range(T):
            ids = raster[raster[:, 0] == t, 1]
            b.step_forced(ids)
            o.step_forced(ids)
        rb = b.export_rows(0, b.N)
    _, _, ro = o.csr()
    np.testing.assert_array_equal(ra[2], rb[2])
    np.testing.assert_array_equal(ra[2], ro)


def test_full_size_sampled_synapses(snn, oracle_mod):
    net = dict(W.workload("grid24_exp")["net"], stdp=1, ltp_period=1000)
    say("case: grid24_exp with plasticity, one period at full size")
    tb = oracle_mod.stdp_tables(net)
    with snn.Net(net, hist_cap=1 << 26) as g:
        g.build_synapses()
        g.set_option(snn.OPT_GRAPH_CHUNK, 250)
        g.step(999)
        rng = np.random.default_rng(17)
        raster = g.read_spikes()
        spikers = np.unique(raster[:, 1])
        exc = spikers[(spikers % 1240) < 992]
        rows = sorted(set(int(x) for x in rng.choice(exc, 6, replace=False)))
        rows += [int(rng.integers(0, g.N))]                         # any row, spiking or not
        before = {r: g.export_rows(r, 1) for r in rows}
        g.step(1)                                                  # ends the period
        raster = g.read_spikes()
        say(f"  {raster.shape[0]} spikes in the period; rows {rows}")
        for r in rows:
            rl, be, rc0 = before[r]
            _, _, rc1 = g.export_rows(r, 1)
            rec0 = rc0.view(np.uint32).reshape(-1, 2)
            rec1 = rc1.view(np.uint32).reshape(-1, 2)
            np.testing.assert_array_equal(rec0[:, 0], rec1[:, 0])
            w0 = np.rint(rec0[:, 1].view(np.float32).astype(np.float64) * 65536).astype(np.int64)
            w1 = np.rint(rec1[:, 1].view(np.float32).astype(np.float64) * 65536).astype(np.int64)
            k = np.arange(int(rl[0]))
            delay = net["d_min"] + (be[0].astype(np.int64)[None, :] <= k[:, None]).sum(axis=1)
            pick = np.sort(rng.choice(k.size, min(k.size, 120), replace=False))
            involved = np.concatenate([[r], rec0[pick, 0]])
            sub = raster[np.isin(raster[:, 1], involved)]      # the spikes these synapses can pair
            tot = oracle_mod.stdp_totals(net, sub, np.full(pick.size, r), rec0[pick, 0], delay[pick], 0, 1000)
            want = np.where(tot != 0, np.clip(w0[pick] + tot, 0, tb["wmax_q"]), w0[pick])
            np.testing.assert_array_equal(w1[pick], want, err_msg=f"row {r}")
            if (r % 1240) < 992 and r in spikers:
                assert (tot != 0).any(), f"row {r}: no pair in the sample"


def test_refusals_and_history_overflow(snn):
    base = _plastic()
    for over in (dict(record=W.REC_CODE8), dict(solver=W.SOLVER_EXACT), dict(w_max=1.0), dict(ltp_period=0)):
        with snn.Net(dict(base, **over)) as g:
            with pytest.raises(snn.SNNError):
                g.build_synapses()
    with snn.Net(base) as g:
        g.build_synapses()
        with pytest.raises(snn.SNNError):
            g.time_kernels(10)
    with snn.Batch(1 << 30, 1 << 16) as b:
        with pytest.raises(snn.SNNError):
            b.admit(base, 10)
    with snn.Net(base, hist_cap=64) as g:
        g.build_synapses()
        g.step(100)
        with pytest.raises(snn.SNNError, match="history"):
            g.stats()
