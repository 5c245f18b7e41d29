"""GPU parity of the paper's connectivity preset (Sec. III.B: 80 % local
probability for every source, remote A f(r) for excitatory sources inside
the 7x7 / 21x21 stencil; inhibitory neurons local only), through the C ABI,
against the FP64 oracle.

* Whole-network CSR bit-exact (row lengths, bucket ends, records) on small
  grids, Gaussian and exponential, 8-byte records and 8-bit codes.
* Lock-step (the GPU is fed the oracle's spike set) on a small preset grid:
  state within the lock-step tolerance, the delay ring bit-exact.
* Full size: sampled rows of the 48x48 exponential preset network
  (2.86 M neurons, 6.8 G synapses, 8-bit codes) and of the 24x24 Gaussian
  one bit-exact, and the synapse total within its binomial spread of the
  thresholds' expectation.
"""
import math
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

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


@pytest.mark.parametrize("law,record", [("gauss", W.REC_F32), ("exp", W.REC_F32), ("exp", W.REC_CODE8)])
def test_preset_csr_bit_exact_small(snn, oracle_mod, law, record):
    net = W.make_paper(24, 8, W.PAPER_GAUSS if law == "gauss" else W.PAPER_EXP, 31, n_exc=40, n_inh=12,
                       record=record)
    say(f"case: paper preset {law} record {record}, 24x8 grid of 52-neuron modules, whole CSR")
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    with snn.Net(net) as g:
        g.build_synapses()
        assert g.stats()["nnz"] == int(row_ptr[-1])
        rl, be, rc = g.export_rows(0, g.N)
        np.testing.assert_array_equal(rl, np.diff(row_ptr.astype(np.int64)))
        np.testing.assert_array_equal(be, bend)
        np.testing.assert_array_equal(rc, recs)


def test_preset_lockstep_small(snn, oracle_mod):
    net = W.make_paper(8, 4, W.PAPER_EXP, 32, n_exc=80, n_inh=20, ext_rate_hz=6.0)
    say("case: paper preset exponential, 8x4 grid of 100-neuron modules, lock-step 300 steps")
    o = oracle_mod.Net(net).build()
    with snn.Net(net) as g:
        g.build_synapses()
        for t in range(300):
            o.step(1)
            sp = o.spikes()
            g.step_forced(sp[sp[:, 0] == t, 1])
            Vg, Wg, Rg = g.read_state()
            Vo, Wo, Ro = o.state()
            tolV = 1e-5 * np.maximum(np.abs(Vo), net["v_th"] - net["e_rest"])
            assert np.all(np.abs(Vg.astype(np.float64) - Vo) <= tolV), f"step {t}"
            tolw = 1e-5 * np.maximum(np.abs(Wo), net["alpha_w"])
            assert np.all(np.abs(Wg.astype(np.float64) - Wo) <= tolw), f"step {t}"
            np.testing.assert_array_equal(Rg.astype(np.int32), Ro)
            if t % 25 == 0:
                np.testing.assert_array_equal(g.read_ring(), o.ring(), err_msg=f"ring at step {t}")
        np.testing.assert_array_equal(g.read_ring(), o.ring())
        np.testing.assert_array_equal(g.read_spikes(), o.spikes())
        assert g.stats()["rec_events"] == o.stats()["rec_events"]
        say(f"  spikes {g.stats()['spikes']}, recurrent events {g.stats()['rec_events']}")


@pytest.mark.parametrize("name", ["grid24_gauss_paper", "grid48_exp_paper_code8"])
def test_preset_full_size_sampled_rows(snn, oracle_mod, name):
    net = W.workload(name)["net"]
    say(f"case: {name} full-size build, sampled rows")
    tb = oracle_mod.tables(net)
    M, n_exc = net["n_exc"] + net["n_inh"], net["n_exc"]
    pe = tb["T"].astype(np.float64) / 2.0**32
    pi = tb["T_inh"].astype(np.float64) / 2.0**32
    n = np.full(pe.shape, float(M))
    n[0, 0] = M - 1
    mean = (n_exc * (n * pe).sum() + net["n_inh"] * (n * pi).sum()) / M
    with snn.Net(net) as g:
        g.build_synapses()
        N = g.N
        nnz = g.stats()["nnz"]
        var = (n_exc * (n * pe * (1 - pe)).sum() + net["n_inh"] * (n * pi * (1 - pi)).sum()) / M * N
        say(f"  {N} neurons, {nnz} synapses ({nnz / N:.1f} per neuron, expected {mean:.1f})")
        assert abs(nnz - mean * N) < 6.0 * math.sqrt(var)
        rng = np.random.default_rng(6)
        rows = sorted(set([0, n_exc - 1, n_exc, M - 1, N - 1] + list(rng.integers(0, N, 12))))
        for r in rows:
            rl, be, rc = g.export_rows(int(r), 1)
            orl, obe, orc = oracle_mod.build_rows(net, int(r), 1)
            np.testing.assert_array_equal(rl, orl, err_msg=f"row {r}")
            np.testing.assert_array_equal(be, obe, err_msg=f"row {r}")
            np.testing.assert_array_equal(rc, orc, err_msg=f"row {r}")
