"""GPU parity of exponential delays (Sec. II.B), through the C ABI, against
the FP64 oracle: whole-network CSR bit-exact (bucket ends follow the
exponential law's thresholds) and 200 lock-step steps with the delay ring
bit-exact."""
import sys

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snn():
    from paper_1803_08833_amd import snn as S

    S.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


@pytest.mark.parametrize("record", [W.REC_F32, W.REC_CODE8])
def test_exponential_delays_csr_and_lockstep(snn, oracle_mod, record):
    net = W.make(4, 4, W.EXP, 2.0, 300, 63, n_exc=80, n_inh=20, delay_dist=W.DELAY_EXP, delay_tau=3.0,
                 record=record, ext_rate_hz=6.0)
    print(f"case: exponential delays (tau 3 ms), record {record}", flush=True)
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    with snn.Net(net) as g:
        g.build_synapses()
        rl, be, rc = g.export_rows(0, g.N)
        np.testing.assert_array_equal(rl, np.diff(row_ptr.astype(np.int64)))
        np.testing.assert_array_equal(be, bend)
        np.testing.assert_array_equal(rc, recs)
        for t in range(200):
            o.step(1)
            sp = o.spikes()
            g.step_forced(sp[sp[:, 0] == t, 1])
            if t % 20 == 0:
                np.testing.assert_array_equal(g.read_ring(), o.ring(), err_msg=f"ring at step {t}")
        np.testing.assert_array_equal(g.read_ring(), o.ring())
        np.testing.assert_array_equal(g.read_spikes(), o.spikes())
        assert g.stats()["rec_events"] == o.stats()["rec_events"]
