"""GPU parity of the binomial synapse generator (a Binomial(n, p) count per
source and target module by integer CDF thresholds, then a uniform subset of
that size by Floyd's algorithm), through the C ABI, against the FP64 oracle:

* whole-network CSR bit-exact on small networks: the normalised lateral law
  and the paper's connectivity preset (counts near 990 in the own module),
  8-byte records and 8-bit codes;
* full size: sampled rows of the 96x96 exponential network built with the
  binomial generator bit-exact, its synapse total within the binomial spread
  of the expectation, and its construction time reported against the
  one-trial-per-pair build.
"""
import math
import sys
import time

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


CASES = [
    ("lateral gauss", dict(gx=6, gy=5, kernel=W.GAUSS, range=1.0, k_in=400.0, n_exc=80, n_inh=20)),
    ("lateral exp code8", dict(gx=7, gy=4, kernel=W.EXP, range=3.0, k_in=700.0, n_exc=96, n_inh=24,
                               record=W.REC_CODE8)),
    ("paper exp", None),
]


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_binomial_csr_bit_exact_small(snn, oracle_mod, name, over):
    if over is None:
        net = W.make_paper(24, 8, W.PAPER_EXP, 51, n_exc=40, n_inh=12, gen=W.GEN_BINOMIAL)
    else:
        net = W.make(over.pop("gx"), over.pop("gy"), over.pop("kernel"), over.pop("range"), over.pop("k_in"), 52,
                     gen=W.GEN_BINOMIAL, **over)
    say(f"case: binomial generator, {name}, whole CSR")
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    with snn.Net(net) as g:
        g.build_synapses()
        assert g.stats()["nnz"] == int(row_ptr[-1])
        rl, be, rc = g.export_rows(0, g.N)
        np.testing.assert_array_equal(rl, np.diff(row_ptr.astype(np.int64)))
        np.testing.assert_array_equal(be, bend)
        np.testing.assert_array_equal(rc, recs)


def test_binomial_full_size_96x96(snn, oracle_mod):
    net = W.workload("grid96_exp_code8", gen=W.GEN_BINOMIAL)["net"]
    say("case: grid96_exp_code8 with the binomial generator, full-size build, sampled rows")
    with snn.Net(net) as g:
        t0 = time.perf_counter()
        g.build_synapses()
        st = g.stats()
        dt = time.perf_counter() - t0
        N = g.N
        say(f"  {N} neurons, {st['nnz']} synapses in {dt:.2f} s (library build {st['build_ms'] / 1e3:.2f} s)")
        kin = net["k_in"]
        assert abs(st["nnz"] - kin * N) < 6.0 * math.sqrt(kin * N)
        rng = np.random.default_rng(7)
        rows = sorted(set([0, 991, 992, N - 1] + list(rng.integers(0, N, 6))))
        for r in rows:
            rl, be, rc = g.export_rows(int(r), 1)
            orl, obe, orc = oracle_mod.build_rows(net, int(r), 1)
            np.testing.assert_array_equal(rl, orl, err_msg=f"row {r}")
            np.testing.assert_array_equal(be, obe, err_msg=f"row {r}")
            np.testing.assert_array_equal(rc, orc, err_msg=f"row {r}")
