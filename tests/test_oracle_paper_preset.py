"""Pins of the oracle's paper connectivity preset (Sec. III.B): local
probability 0.8 inside a module for every source, remote probability
A exp(-r^2 / 2 sigma^2) (A = 0.05, sigma = 100 um) or A exp(-r / lambda)
(A = 0.03, lambda = 290 um) for excitatory sources only, cut off at
probability 1/1000.

* The synapse counts and stencil sizes the paper prints (fixture
  tests/golden/paper_preset_counts.txt) from the oracle's thresholds: local,
  remote and total expected in-degree, remote fraction, stencil side.
* The stencil reading: the square's edge is the first ring past the cut-off
  distance (probability at half-width h below 1/1000, at h - 1 above it).
* Inhibitory sources: only their own module.
* Built rows of a small network: inhibitory rows stay in the own module,
  excitatory rows inside the stencil, and the in-degree matches the
  thresholds' expectation within its binomial spread.
"""
import math
import os

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_preset_counts.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v, tol = line.split()
            out[k] = (float(v), float(tol))
    return out


def _signed(g):
    d = np.arange(g)
    return np.where(2 * d <= g, d, d - g)


def _counts(oracle_mod, law):
    net = W.make_paper(48, 48, law, 1)
    tb = oracle_mod.tables(net)
    M, n_exc = net["n_exc"] + net["n_inh"], net["n_exc"]
    pe = tb["T"].astype(np.float64) / 2.0**32
    pi = tb["T_inh"].astype(np.float64) / 2.0**32
    # expected in-degree of a target: its own module's other neurons (both
    # types) plus every other module's excitatory neurons
    local = (n_exc - 1) * pe[0, 0] + net["n_inh"] * pi[0, 0]
    remote = n_exc * (pe.sum() - pe[0, 0]) + net["n_inh"] * (pi.sum() - pi[0, 0])
    return net, tb, local, remote


@pytest.mark.parametrize("which", ["gauss", "exp"])
def test_printed_counts(oracle_mod, which):
    g = _golden()
    law = W.PAPER_GAUSS if which == "gauss" else W.PAPER_EXP
    net, tb, local, remote = _counts(oracle_mod, law)
    total = local + remote

    def near(key, got):
        want, tol = g[key]
        assert abs(got - want) <= tol * want, f"{key}: {got} vs printed {want}"

    near("local_synapses", local)
    near(f"{which}_remote_synapses", remote)
    near(f"{which}_total_synapses", total)
    near(f"{which}_remote_fraction", remote / total)
    # stencil: the nonzero excitatory offsets form a centred square of the printed side
    nz = tb["T"] > 0
    dx, dy = _signed(net["gx"]), _signed(net["gy"])
    side = int(g[f"{which}_stencil_side"][0])
    h = side // 2
    want = (np.abs(dy)[:, None] <= h) & (np.abs(dx)[None, :] <= h)
    np.testing.assert_array_equal(nz, want)
    # inhibitory sources: own module only
    assert tb["T_inh"][0, 0] == tb["T"][0, 0] and int((tb["T_inh"] > 0).sum()) == 1


@pytest.mark.parametrize("which", ["gauss", "exp"])
def test_stencil_edge_is_first_ring_past_cutoff(oracle_mod, which):
    law = W.PAPER_GAUSS if which == "gauss" else W.PAPER_EXP
    net = W.make_paper(48, 48, law, 1)
    tb = oracle_mod.tables(net)
    pe = tb["T"].astype(np.float64) / 2.0**32
    h = int(np.abs(_signed(net["gx"])[pe[0] > 0]).max())
    assert pe[0, h] < net["p_cut"] < pe[0, h - 1]
    assert pe[0, h + 1] == 0.0


def test_local_probability_exact(oracle_mod):
    for law in (W.PAPER_GAUSS, W.PAPER_EXP):
        tb = oracle_mod.tables(W.make_paper(8, 8, law, 1))
        assert tb["T"][0, 0] == round(0.8 * 2**32) == tb["T_inh"][0, 0]


@pytest.mark.parametrize("which", ["gauss", "exp"])
def test_built_rows_respect_the_preset(oracle_mod, which):
    law = W.PAPER_GAUSS if which == "gauss" else W.PAPER_EXP
    net = W.make_paper(24, 8, law, 21, n_exc=40, n_inh=10)
    M, gx = net["n_exc"] + net["n_inh"], net["gx"]
    N = gx * net["gy"] * M
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    tgt = recs.view(np.uint32).reshape(-1, 2)[:, 0]
    pre = np.repeat(np.arange(N), np.diff(row_ptr.astype(np.int64)))
    mi, mj = pre // M, tgt // M
    dx = (mj % gx - mi % gx) % gx
    dy = (mj // gx - mi // gx) % net["gy"]
    sdx = np.where(2 * dx <= gx, dx, dx - gx)
    sdy = np.where(2 * dy <= net["gy"], dy, dy - net["gy"])
    inh = (pre % M) >= net["n_exc"]
    assert np.all(mi[inh] == mj[inh])
    h = 3 if which == "gauss" else 10
    assert np.all((np.abs(sdx) <= h) & (np.abs(sdy) <= h))
    # in-degree against the thresholds' expectation (binomial spread)
    tb = oracle_mod.tables(net)
    pe = tb["T"].astype(np.float64) / 2.0**32
    expect = (net["n_exc"] - 1) * pe[0, 0] + net["n_inh"] * pe[0, 0] + net["n_exc"] * (pe.sum() - pe[0, 0])
    indeg = np.bincount(tgt, minlength=N)
    assert abs(indeg.mean() - expect) < 4.0 * math.sqrt(expect / N)


def test_problem_table_sizes(oracle_mod):
    """Neurons of the paper's three grids, and the Gaussian preset's recurrent
    synapse totals on the torus within 3 % of the printed ones."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_problem_sizes.txt")
    rows = [line.split("#", 1)[0].split() for line in open(path)]
    for g, neurons_m, syn_g, tol in (r for r in rows if r):
        g = int(g)
        net = W.make_paper(g, g, W.PAPER_GAUSS, 1)
        N = W.n_neurons(net)
        assert round(N / 1e6, 1) == float(neurons_m)
        tb = oracle_mod.tables(net)
        M = net["n_exc"] + net["n_inh"]
        n = np.full(tb["T"].shape, float(M))
        n[0, 0] = M - 1
        mean = (net["n_exc"] * (n * tb["T"]).sum() + net["n_inh"] * (n * tb["T_inh"]).sum()) / 2.0**32 / M
        assert abs(N * mean / 1e9 - float(syn_g)) <= float(tol) * float(syn_g), g
