"""Pins of the oracle's host tables against closed forms and library routines.

* Connection thresholds: normalisation (expected in-degree equals k_in), the
  two limits with a textbook answer (uniform law, purely local law), torus
  symmetry and monotone decrease with distance, and the prefactors of the
  workloads computed by hand from the lateral laws, independently of the
  oracle's code.
* Weight table and codebook: conditional means of normal bins against
  scipy.stats.truncnorm.
* Poisson CDF thresholds against scipy.stats.poisson.
* Neuron propagator against scipy.linalg.expm of the 2x2 linear system.
"""
import math

import numpy as np
import pytest
from scipy import linalg, special, stats

from paper_1803_08833_amd import workloads as W


def _tables(oracle_mod, name, **over):
    net = W.workload(name, **over)["net"]
    return net, oracle_mod.tables(net)


def _offset_counts(net):
    gx, gy, M = net["gx"], net["gy"], net["n_exc"] + net["n_inh"]
    n = np.full((gy, gx), float(M))
    n[0, 0] = M - 1
    return n


def _r2(net):
    gx, gy = net["gx"], net["gy"]
    dx = np.arange(gx)
    dx = np.where(2 * dx <= gx, dx, dx - gx)
    dy = np.arange(gy)
    dy = np.where(2 * dy <= gy, dy, dy - gy)
    return dy[:, None] ** 2 + dx[None, :] ** 2


@pytest.mark.parametrize("name", ["grid4_gauss", "grid24_gauss", "grid24_exp", "grid96_exp_code8"])
def test_threshold_normalisation(oracle_mod, name):
    net, tb = _tables(oracle_mod, name)
    T = tb["T"].astype(np.float64)
    n = _offset_counts(net)
    expected_k = (n * T).sum() / 2**32
    # rounding each threshold to an integer moves the sum by at most n/2 per offset
    assert abs(expected_k - net["k_in"]) <= n.sum() * 0.5 / 2**32 + 1e-9


# Prefactors B computed by hand from the lateral laws on the torus with
# n(0) = module size - 1 (independently of the oracle's code).
@pytest.mark.parametrize("name,B", [("grid4_gauss", 0.160876), ("grid24_gauss", 0.0627528),
                                    ("grid24_exp", 0.0075768), ("grid96_exp_code8", 0.00527054)])
def test_threshold_prefactor(oracle_mod, name, B):
    net, tb = _tables(oracle_mod, name)
    assert tb["T"][0, 0] / 2**32 == pytest.approx(B, rel=2e-5)


def test_gauss_24_stencil_size(oracle_mod):
    # sigma = 1.5 modules on 24x24: 293 of 576 offsets have a non-zero 32-bit threshold
    _, tb = _tables(oracle_mod, "grid24_gauss")
    assert int((tb["T"] > 0).sum()) == 293


def test_threshold_uniform_limit(oracle_mod):
    # lambda -> infinity: f = 1 everywhere, p = k_in / (N - 1) for every pair
    net, tb = _tables(oracle_mod, "grid4_gauss", kernel=W.EXP, range=1e15)
    N = W.n_neurons(net)
    want = round(net["k_in"] / (N - 1) * 2**32)
    assert np.all(np.abs(tb["T"].astype(np.int64) - want) <= 1)


def test_threshold_local_limit(oracle_mod):
    # sigma -> 0: only the own module connects, p = k_in / (M - 1)
    net, tb = _tables(oracle_mod, "grid4_gauss", range=0.05, k_in=600)
    M = net["n_exc"] + net["n_inh"]
    assert tb["T"][0, 0] == round(600 / (M - 1) * 2**32)
    assert int((tb["T"] > 0).sum()) == 1


@pytest.mark.parametrize("name", ["grid24_gauss", "grid24_exp"])
def test_threshold_symmetry_and_monotone(oracle_mod, name):
    net, tb = _tables(oracle_mod, name)
    T = tb["T"].astype(np.int64)
    gx, gy = net["gx"], net["gy"]
    for ry in range(gy):
        for rx in range(gx):
            assert T[ry, rx] == T[(-ry) % gy, (-rx) % gx] == T[rx % gy, ry % gx]
    r2 = _r2(net).ravel()
    order = np.argsort(r2, kind="stable")
    ts = T.ravel()[order]
    assert np.all(np.diff(ts) <= 0)
    # shape of the law: T(r) / T(0) follows f(r) / f(0)
    r = np.sqrt(r2.astype(np.float64))
    f = np.exp(-r / net["range"]) if net["kernel"] == W.EXP else np.exp(-r**2 / (2 * net["range"] ** 2))
    big = T.ravel() > 10**4
    np.testing.assert_allclose(T.ravel()[big] / T[0, 0], f[big], rtol=2e-4)


def test_weight_table_conditional_means(oracle_mod):
    net, tb = _tables(oracle_mod, "grid4_gauss")
    k = np.arange(65536)
    a = special.ndtri(k / 65536.0)
    b = special.ndtri((k + 1) / 65536.0)
    m = stats.truncnorm.mean(a, b)
    exact = 65536.0 * (net["w_exc"] + net["w_exc_sd"] * m)
    err = np.abs(tb["wtab"] - exact)
    assert err.max() <= 0.5 + 1e-6
    assert np.all(np.diff(tb["wtab"]) >= 0)
    # the table's mean is the distribution mean (conditional means preserve it)
    assert abs(tb["wtab"].mean() / 65536 - net["w_exc"]) < 1e-6
    assert tb["wtab"].std() / 65536 == pytest.approx(net["w_exc_sd"], rel=1e-3)


def test_codebook_conditional_means(oracle_mod):
    net, tb = _tables(oracle_mod, "grid96_exp_code8")
    cb = tb["cb"]
    c = np.arange(256, dtype=object)
    edges = np.array([-(-(int(x) * 2**32) // 255) for x in c], dtype=np.float64) / 2**32
    a, b = special.ndtri(edges[:255]), special.ndtri(edges[1:256])
    m = stats.truncnorm.mean(a, b)
    exact = 65536.0 * (net["w_exc"] + net["w_exc_sd"] * m)
    assert np.abs(cb[:255] - exact).max() <= 0.5 + 1e-6
    assert cb[255] == round(net["w_inh"] * 65536)
    # probability-weighted codebook mean equals the excitatory mean
    p = np.diff(edges)
    assert abs((p * cb[:255]).sum() / 65536 - net["w_exc"]) < 2e-6


def test_poisson_thresholds(oracle_mod):
    for rate in (3.0, 0.5, 10.0):
        net, tb = _tables(oracle_mod, "grid4_gauss", ext_rate_hz=rate)
        m = net["ext_n"] * rate * 1e-3
        pc = tb["poisc"].astype(np.float64)
        k = np.arange(pc.size)
        exact = stats.poisson.cdf(k, m) * 2**32
        assert np.abs(pc - exact).max() <= 0.5 + 2**32 * 1e-14
        # the table stops exactly where the rounded CDF reaches 2^32
        assert round(stats.poisson.cdf(pc.size, m) * 2**32) >= 2**32 - 1
    assert tb["jext_q"] == round(net["ext_w"] * 65536)


def test_propagator_matches_expm(oracle_mod):
    for tau_m, tau_w in ((20.0, 500.0), (10.0, 30.0), (20.0, 20.0)):
        net, tb = _tables(oracle_mod, "grid4_gauss", tau_m=tau_m, tau_w=tau_w)
        # state (u, w): du/dt = -(u + w)/tau_m, dw/dt = -w/tau_w, one 1 ms step
        A = np.array([[-1 / tau_m, -1 / tau_m], [0.0, -1 / tau_w]])
        E = linalg.expm(A)
        assert tb["dm"] == pytest.approx(1 - E[0, 0], rel=1e-12)
        assert tb["dw"] == pytest.approx(1 - E[1, 1], rel=1e-12)
        assert tb["kappa"] == pytest.approx(-E[0, 1], rel=1e-10)
    assert tb["nref"] == round(net["t_ref"])
    assert math.isclose(tb["winh_q"], round(net["w_inh"] * 65536))
