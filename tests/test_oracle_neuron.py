"""Pins of the oracle's neuron map (Eq. (1)-(2), threshold, reset, refractory)
against closed-form interspike intervals under constant drive.

With a constant charge J per 1 ms step, no recurrent synapses and E = 0, the
membrane value tested against the threshold at the k-th integrating step after
a refractory period is, in closed form,
    x_k = V_r P^(k-1) + J (1 - P^k)/(1 - P) - kappa w_1 (Q^(k-1) - P^(k-1))/(Q - P)
with P = exp(-1/tau_m), Q = exp(-1/tau_w) and w_1 the fatigue at the first
integrating step; the interval is 2 refractory steps plus the first k with
x_k > V_th.  Without adaptation (alpha = 0) the last term vanishes and every
interval is equal.
"""
import math

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W


def _net(J_mv, alpha=0.0, n_exc=4, n_inh=4, **over):
    return W.make(1, 1, W.GAUSS, 1.0, 0, 11, n_exc=n_exc, n_inh=n_inh, alpha_w=alpha,
                  ext_mode=W.EXT_CONST, ext_const_q=round(J_mv * 65536), **over)


def _isis(spikes, gid):
    t = spikes[spikes[:, 1] == gid, 0].astype(np.int64)
    return t, np.diff(t)


def _closed_form_isi(J, tau_m, tau_w, v_r, v_th, kappa, w1):
    P, Q = math.exp(-1 / tau_m), math.exp(-1 / tau_w)
    for k in range(1, 100000):
        x = v_r * P ** (k - 1) + J * (1 - P**k) / (1 - P)
        if w1 and Q != P:
            x -= kappa * w1 * (Q ** (k - 1) - P ** (k - 1)) / (Q - P)
        if x > v_th:
            return k + 2, x - v_th
    raise AssertionError("no threshold crossing")


@pytest.mark.parametrize("J,want", [(1.05, 29), (1.2, 16), (1.5, 9), (2.0, 6), (3.0, 4)])
def test_isi_without_adaptation(oracle_mod, J, want):
    net = _net(J)
    o = oracle_mod.Net(net).build()
    o.step(400)
    sp = o.spikes()
    Jq = round(J * 65536) / 65536
    isi, margin = _closed_form_isi(Jq, net["tau_m"], net["tau_w"], net["v_reset"], net["v_th"], 0, 0)
    assert margin > 1e-9
    assert isi == want  # values worked out by hand from the closed form
    for g in range(8):
        t, d = _isis(sp, g)
        assert len(d) >= 5
        assert np.all(d == isi)


def test_continuous_time_limit(oracle_mod):
    # as the drive shrinks the per-step map approaches the continuous LIF
    # interval tau_ref + tau_m ln((I tau_m - V_r)/(I tau_m - V_th)) (I = J/ms)
    net = _net(1.2)
    J = round(1.2 * 65536) / 65536
    cont = 2 + 20 * math.log((J * 20 - 15) / (J * 20 - 20))
    isi, _ = _closed_form_isi(J, 20.0, 500.0, 15.0, 20.0, 0, 0)
    assert abs(isi - cont) < 2.5


@pytest.mark.parametrize("J", [1.05, 1.2, 1.5, 2.0, 3.0])
def test_isi_with_adaptation(oracle_mod, J):
    net = _net(J, alpha=0.2)
    o = oracle_mod.Net(net).build()
    o.step(3000)
    sp = o.spikes()
    tb = oracle_mod.tables(net)
    Jq = round(J * 65536) / 65536
    Q = math.exp(-1 / net["tau_w"])
    for g in range(4):  # excitatory: adaptation on
        t, d = _isis(sp, g)
        assert len(d) >= 10
        # before the first spike w = 0, so w right after the first spike is alpha
        ws = net["alpha_w"]
        for k, got in enumerate(d):
            w1 = ws * Q**3
            isi, margin = _closed_form_isi(Jq, net["tau_m"], net["tau_w"], net["v_reset"], net["v_th"],
                                           tb["kappa"], w1)
            assert margin > 1e-9, "closed form too close to threshold to decide"
            assert got == isi, f"interval {k}"
            ws = ws * Q**isi + net["alpha_w"]
    for g in range(4, 8):  # inhibitory: no adaptation, constant intervals
        t, d = _isis(sp, g)
        assert np.all(d == d[0])
    V, w, ref = o.state()
    assert np.all(w[4:] == 0.0)


def test_adaptation_interval_sequences(oracle_mod):
    # worked out by hand from the one-step map: J = 1.2 mV, alpha = 0.2 mV:
    # first intervals 16, 16, 17, 17; J = 2 mV settles at 9; J = 3 mV at 5
    for J, head, tail in ((1.2, [16, 16, 17, 17], None), (2.0, None, 9), (3.0, None, 5)):
        net = _net(J, alpha=0.2)
        o = oracle_mod.Net(net).build()
        o.step(4000)
        t, d = _isis(o.spikes(), 0)
        if head:
            assert list(d[:4]) == head
        if tail:
            assert np.all(d[-20:] == tail)


def test_refractory_discards_input(oracle_mod):
    # a huge constant drive fires every 3 steps (spike + 2 refractory steps):
    # inputs during the refractory steps must not carry over
    net = _net(30.0)
    o = oracle_mod.Net(net).build()
    o.step(60)
    t, d = _isis(o.spikes(), 0)
    assert np.all(d == 3)
    V, w, ref = o.state()
    assert np.all((V == net["v_reset"]) | (ref == 0))


def test_initial_state(oracle_mod):
    net = W.workload("grid4_gauss")["net"]
    o = oracle_mod.Net(net)
    V, w, ref = o.state()
    assert np.all((V >= 0) & (V < 20)) and np.all(w == 0) and np.all(ref == 0)
    # uniform on [E, V_th): mean 10 mV, sd 20/sqrt(12)
    assert abs(V.mean() - 10.0) < 5 * (20 / math.sqrt(12)) / math.sqrt(V.size)
    assert V.std() == pytest.approx(20 / math.sqrt(12), rel=0.02)
