"""Pins of the oracle's spike-timing plasticity (Sec. II: STDP with long-term
potentiation/depression; Sec. II.A steps 1 and 4 compute the contributions
at postsynaptic spikes and at synaptic arrivals; they are integrated and
applied every second).

Reading (pair-based, exponential windows, integer weights in 2^-16 mV): a
synapse i -> j of delay d sees a presynaptic event at each arrival a = s + d
of a spike of i at step s and a postsynaptic event at each spike of j at step
p.  Every pair within the window contributes kp[p - a] when p >= a and
-km[a - p] when p < a; the changes of a period are applied at its end, with
the weight clipped to [0, w_max] (a synapse whose total change is zero keeps
its weight); inhibitory synapses are fixed.

Pinned against closed forms computed here, not by the oracle's event loop:
* tables: kp[0] = round(A+ 2^16), successive ratios exp(-1/tau) within the
  rounding, the window ends at the first lag where both round to zero;
* one pair at every lag from -(win+2) to win+2, in a network driven only by
  forced spikes, changes exactly the synapse's weight by F(lag);
* a periodic pair train of n pairs (period T, offset delta) changes the weight
  by sum_q (n - |q|) F(delta + qT), the all-to-all pair count;
* a pair whose later event falls after a period's end changes the weight at
  the next period's end, not before;
* clipping at 0 and w_max; inhibitory synapses unchanged.
Planted mistakes (compiled from the oracle's source with one line changed)
must each fail one of these pins.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1803_08833_amd import workloads as W

A_PLUS, A_MINUS, TAU_P, TAU_M = 0.004, 0.0042, 20.0, 17.0
PERIOD = 300


def _net(seed=5, **over):
    d = W.make(1, 1, W.GAUSS, 1.0, 8, seed, n_exc=16, n_inh=4, ext_mode=W.EXT_CONST, ext_const_q=0,
               stdp=1, a_plus=A_PLUS, a_minus=A_MINUS, tau_plus=TAU_P, tau_minus=TAU_M, w_max=0.8,
               ltp_period=PERIOD, d_min=1, d_max=6)
    d.update(over)
    return d


def _closed_tables(win):
    k = np.arange(win)
    kp = np.rint(A_PLUS * np.exp(-k / TAU_P) * 65536.0).astype(np.int64)
    km = np.rint(A_MINUS * np.exp(-k / TAU_M) * 65536.0).astype(np.int64)
    km[0] = 0
    return kp, km


def _F(lag, kp, km):
    win = len(kp)
    if 0 <= lag < win:
        return int(kp[lag])
    if lag < 0 and -lag < win:
        return -int(km[-lag])
    return 0


def _synapses(o, net):
    """(pre, target, delay, weight_q, index) of every synapse of the CSR."""
    row_ptr, bend, recs = o.csr()
    rec = recs.view(np.uint32).reshape(-1, 2)
    tgt = rec[:, 0]
    wq = np.rint(rec[:, 1].view(np.float32).astype(np.float64) * 65536).astype(np.int64)
    out = []
    for i in range(o.N):
        r0, r1 = int(row_ptr[i]), int(row_ptr[i + 1])
        for k in range(r0, r1):
            b = int(np.searchsorted(bend[i].astype(np.int64), k - r0, side="right"))
            out.append((i, int(tgt[k]), net["d_min"] + b, int(wq[k]), k))
    return out


def _exc_pair(o, net):
    """An excitatory -> excitatory synapse with no synapse back."""
    syn = _synapses(o, net)
    pairs = {(i, j) for i, j, _, _, _ in syn}
    for i, j, d, w, k in syn:
        if i < net["n_exc"] and j < net["n_exc"] and (j, i) not in pairs:
            return i, j, d, w, k
    raise AssertionError("no one-way excitatory synapse")


def _run(net, spikes, steps):
    """Oracle driven only by forced spikes {step: [gids]}; returns the weights
    (q) of every synapse afterwards."""
    o = oracle.Net(net).build()
    for t in range(steps):
        o.step_forced(np.array(spikes.get(t, []), dtype=np.uint32))
    return o, {(i, j): w for i, j, _, w, _ in _synapses(o, net)}


def pin_tables():
    tb = oracle.stdp_tables(_net())
    kp, km = tb["kp"].astype(np.int64), tb["km"].astype(np.int64)
    ckp, ckm = _closed_tables(tb["win"])
    ok = np.array_equal(kp, ckp) and np.array_equal(km, ckm)
    # the window is the first lag where both round to zero
    nxt = np.rint(np.array([A_PLUS * np.exp(-tb["win"] / TAU_P), A_MINUS * np.exp(-tb["win"] / TAU_M)]) * 65536)
    ok = ok and not nxt.any() and (kp[-1] or km[-1])
    # successive ratios within the rounding
    big = kp > 50
    r = kp[1:][big[1:]] / kp[:-1][big[1:]]
    ok = ok and np.all(np.abs(r - np.exp(-1 / TAU_P)) < 1.0 / kp[1:][big[1:]])
    return bool(ok), f"win {tb['win']} kp0 {kp[0]} km1 {km[1]}"


def _run_cases(net, i, j, cases):
    """One case per period: cases[c] is the period-relative {step: [gids]}
    schedule; returns the weight of i -> j at the end of every period."""
    o = oracle.Net(net).build()
    out = []
    for c, spikes in enumerate(cases):
        for t in range(PERIOD):
            o.step_forced(np.array(spikes.get(t, []), dtype=np.uint32))
        out.append({(a, b): x for a, b, _, x, _ in _synapses(o, net)}[(i, j)])
    return out


def pin_single_pairs():
    """One pair per period, far enough from the next period's pair to be
    outside each other's window."""
    net = _net()
    o0 = oracle.Net(net).build()
    i, j, d, w0, _ = _exc_pair(o0, net)
    tb = oracle.stdp_tables(net)
    kp, km = _closed_tables(tb["win"])
    lags = list(range(-(tb["win"] + 2), tb["win"] + 3, 7)) + [-2, -1, 0, 1, 2, tb["win"] - 1, tb["win"]]
    cases = []
    for lag in lags:
        s = 150 - max(lag, 0) // 2 - d
        spikes = {s: [i]}
        spikes.setdefault(s + d + lag, []).append(j)   # may be the same step as i's spike
        cases.append(spikes)
    got = _run_cases(net, i, j, cases)
    bad, w = [], w0
    for lag, g in zip(lags, got):
        w = min(max(w + _F(lag, kp, km), 0), tb["wmax_q"])
        if g != w:
            bad.append((lag, g, w))
            w = g
    return not bad, f"lags with a wrong change: {bad[:5]}"


def pin_trains():
    net = _net(seed=9)
    o0 = oracle.Net(net).build()
    i, j, d, w0, _ = _exc_pair(o0, net)
    tb = oracle.stdp_tables(net)
    kp, km = _closed_tables(tb["win"])
    trains = ((7, 0), (7, -3), (11, 2), (5, -1), (40, 4))
    cases, wants = [], []
    for T, delta in trains:
        n = 8 if T < 30 else 3        # every event inside its period, clear of the next
        spikes = {}
        for k in range(n):
            spikes.setdefault(20 + k * T, []).append(i)
            spikes.setdefault(20 + k * T + d + delta, []).append(j)
        cases.append(spikes)
        wants.append(sum((n - abs(q)) * _F(delta + q * T, kp, km) for q in range(-(n - 1), n)))
    got = _run_cases(net, i, j, cases)
    bad, w = [], w0
    for tr, g, dw in zip(trains, got, wants):
        w = min(max(w + dw, 0), tb["wmax_q"])
        if g != w:
            bad.append((tr, g, w))
            w = g
    return not bad, f"trains with a wrong change: {bad}"


def pin_period_boundary():
    net = _net(seed=11)
    o0 = oracle.Net(net).build()
    i, j, d, w0, _ = _exc_pair(o0, net)
    tb = oracle.stdp_tables(net)
    kp, km = _closed_tables(tb["win"])
    bad = []
    # potentiation: arrival before the end, spike after it
    s = PERIOD - d - 2
    p = PERIOD + 3
    o = oracle.Net(net).build()
    for t in range(2 * PERIOD):
        ids = [i] if t == s else ([j] if t == p else [])
        o.step_forced(np.array(ids, dtype=np.uint32))
        if t == PERIOD - 1 or t == 2 * PERIOD - 1:
            w = {(a, b): x for a, b, _, x, _ in _synapses(o, net)}[(i, j)]
            want = w0 if t == PERIOD - 1 else w0 + _F(p - s - d, kp, km)
            if w != want:
                bad.append(("ltp", t, w - w0, want - w0))
    # depression: spike before the end, arrival after it
    p = PERIOD - 4
    s = PERIOD - d + 2
    o = oracle.Net(net).build()
    for t in range(2 * PERIOD):
        ids = [j] if t == p else ([i] if t == s else [])
        o.step_forced(np.array(ids, dtype=np.uint32))
        if t == PERIOD - 1 or t == 2 * PERIOD - 1:
            w = {(a, b): x for a, b, _, x, _ in _synapses(o, net)}[(i, j)]
            want = w0 if t == PERIOD - 1 else w0 + _F(p - s - d, kp, km)
            if w != want:
                bad.append(("ltd", t, w - w0, want - w0))
    # pairs completed at the last step of the period (counted in it) and at
    # the first step of the next (counted there)
    for p, first in ((PERIOD - 1, True), (PERIOD, False)):
        s = p - d - 3
        o = oracle.Net(net).build()
        for t in range(PERIOD):
            ids = [i] if t == s else ([j] if t == p else [])
            o.step_forced(np.array(ids, dtype=np.uint32))
        w = {(a, b): x for a, b, _, x, _ in _synapses(o, net)}[(i, j)]
        want = w0 + _F(3, kp, km) if first else w0
        if w != want:
            bad.append(("edge", p, w - w0, want - w0))
    return not bad, f"{bad}"


def pin_clip_and_inhibitory():
    bad = []
    # 60 pairs at lag 0 (potentiation beyond w_max), then 60 pairs at lag -1
    # with a strong depression amplitude (below zero): the closed-form totals
    # cross the bounds, the weights stop at them
    for a_minus, delta, bound in ((A_MINUS, 0, "max"), (0.02, -1, "zero")):
        net = _net(seed=13, w_max=0.45, a_minus=a_minus)
        o0 = oracle.Net(net).build()
        i, j, d, w0, _ = _exc_pair(o0, net)
        tb = oracle.stdp_tables(net)
        k = np.arange(tb["win"])
        kp = np.rint(A_PLUS * np.exp(-k / TAU_P) * 65536.0).astype(np.int64)
        km = np.rint(a_minus * np.exp(-k / TAU_M) * 65536.0).astype(np.int64)
        km[0] = 0
        n, T = 60, 4
        spikes = {}
        for m in range(n):
            spikes.setdefault(10 + T * m, []).append(i)
            spikes.setdefault(10 + T * m + d + delta, []).append(j)
        total = sum((n - abs(q)) * _F(delta + q * T, kp, km) for q in range(-(n - 1), n))
        want = tb["wmax_q"] if bound == "max" else 0
        assert (w0 + total > tb["wmax_q"]) if bound == "max" else (w0 + total < 0)
        _, w = _run(net, spikes, PERIOD)
        if w[(i, j)] != want:
            bad.append((bound, w[(i, j)], want))
    # every neuron firing every 3 steps: inhibitory synapses keep their weight
    net = _net(seed=13)
    o0 = oracle.Net(net).build()
    syn0 = _synapses(o0, net)
    allspk = {t: list(range(o0.N)) for t in range(5, PERIOD - 30, 3)}
    _, w = _run(net, allspk, PERIOD)
    changed_exc = 0
    for a, b, _, x, _ in syn0:
        if a >= net["n_exc"] and w[(a, b)] != x:
            bad.append(("inh", a, b))
            break
        changed_exc += a < net["n_exc"] and w[(a, b)] != x
    if not changed_exc:
        bad.append(("no excitatory synapse changed",))
    return not bad, f"{bad}"


PINS = [pin_tables, pin_single_pairs, pin_trains, pin_period_boundary, pin_clip_and_inhibitory]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_stdp_pin(oracle_mod, pin):
    ok, detail = pin()
    assert ok, detail


def test_stdp_off_leaves_weights():
    net = _net(seed=7, stdp=0)
    o0 = oracle.Net(net).build()
    w0 = {(i, j): w for i, j, _, w, _ in _synapses(o0, net)}
    spikes = {t: list(range(o0.N)) for t in range(5, PERIOD, 3)}
    _, w = _run(net, spikes, PERIOD + 1)
    assert w == w0


def test_stdp_needs_f32_step_solver():
    with pytest.raises(ValueError):
        oracle.Net(_net(record=W.REC_CODE8))
    with pytest.raises(ValueError):
        oracle.Net(_net(solver=W.SOLVER_EXACT))


PLANTED = {
    "same-step pair not potentiating": ("                if (a > t) break;", "                if (a >= t) break;"),
    "delay ignored": ("                uint32_t a = n->spk[i][q] + d;", "                uint32_t a = n->spk[i][q];"),
    "depression sign": ("                    n->acc[k] -= tb->km[t - p];", "                    n->acc[k] += tb->km[t - p];"),
    "lag off by one": ("                if (t - a < win) n->acc[k] += tb->kp[t - a];",
                       "                if (t - a < win) n->acc[k] += tb->kp[t - a + 1];"),
    "applied one step early": ("        if ((t + 1) % c->ltp_period == 0) stdp_apply(n);",
                               "        if ((t + 2) % c->ltp_period == 0) stdp_apply(n);"),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_mistake_fails_a_pin(oracle_mod, name):
    old, new = PLANTED[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, old
    d = tempfile.mkdtemp(prefix="oracle_variant_")
    path = os.path.join(d, "variant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(d, "variant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", so, path, "-lm"])
    with oracle.library(so):
        results = [p() for p in PINS[1:]]
    assert not all(ok for ok, _ in results), f"planted mistake '{name}' passed every pin"


def test_pair_totals_match_event_driven_run(oracle_mod):
    """stdp_totals (the period's change summed pair by pair from a raster,
    used for sampled checks of large networks) equals the weight change the
    event-driven run applies, for every excitatory synapse of a recurrent
    network with Poisson drive over two periods."""
    net = W.make(2, 1, W.EXP, 2.0, 60, 31, n_exc=80, n_inh=20, ext_rate_hz=8.0, stdp=1, a_plus=0.01,
                 a_minus=0.011, tau_plus=TAU_P, tau_minus=TAU_M, w_max=0.9, ltp_period=150)
    o = oracle.Net(net).build()
    syn0 = _synapses(o, net)
    o.step(150)
    syn1 = _synapses(o, net)
    o.step(150)
    syn2 = _synapses(o, net)
    raster = o.spikes()
    assert raster.shape[0] > 300
    pre = np.array([x[0] for x in syn0])
    tgt = np.array([x[1] for x in syn0])
    dl = np.array([x[2] for x in syn0])
    wmax = oracle.stdp_tables(net)["wmax_q"]
    changed = 0
    for (T0, T1), before, after in (((0, 150), syn0, syn1), ((150, 300), syn1, syn2)):
        tot = oracle.stdp_totals(net, raster, pre, tgt, dl, T0, T1)
        w0 = np.array([x[3] for x in before])
        w1 = np.array([x[3] for x in after])
        want = np.where(tot != 0, np.clip(w0 + tot, 0, wmax), w0)
        np.testing.assert_array_equal(w1, want)
        changed += int((w1 != w0).sum())
    assert changed > 100
