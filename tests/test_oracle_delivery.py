"""Pins of the oracle's spike delivery (Sec. II.A steps 2-4, Sec. II.E):

* brute force: a dense W[delay][post][pre] simulation (matrix products over
  the spike history, no delay ring) gives the same per-step charge, the same
  spike raster and the same membrane potentials as the oracle's ring;
* exact charge conservation: the charge read out of the ring over a run plus
  what is still queued equals the sum, over all spikes, of the fixed-point
  weights of the spiker's projection (int64, no rounding anywhere);
* event counting: recurrent events = sum of the spikers' row lengths.
"""
import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

from test_oracle_connectivity import decode


def test_dense_brute_force(oracle_mod):
    # 1x2 grid of 200-neuron modules, Gaussian sigma 1, 100 synapses per neuron,
    # constant external charge: small enough for dense matrices
    net = W.make(2, 1, W.GAUSS, 1.0, 100, 21, n_exc=160, n_inh=40, ext_mode=W.EXT_CONST,
                 ext_const_q=round(1.1 * 65536))
    N = W.n_neurons(net)
    D = net["d_max"] - net["d_min"] + 1
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    pre, tgt, wq, delay = decode(net, row_ptr, bend, recs)
    Wd = np.zeros((D + 1, N, N), dtype=np.int64)
    np.add.at(Wd, (delay, tgt, pre), wq)
    tb = oracle_mod.tables(net)
    V, w, ref = o.state()
    V = V.copy()
    w = w.copy()
    ref = ref.copy()
    exc = (np.arange(N) % 200) < 160
    steps = 300
    S = np.zeros((steps, N), dtype=np.int64)
    dense_spikes = []
    for t in range(steps):
        I = np.full(N, net["ext_const_q"], dtype=np.int64)
        for d in range(1, D + 1):
            if t - d >= 0:
                I += Wd[d] @ S[t - d]
        J = I / 65536.0
        refr = ref > 0
        Vn = V + J
        spk = (~refr) & (Vn > net["v_th"])
        u = Vn - net["e_rest"]
        u = u - u * tb["dm"] - tb["kappa"] * w
        V = np.where(refr, net["v_reset"], np.where(spk, net["v_reset"], net["e_rest"] + u))
        w = np.where(spk & exc, w + net["alpha_w"], w)
        ref = np.where(refr, ref - 1, np.where(spk, tb["nref"], ref))
        w = w - w * tb["dw"]
        S[t] = spk
        dense_spikes += [(t, g) for g in np.nonzero(spk)[0]]
    o.step(steps)
    got = [tuple(x) for x in o.spikes()]
    assert len(got) > 200
    assert got == dense_spikes
    Vo, wo, refo = o.state()
    np.testing.assert_allclose(Vo, V, rtol=0, atol=1e-9)
    np.testing.assert_allclose(wo, w, rtol=0, atol=1e-12)


def test_charge_conservation(oracle_mod):
    net = W.workload("grid4_gauss")["net"]
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    pre, tgt, wq, delay = decode(net, row_ptr, bend, recs)
    rowsum = np.bincount(pre, weights=wq, minlength=W.n_neurons(net)).astype(np.int64)
    rowlen = np.diff(row_ptr.astype(np.int64))
    read = 0
    for t in range(150):
        read += int(o.ring()[t % 32].astype(np.int64).sum())
        o.step(1)
    residual = int(o.ring().astype(np.int64).sum())
    sp = o.spikes()
    sent = int(rowsum[sp[:, 1]].sum())
    assert len(sp) > 1000
    assert read + residual == sent
    assert o.stats()["rec_events"] == int(rowlen[sp[:, 1]].sum())


def test_forced_step_matches_free_run(oracle_mod):
    # feeding the free run's own spike sets back as forced sets reproduces it
    net = W.make(2, 1, W.GAUSS, 1.0, 100, 22, n_exc=160, n_inh=40)
    a = oracle_mod.Net(net).build()
    b = oracle_mod.Net(net).build()
    for t in range(200):
        a.step(1)
        sp = a.spikes()
        b.step_forced(sp[sp[:, 0] == t, 1])
    np.testing.assert_array_equal(a.spikes(), b.spikes())
    for x, y in zip(a.state(), b.state()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.ring(), b.ring())


def test_col_pending_is_the_ring_in_flight(oracle_mod):
    """col_pending (the charge in flight for one target, regenerated from the
    pair draws of a raster's recent spikers) equals what the oracle's own
    delay ring holds after the same steps, for every target and every arrival
    step ahead; the ring is pinned to the dense brute force above."""
    net = W.make(2, 1, W.EXP, 2.0, 120, 23, n_exc=160, n_inh=40, ext_rate_hz=4.0)
    o = oracle_mod.Net(net).build()
    for T in (37, 90):
        o.step(T - o.stats()["t"])
        raster = o.spikes()
        assert (raster[:, 0] >= T - net["d_max"]).sum() > 50
        ring = o.ring()
        for j in range(0, o.N, 23):
            want = np.array([ring[(T + a) % oracle_mod.RING, j] for a in range(net["d_max"])], dtype=np.int64)
            np.testing.assert_array_equal(oracle_mod.col_pending(net, j, raster, T), want, err_msg=f"target {j}")
