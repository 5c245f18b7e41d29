"""GPU parity of the exact-time event-driven solver (Sec. II.A, Sec. II.C)
against the oracle, through the C ABI.

* Lock-step: the oracle runs free and its spikes, with their offsets, are
  forced on the GPU each step.  After every step the spike history (step,
  id, offset) and every queued input (target, offset, charge, for each
  arrival step ahead) must be bit-exact, the state within the R13
  tolerance, the refractory steps exact and the counters equal.  Several
  256-neuron workgroups and a ragged tail; F32 and 8-bit-code records;
  Poisson and constant drive; a strong drive that sends neurons more inputs
  in one step than the LDS sort holds (16; the slow path).
* Free run at the full 24x24 exponential size: every sampled spike happens
  at the exact time of one of its neuron's inputs (an external input, or a
  presynaptic spike plus the synapse's delay), no neuron fires twice within
  t_ref, and nothing overflows.
* Errors: the calls of one solver refuse the other's networks.
"""
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


def _compare_state(net, gs, os_, t):
    """R13: V within 1e-5 of max(|V|, V_th - E), w within 1e-5 of max(|w|, alpha)."""
    Vg, Wg, Rg = gs
    Vo, Wo, Ro = os_
    tolV = 1e-5 * np.maximum(np.abs(Vo), net["v_th"] - net["e_rest"])
    dv = np.abs(Vg.astype(np.float64) - Vo)
    assert np.all(dv <= tolV), f"step {t}: V error {dv.max()} at {dv.argmax()} (V={Vo[dv.argmax()]})"
    tolw = 1e-5 * np.maximum(np.abs(Wo), net["alpha_w"])
    dw = np.abs(Wg.astype(np.float64) - Wo)
    assert np.all(dw <= tolw), f"step {t}: w error {dw.max()}"
    np.testing.assert_array_equal(Rg.astype(np.int32), Ro)


def _lockstep(snn, oracle_mod, net, steps, check_every=1, qcap=0):
    o = oracle_mod.Net(net).build()
    R = net["d_max"] + 1
    big = 0
    with snn.Net(net) as g:
        g.set_option(snn.OPT_QUEUE_CAP, qcap)
        g.build_synapses()
        _compare_state(net, g.read_state(), o.state(), -1)
        for t in range(steps):
            o.step(1)
            sp, fr = o.spikes(), o.spike_fracs()
            now = sp[:, 0] == t
            g.step_forced_exact(sp[now, 1], fr[now])
            if t % check_every and t != steps - 1:
                continue
            gsp, gfr = g.read_spike_times()
            np.testing.assert_array_equal(gsp, sp, err_msg=f"spikes after step {t}")
            np.testing.assert_array_equal(gfr, fr, err_msg=f"offsets after step {t}")
            for k in range(R):
                q = o.queue((t + 1 + k) % oracle_mod.RING)
                np.testing.assert_array_equal(g.read_queue(k), q, err_msg=f"queue {k} ahead after step {t}")
                if len(q):
                    big = max(big, int(np.bincount(q[:, 0]).max()))
            _compare_state(net, g.read_state(), o.state(), t)
        st, ost = g.stats(), o.stats()
        for key in ("spikes", "rec_events", "ext_events"):
            assert st[key] == ost[key], key
        assert st["t"] == steps
        return st, len(sp), big


@pytest.mark.parametrize("record,drive", [(W.REC_F32, "poisson"), (W.REC_CODE8, "poisson"),
                                          (W.REC_F32, "const"), (W.REC_CODE8, "poisson-expdelay")])
def test_lockstep_exact(snn, oracle_mod, record, drive):
    over = dict(n_exc=200, n_inh=52, record=record, solver=W.SOLVER_EXACT)
    if drive == "const":
        over.update(ext_mode=W.EXT_CONST, ext_const_q=round(1.3 * 65536))
    if drive == "poisson-expdelay":
        over.update(delay_dist=W.DELAY_EXP, delay_tau=4.0)
    net = W.make(3, 2, W.EXP, 2.0, 150, 61, **over)   # 1512 neurons: 5 full workgroups + a ragged one
    say(f"case: exact lock-step, record {record}, drive {drive}, N {W.n_neurons(net)}")
    st, nsp, _ = _lockstep(snn, oracle_mod, net, 120)
    assert nsp > 100
    assert st["disagree"] <= max(2, nsp // 1000)


def test_lockstep_exact_many_inputs(snn, oracle_mod):
    """Strong drive and in-degree: some neurons take more inputs in a step
    than the LDS sort holds (16), up to 40 and more, which the slow path orders."""
    net = W.make(2, 2, W.GAUSS, 1.5, 400, 67, n_exc=160, n_inh=40, solver=W.SOLVER_EXACT, d_max=4,
                 ext_rate_hz=12.0, w_inh=-0.4)
    say(f"case: exact lock-step, many inputs per step, N {W.n_neurons(net)}")
    st, nsp, big = _lockstep(snn, oracle_mod, net, 60, check_every=3, qcap=1 << 20)
    assert big > 40, big
    assert st["disagree"] <= max(2, nsp // 1000)


@pytest.mark.parametrize("case", ["upto512", "past1024"])
def test_lockstep_exact_busy_sorted_by_waves(snn, oracle_mod, case):
    """A 12 Hz drive bursts the network within a few steps, so that every
    update workgroup is busy and its neurons' slices, at hundreds of distinct
    offsets with ties, span each width the busy kernel's waves sort together
    (2-64 ... 513-1024 inputs) and, past 1024, the single-lane heap sort, with
    hundreds of thousands of inputs per workgroup.  Lock-step against the
    oracle's free run."""
    if case == "upto512":
        net = W.make(2, 1, W.GAUSS, 1.0, 1100, 71, n_exc=960, n_inh=240, solver=W.SOLVER_EXACT, d_max=2,
                     ext_rate_hz=12.0)
        steps, want = 8, 256
    else:
        net = W.make(2, 1, W.GAUSS, 1.0, 2200, 71, n_exc=1920, n_inh=480, solver=W.SOLVER_EXACT, d_max=1,
                     ext_rate_hz=12.0)
        steps, want = 6, 1024
    say(f"case: exact lock-step, busy workgroups sorted by waves ({case}), N {W.n_neurons(net)}")
    st, nsp, big = _lockstep(snn, oracle_mod, net, steps, qcap=1 << 23)
    assert big > want, big
    assert st["disagree"] <= max(2, nsp // 1000)


def test_graph_replay_equals_single_launches(snn):
    """Free runs stepped through captured R-step graphs (from any phase) and
    launched step by step give bitwise identical rasters, offsets and state."""
    net = W.make(3, 2, W.EXP, 2.0, 150, 71, n_exc=200, n_inh=52, solver=W.SOLVER_EXACT)
    say("case: exact solver, graph replay vs single launches")
    out = []
    for chunk, calls in ((0, (100, 57)), (64, (5, 95, 3, 54))):
        with snn.Net(net) as g:
            g.build_synapses()
            g.set_option(snn.OPT_GRAPH_CHUNK, chunk)
            for c in calls:
                g.step(c)
            out.append((g.read_spike_times(), g.read_state(), g.stats()))
    (s0, f0), st0, a = out[0]
    (s1, f1), st1, b = out[1]
    assert len(s0) > 100 and a["t"] == b["t"] == 157
    np.testing.assert_array_equal(s0, s1)
    np.testing.assert_array_equal(f0, f1)
    for x, y in zip(st0, st1):
        np.testing.assert_array_equal(x, y)
    assert a["rec_events"] == b["rec_events"] and a["ext_events"] == b["ext_events"]


def test_drive_change_equals_fresh_network(snn):
    """A run-time change of the external rate (SNN_OPT_EXT_RATE_UHZ) under the
    exact solver gives the raster of a network built at the new rate."""
    net = W.make(3, 2, W.EXP, 2.0, 150, 73, n_exc=200, n_inh=52, solver=W.SOLVER_EXACT, ext_rate_hz=3.0)
    say("case: exact solver, run-time drive change vs fresh network")
    out = []
    with snn.Net(net) as g:
        g.build_synapses()
        g.set_option(snn.OPT_EXT_RATE_UHZ, 6_000_000)
        g.step(100)
        out.append(g.read_spike_times())
    with snn.Net(dict(net, ext_rate_hz=6.0)) as g:
        g.build_synapses()
        g.step(100)
        out.append(g.read_spike_times())
    assert len(out[0][0]) > 100
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def _ext_offsets(oracle_mod, net, poisc, g, t):
    key = [net["seed"] & 0xFFFFFFFF, net["seed"] >> 32]
    u = int(oracle_mod.philox([g >> 2, t, 3, 0], key)[g & 3])
    c = int(np.sum(poisc.astype(np.int64) <= u))
    return {int(oracle_mod.philox([g, t, 7, k >> 2], key)[k & 3]) for k in range(c)}


def test_full_size_free_run_causality(snn, oracle_mod):
    net = dict(W.workload("grid24_exp")["net"], solver=W.SOLVER_EXACT, ext_rate_hz=3.0)
    N = W.n_neurons(net)
    D = net["d_max"] - net["d_min"] + 1
    say(f"case: exact solver free run, 24x24 exponential, N {N}")
    steps = 60
    with snn.Net(net) as g:
        # the first steps are a synchronous transient: room for a 300 Hz mean rate
        g.set_option(snn.OPT_QUEUE_CAP, int(N * 1101 * 0.3))
        g.build_synapses()
        g.step(steps)
        sp, fr = g.read_spike_times()
        st = g.stats()   # raises on an overflowing queue or history
        say(f"spikes {st['spikes']} ({st['spikes'] / N / steps * 1e3:.1f} Hz), events {st['rec_events']}, "
            f"device memory {st['bytes_device'] / 2**30:.1f} GiB")
        assert st["t"] == steps and st["spikes"] == len(sp) > 1000
        assert np.all(np.diff(sp[:, 0].astype(np.int64)) >= 0)
        # refractoriness: consecutive spikes of a neuron at least t_ref apart
        T = (sp[:, 0].astype(np.int64) << 32) | fr.astype(np.int64)
        order = np.lexsort((T, sp[:, 1]))
        same = sp[order[1:], 1] == sp[order[:-1], 1]
        gaps = T[order[1:]] - T[order[:-1]]
        assert np.all(gaps[same] >= round(net["t_ref"] * 2**32))
        # causality of a sample of spikes
        poisc = oracle_mod.tables(net)["poisc"]
        spiked = {}
        for (t, gid), f in zip(sp, fr):
            spiked.setdefault((int(t), int(f)), set()).add(int(gid))
        rng = np.random.default_rng(5)
        sample = rng.choice(len(sp), size=min(300, len(sp)), replace=False)
        ext_caused = rec_caused = 0
        for i in sample:
            t, gid, f = int(sp[i, 0]), int(sp[i, 1]), int(fr[i])
            if f in _ext_offsets(oracle_mod, net, poisc, gid, t):
                ext_caused += 1
                continue
            # a presynaptic spike at (t - d, f) with a synapse pre -> gid of delay d
            found = False
            for d in range(net["d_min"], net["d_max"] + 1):
                for pre in spiked.get((t - d, f), ()):
                    row_len, bend, recs = g.export_rows(pre, 1)
                    b = bend[0]
                    lo = 0 if d == net["d_min"] else int(b[d - net["d_min"] - 1])
                    hi = int(b[d - net["d_min"]])
                    tg = recs.view(np.uint32).reshape(-1, 2)[lo:hi, 0]
                    if gid in set(tg.tolist()):
                        found = True
                        break
                if found:
                    break
            assert found, (t, gid, f)
            rec_caused += 1
        assert ext_caused > 0 and rec_caused > 0


def test_solver_specific_calls(snn):
    step_net = W.make(2, 1, W.EXP, 2.0, 60, 3, n_exc=80, n_inh=20)
    exact_net = dict(step_net, solver=W.SOLVER_EXACT)
    with snn.Net(step_net) as g:
        g.build_synapses()
        for call in (lambda: g.step_forced_exact([0], [0]), lambda: g.read_spike_times(), lambda: g.read_queue(0)):
            with pytest.raises(snn.SNNError) as e:
                call()
            assert e.value.status == snn.SNN_E_STATE
    with snn.Net(exact_net) as g:
        g.build_synapses()
        with pytest.raises(snn.SNNError) as e:
            g.step_forced([0])
        assert e.value.status == snn.SNN_E_STATE
        with pytest.raises(snn.SNNError):
            g.read_queue(exact_net["d_max"] + 1)
        with pytest.raises(snn.SNNError):
            g.step_forced_exact([0, 0], [1, 2])
        g.step(5)
        g.reset()
        assert g.stats()["t"] == 0 and len(g.read_spikes()) == 0
        for k in range(exact_net["d_max"] + 1):
            assert len(g.read_queue(k)) == 0
    # a queue too small for the traffic: inputs are dropped and reported
    with snn.Net(dict(exact_net, ext_rate_hz=12.0)) as g:
        g.set_option(snn.OPT_QUEUE_CAP, 64)
        g.build_synapses()
        g.step(30)
        with pytest.raises(snn.SNNError) as e:
            g.stats()
        assert e.value.status == snn.SNN_E_OVERFLOW
    with snn.Net(dict(exact_net, t_ref=0.5)) as g:
        with pytest.raises(snn.SNNError) as e:
            g.build_synapses()
        assert e.value.status == snn.SNN_E_INVAL
    with snn.Batch(1 << 30, 1 << 16) as b:
        with pytest.raises(snn.SNNError):
            b.admit(exact_net, 10)


def test_busy_workgroups_with_many_inputs(snn, oracle_mod):
    """Workgroups with far more queued inputs in one step than LDS holds
    (over 30,720): a 1000-neuron module with 300 synapses per neuron, all of
    delay 1, where every neuron is forced to fire in step 0 (at its
    constant-drive input, offset 0), so that each 256-neuron workgroup
    receives ~77 K inputs in step 1, all at one instant; then some neurons
    fire again.  Lock-step against the oracle: history with offsets, every queued
    input and the state after each step."""
    net = W.make(1, 1, W.GAUSS, 1.0, 300, 77, n_exc=800, n_inh=200, d_min=1, d_max=1, t_ref=1.0,
                 solver=W.SOLVER_EXACT, ext_mode=W.EXT_CONST, ext_const_q=round(0.3 * 65536))
    say("case: exact solver, workgroups with more inputs than one LDS window")
    o = oracle_mod.Net(net).build()
    rng = np.random.default_rng(5)
    R = net["d_max"] + 1
    with snn.Net(net) as g:
        g.set_option(snn.OPT_QUEUE_CAP, 1 << 19)   # a step's 300 K inputs in one arrival slot
        g.build_synapses()
        for t in range(6):
            if t == 0:
                gids = np.arange(o.N, dtype=np.uint32)
            elif t == 3:
                gids = np.sort(rng.choice(o.N, 700, replace=False)).astype(np.uint32)
            else:
                gids = np.zeros(0, dtype=np.uint32)
            fr = np.zeros(gids.size, dtype=np.uint32)   # the instant of the constant drive
            o.step_forced_exact(gids, fr)
            g.step_forced_exact(gids, fr)
            gsp, gfr = g.read_spike_times()
            np.testing.assert_array_equal(gsp, o.spikes(), err_msg=f"spikes after step {t}")
            np.testing.assert_array_equal(gfr, o.spike_fracs(), err_msg=f"offsets after step {t}")
            for k in range(R):
                q = o.queue((t + 1 + k) % oracle_mod.RING)
                np.testing.assert_array_equal(g.read_queue(k), q, err_msg=f"queue {k} ahead after step {t}")
                if t in (0, 3) and k == 0:
                    per_wg = np.bincount(q[:, 0] // 256)
                    say(f"  step {t}: inputs per workgroup next step {per_wg.tolist()}")
                    if t == 0:
                        assert per_wg.max() > 2 * 15 * 1024
            _compare_state(net, g.read_state(), o.state(), t)
