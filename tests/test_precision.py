"""Precision statement of the compressed synapse records (8-bit weight codes),
made entirely with the FP64 oracle: the same network is simulated with
  (a) the 255-bin codebook weights (what the 8-bit records deliver exactly),
  (b) the 65536-bin weight table (F32 records),
  (c) the uncompressed FP64 weights mu + sd * Phi^-1((u + 1/2) / 2^32) of the
      same draws.
It reports the firing-rate differences and, with (c) forced onto (a)'s spike
raster, the membrane-potential differences caused by weight quantisation
alone.  The figures are stated, not bounded; the loose assertions only catch
a broken comparison.
"""
import json
import os

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

STEPS = 600


def _net(record):
    return W.make(2, 1, W.EXP, 2.0, 600, 41, record=record, ext_rate_hz=2.5)


def _run(oracle_mod, net, fp64):
    o = oracle_mod.Net(net, fp64_weights=fp64).build()
    o.step(STEPS)
    return o


@pytest.mark.slow
def test_code8_precision_statement(oracle_mod):
    code = _run(oracle_mod, _net(W.REC_CODE8), False)
    f32 = _run(oracle_mod, _net(W.REC_F32), False)
    exact = _run(oracle_mod, _net(W.REC_CODE8), True)
    N = code.N
    r = {name: o.stats()["spikes"] / N / (STEPS * 1e-3) for name, o in
         (("code8", code), ("f32", f32), ("fp64", exact))}
    # membrane error from weight quantisation alone: the uncompressed network
    # is forced onto the 8-bit-code network's spike raster
    forced = oracle_mod.Net(_net(W.REC_CODE8), fp64_weights=True).build()
    ref = oracle_mod.Net(_net(W.REC_CODE8), fp64_weights=False).build()
    dv_max, dv_sq, cnt = 0.0, 0.0, 0
    for t in range(STEPS):
        ref.step(1)
        sp = ref.spikes()
        forced.step_forced(sp[sp[:, 0] == t, 1])
        Va, _, ra = ref.state()
        Vb, _, rb = forced.state()
        live = (ra == 0) & (rb == 0)
        d = np.abs(Va - Vb)[live]
        dv_max = max(dv_max, float(d.max(initial=0.0)))
        dv_sq += float((d**2).sum())
        cnt += int(d.size)
    stmt = dict(
        network="2x1 modules of 992+248 neurons, exponential lambda 2, k_in 600, 2.5 Hz drive, 600 ms",
        rate_hz=r,
        rate_rel_err_code8_vs_fp64=(r["code8"] - r["fp64"]) / r["fp64"],
        rate_rel_err_f32_vs_fp64=(r["f32"] - r["fp64"]) / r["fp64"],
        vm_err_code8_vs_fp64_mV=dict(max=dv_max, rms=(dv_sq / max(cnt, 1)) ** 0.5),
    )
    print("PRECISION", json.dumps(stmt), flush=True)
    assert r["fp64"] > 0
    assert abs(stmt["rate_rel_err_code8_vs_fp64"]) < 0.5
    assert stmt["vm_err_code8_vs_fp64_mV"]["rms"] < 1.0
