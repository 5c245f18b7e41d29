"""Benchmark: synaptic events/s and simulated seconds per wall second of the
24x24-module exponential-connectivity network (lambda 5 modules, 1100
synapses/neuron, 714,240 neurons, ~786 M synapses) on one MI355X.

One benchmark step = one second of biological time = 1000 steps of 1 ms
through the whole hot path (fused neuron update, ordered spike compaction,
fan-out delivery into the delay ring).  The network is built on the device
first (construction time reported separately), so inputs are resident in HBM
when timing starts.

Printed: one JSON line with the headline value, the roofline of the dominant
kernel (algorithmic bytes per launch over its HIP-event-timed duration) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E peak
BYTES_PER_EVENT = {0: 16, 1: 12}      # record + ring slot read + write (F32 / 8-bit code records)
BYTES_PER_NEURON_STEP = 26            # V 4+4, w 4+4, ref 1+1, ring slot 4+4


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10, help="timed seconds of biological time")
    p.add_argument("--warmup", type=int, default=1, help="untimed seconds of biological time")
    p.add_argument("--workload", default="grid24_exp")
    p.add_argument("--ext-rate", type=float, default=None, help="override external Poisson rate (Hz)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--kernel-steps", type=int, default=200, help="steps timed per kernel with HIP events")
    p.add_argument("--deliver-mode", type=int, default=None, help="0 direct atomics, 1 tile-binned")
    return p.parse_args()


def workload(args):
    from paper_1803_08833_amd import workloads as W

    over = {}
    if args.ext_rate is not None:
        over["ext_rate_hz"] = args.ext_rate
    return W.workload(args.workload, **over)


def cpu_baseline(net, spikes_per_step, seconds_budget=12.0):
    """The FP64 oracle on a bounded sample of the same network: every neuron
    of the full grid is updated each step, and each step delivers the
    projections of `spikes_per_step` spikers (rows built beforehand by the
    oracle, three disjoint groups in rotation so that no forced spiker is
    refractory).  Value = recurrent events delivered / oracle wall time."""
    import multiprocessing as mp

    import numpy as np

    import oracle

    N = net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])
    D = net["d_max"] - net["d_min"] + 1
    group = int(max(1, min(spikes_per_step, 1000)))
    # 3 * group consecutive rows starting at a module boundary, built by the
    # oracle in contiguous slices on the host cores (not timed)
    M = net["n_exc"] + net["n_inh"]
    r0 = (N // 2) // M * M
    rows = np.arange(r0, r0 + 3 * group, dtype=np.int64)
    workers = min(16, os.cpu_count() or 1)
    cuts = np.linspace(0, rows.size, workers + 1).astype(np.int64)
    jobs = [(net, int(rows[a]), int(b - a)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        parts = pool.starmap(oracle.build_rows, jobs)
    lens = np.zeros(N, dtype=np.int64)
    bend = np.zeros((N, D), dtype=np.uint16)
    tg, dl, wq = [], [], []
    for (_, p0, cnt), (rl, be, rc) in zip(jobs, parts):
        lens[p0:p0 + cnt] = rl.astype(np.int64)
        bend[p0:p0 + cnt] = be
        rec = rc.view(np.uint32).reshape(-1, 2)
        tg.append(rec[:, 0])
        wq.append(np.rint(rec[:, 1].view(np.float32).astype(np.float64) * 65536).astype(np.int32))
        for r in range(cnt):
            k = np.arange(int(rl[r]))
            dl.append((net["d_min"] + (be[r].astype(np.int64)[None, :] <= k[:, None]).sum(axis=1)).astype(np.uint32))
    row_ptr = np.zeros(N + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(lens)
    o = oracle.Net(net)
    o.set_csr(row_ptr, bend, np.concatenate(tg), np.concatenate(dl), np.concatenate(wq))
    groups = [rows[g::3] for g in range(3)]
    t0 = time.perf_counter()
    steps = 0
    ev0 = o.stats()["rec_events"]
    while True:
        o.step_forced(groups[steps % 3].astype(np.uint32))
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_budget or steps >= 400:
            break
    events = o.stats()["rec_events"] - ev0
    return dict(value=events / el, unit="synaptic events/s", cores=1, kind="oracle",
                sample=(f"FP64 oracle, {net['gx']}x{net['gy']} grid ({N} neurons), {steps} forced 1 ms steps: "
                        f"all neurons updated each step, {group} spikers delivered per step "
                        f"(oracle-built projection rows), single thread"),
                ms_per_step=1e3 * el / steps, sim_s_per_wall_s=steps * 1e-3 / el)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU scaling is not "
                                   "implemented (see the sharding design note)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_1803_08833_amd import snn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = workload(args)
    net = wl["net"]
    stream = snn.current_stream_handle()
    N = net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])
    hist_cap = int(min(2**27, N * 60 * (args.steps + args.warmup) + (1 << 22)))
    g = snn.Net(net, hist_cap=hist_cap, stream=stream)
    tb = time.perf_counter()
    g.build_synapses()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    if args.deliver_mode is not None:
        g.set_option(snn.OPT_DELIVER_MODE, args.deliver_mode)
    st0 = g.stats()
    print(f"# built {args.workload}: {N} neurons, {st0['nnz']} synapses in {build_s:.2f} s", file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        g.step(1000)
    torch.cuda.synchronize()
    s0 = g.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g.step(1000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = g.stats()
    rec = s1["rec_events"] - s0["rec_events"]
    ext = s1["ext_events"] - s0["ext_events"]
    spikes = s1["spikes"] - s0["spikes"]
    sim_s = args.steps * 1.0
    rate_hz = spikes / N / sim_s if sim_s else 0.0
    print(f"# timed {args.steps} s bio in {wall:.3f} s wall, rate {rate_hz:.2f} Hz, {rec} events",
          file=sys.stderr, flush=True)

    kt = g.time_kernels(args.kernel_steps)
    stf = g.stats()
    per_launch_events = kt["rec_events"] / max(1, kt["steps"])
    bpe = BYTES_PER_EVENT[net["record"]]
    deliver_bytes = per_launch_events * bpe
    update_bytes = N * BYTES_PER_NEURON_STEP
    kern = {
        "update": dict(ms=kt["update_ms"], bytes=update_bytes),
        "compact": dict(ms=kt["compact_ms"], bytes=None),
        "deliver": dict(ms=kt["deliver_ms"], bytes=deliver_bytes),
    }
    dom = "deliver" if kt["deliver_ms"] >= kt["update_ms"] else "update"
    dom_bytes = kern[dom]["bytes"]
    achieved = dom_bytes / (kern[dom]["ms"] * 1e-3) / 1e9 if kern[dom]["ms"] > 0 else 0.0
    mode = "tile-binned (k_scatter + k_tile)" if stf["deliver_mode"] == 1 else "direct atomics (k_deliver)"
    roofline = {"bound": "hbm", "kernel": dom if dom == "update" else f"deliver: {mode}",
                "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": round(dom_bytes, 1), "avg_launch_ms": round(kern[dom]["ms"], 5),
                "events_per_launch": round(per_launch_events, 1)}
    result = {
        "metric": "synaptic events/s (24x24 exp grid)",
        "value": rec / wall,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 state, int32 fixed-point delivery",
        "data": "synthetic (seeded Philox network, Poisson drive)",
        "config": {"workload": f"{args.workload}: {net['gx']}x{net['gy']} modules, "
                               f"{'exponential lambda' if net['kernel'] == 1 else 'Gaussian sigma'} "
                               f"{net['range']} modules, {int(net['k_in'])} synapses/neuron, "
                               f"{N} neurons, 1 bench step = 1 s biological time",
                   "neurons": N, "synapses": st0["nnz"], "ext_rate_hz": net["ext_rate_hz"],
                   "parallelism": "single GPU"},
        "sim_s_per_wall_s": sim_s / wall,
        "total_equiv_events_per_s": (rec + ext) / wall,
        "mean_rate_hz": rate_hz,
        "build_s": build_s,
        "kernels_ms": {"update": round(kt["update_ms"], 5), "compact": round(kt["compact_ms"], 5),
                       "deliver": round(kt["deliver_ms"], 5), "scatter": round(kt["scatter_ms"], 5),
                       "tile": round(kt["tile_ms"], 5)},
        "deliver_mode": stf["deliver_mode"],
        "bin_overflow_events": stf["bin_overflow"],
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        sps = spikes / max(1, args.steps * 1000)
        result["cpu_baseline"] = cpu_baseline(net, max(1, int(round(sps))))
    g.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
