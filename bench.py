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
# Exact-time solver: per event the record (8 / 4 B), the queue entry written
# (16) and read back (16), the placed {offset, charge} pair written (8) and
# read by the update (8); per neuron and step V, w and the refractory end read
# and written (32), its input offset written (8) and read (8).  The arrival
# sort's group pass (each entry written and read once more) is not counted.
BYTES_EXACT_PER_EVENT = {0: 56, 1: 52}
BYTES_EXACT_PER_NEURON_STEP = 48


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20, help="timed seconds of biological time")
    p.add_argument("--warmup", type=int, default=5, help="untimed seconds of biological time")
    p.add_argument("--workload", default="grid24_exp")
    p.add_argument("--ext-rate", type=float, default=None, help="override external Poisson rate (Hz)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--deliver-mode", type=int, default=None, help="0 direct atomics, 1 tile-binned")
    p.add_argument("--bin-threshold", type=float, default=None,
                   help="binned steps from this many recurrent events, as a multiple of the library's default")
    p.add_argument("--serve-jobs", type=int, default=512, help="served-stream jobs (0: skip serving)")
    p.add_argument("--serve-plain", type=int, default=128, help="first jobs also served one at a time")
    p.add_argument("--serve-capacity", type=int, default=64, help="jobs of the closed-loop capacity run")
    p.add_argument("--serve-tune", type=int, default=16,
                   help="jobs the batch autotuner serves per candidate schedule (0: default schedule)")
    p.add_argument("--serve-gen", type=int, default=1,
                   help="synapse generator of the served jobs: 0 one trial per pair, 1 binomial + Floyd")
    p.add_argument("--graph-chunk", type=int, default=250,
                   help="steps per captured HIP graph (0: launch every kernel directly)")
    p.add_argument("--queue-cap", type=float, default=0.3,
                   help="exact solver: queued inputs per arrival slot, as a mean rate in kHz "
                        "times neurons times synapses per neuron")
    p.add_argument("--gen", type=int, default=None,
                   help="synapse generator of the workload: 0 one trial per pair, 1 binomial + Floyd")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="end with one plain device copy of this size (reference kernel for HBM counters)")
    return p.parse_args()


def workload(args):
    from paper_1803_08833_amd import workloads as W

    over = {}
    if args.ext_rate is not None:
        over["ext_rate_hz"] = args.ext_rate
    if args.gen is not None:
        over["gen"] = args.gen
    return W.workload(args.workload, **over)


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "snn_dev.h"):
        with open(os.path.join(ROOT, "paper_1803_08833_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_from_profile(args):
    """Per-step counter figures of the step kernels from the committed
    rocprofv3 summary of this workload (profiles/<workload>_hbm_counters.json):
    HBM bytes (FETCH_SIZE and WRITE_SIZE summed over the replayed steps'
    dispatches, each divided by the same counter's reading per byte of a plain
    device copy of known size) and atomic requests at the L2 (TCC_ATOMIC), per
    step.  None when there is no summary for this exact window (workload,
    drive, steps, warm-up) or it was taken on other kernel sources than the
    ones built now."""
    path = os.path.join(ROOT, "profiles", f"{args.workload}_hbm_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    same = (prof.get("kernel_source_sha256_16") == kernel_source_hash()
            and prof.get("ext_rate_hz") == workload(args)["net"]["ext_rate_hz"]
            and prof.get("steps") == args.steps and prof.get("warmup") == args.warmup
            and args.gen is None)
    return prof if same else None


def cpu_baseline(net, spikes_per_step, seconds_budget=12.0):
    """The FP64 oracle, built with OpenMP and run on all the host threads it
    is given, on a bounded sample of the same network: every neuron of the
    full grid is updated each step, and each step delivers the projections of
    `spikes_per_step` spikers (the timed run's mean; rows built beforehand by
    the oracle, three disjoint groups in rotation so that no forced spiker is
    refractory).  Value = recurrent events delivered / oracle wall time."""
    import multiprocessing as mp

    import numpy as np

    import oracle

    N = net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])
    D = net["d_max"] - net["d_min"] + 1
    group = int(max(1, min(spikes_per_step, 8000)))
    # 3 * group consecutive rows starting at a module boundary, built by the
    # oracle in contiguous slices on the host cores (not timed)
    M = net["n_exc"] + net["n_inh"]
    r0 = (N // 2) // M * M
    rows = np.arange(r0, r0 + 3 * group, dtype=np.int64)
    workers = min(16, os.cpu_count() or 1)
    cuts = np.linspace(0, rows.size, 4 * workers + 1).astype(np.int64)
    jobs = [(net, int(rows[a]), int(b - a)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with mp.get_context("fork").Pool(workers) as pool:
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
    groups = [rows[g::3] for g in range(3)]
    with oracle.library(oracle.build(openmp=True)):
        threads = int(oracle.lib().or_threads())
        o = oracle.Net(net)
        o.set_csr(row_ptr, bend, np.concatenate(tg), np.concatenate(dl), np.concatenate(wq))
        t0 = time.perf_counter()
        steps = 0
        ev0 = o.stats()["rec_events"]
        while True:
            o.step_forced(groups[steps % 3].astype(np.uint32))
            steps += 1
            el = time.perf_counter() - t0
            if el > seconds_budget or steps >= 2000:
                break
        events = o.stats()["rec_events"] - ev0
        del o
    return dict(value=events / el, unit="synaptic events/s", cores=threads, kind="oracle",
                sample=(f"FP64 oracle (OpenMP build, {threads} threads; host nproc {os.cpu_count()}), "
                        f"{net['gx']}x{net['gy']} grid ({N} neurons), {steps} forced 1 ms steps: all neurons "
                        f"updated each step, {group} spikers delivered per step (the timed run's mean, "
                        f"{events // max(1, steps)} events per step; oracle-built projection rows)"),
                ms_per_step=1e3 * el / steps, sim_s_per_wall_s=steps * 1e-3 / el, nproc=os.cpu_count())


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on exactly one GPU: the simulator has no multi-GPU "
                                   "path (a network runs on one device)", "n_gpus": args.gpus}))
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
    exact = net.get("solver", 0) == snn.SOLVER_EXACT
    if exact:
        g.set_option(snn.OPT_QUEUE_CAP, int(N * (net["k_in"] + 1) * args.queue_cap))
    tb = time.perf_counter()
    g.build_synapses()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    if args.deliver_mode is not None and not exact:
        g.set_option(snn.OPT_DELIVER_MODE, args.deliver_mode)
    if args.bin_threshold is not None and not exact:
        g.set_option(snn.OPT_BIN_THRESHOLD, int(args.bin_threshold * g.stats()["bin_threshold"]))
    g.set_option(snn.OPT_GRAPH_CHUNK, args.graph_chunk)   # default: a bench step (1000 ms) is four graphs
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

    # Kernel roofline: the timed region is replayed from the same initial state
    # (reset, same warm-up) with every launch stamped by its own HIP events;
    # the network is deterministic, so the replay delivers exactly the timed
    # region's events with the same kernels, and per-launch durations are free
    # of host gaps.
    g.reset()
    for _ in range(args.warmup):
        g.step(1000)
    kt = g.time_kernels(1000 * args.steps)
    stf = g.stats()
    replay_ok = kt["rec_events"] == rec and kt["spikes"] == spikes
    steps_k = max(1, kt["steps"])
    bpe = BYTES_PER_EVENT[net["record"]]
    bpn = BYTES_PER_NEURON_STEP
    ev_per_step = kt["rec_events"] / steps_k
    if exact:
        # one step: arrival sort (k_xs_*), k_x_update(_busy), k_x_list, k_x_offsets, k_x_deliver, k_x_finish
        name = ("k_xs_*+k_x_update+k_x_offsets+k_x_deliver and the rest of one 1 ms step of the "
                "exact-time solver")
        ms = kt["step_ms"]
        bpe, bpn = BYTES_EXACT_PER_EVENT[net["record"]], BYTES_EXACT_PER_NEURON_STEP
    elif stf["deliver_mode"] == 1:
        # one step = k_scatter (compaction + delivery phase A) + k_tile (phase B
        # + the next step's neuron update)
        name = "k_scatter+k_tile (one 1 ms step: compaction, delivery, fused neuron update)"
        ms = kt["scatter_ms"] + kt["tile_ms"]
    elif stf["deliver_mode"] == 2:
        name = ("k_compact+k_seg_emit+k_seg_bin+k_tile (one 1 ms step: compaction, two-level binned "
                "delivery, fused neuron update)")
        ms = kt["compact_ms"] + kt["scatter_ms"] + kt["sub_ms"] + kt["tile_ms"]
    else:
        name = "k_update+k_compact+k_deliver (one 1 ms step, direct atomics)"
        ms = kt["update_ms"] + kt["compact_ms"] + kt["deliver_ms"]
    step_bytes = ev_per_step * bpe + N * bpn
    achieved = step_bytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    prof = None if exact else counters_from_profile(args)
    # scattered int32 atomic adds per second on this GPU (the unit of direct
    # delivery), from the library's own probe: the peak atomics are read against
    atomic_peak = snn.probe_atomics(1 << 26, 1 << 28, stream)
    atomics = {"probe_peak_per_s": atomic_peak,
               "requests_per_step": prof.get("atomic_requests_per_step") if prof else None,
               "achieved_per_s": (prof["atomic_requests_per_step"] / (ms * 1e-3)
                                  if prof and prof.get("atomic_requests_per_step") and ms > 0 else None)}
    roofline = {"bound": "hbm", "kernel": name,
                "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": prof.get("hbm_bytes_per_step") if prof else None,
                "atomics": atomics,
                "bytes_per_launch": round(step_bytes, 1), "avg_launch_ms": round(ms, 6),
                "events_per_launch": round(ev_per_step, 1),
                "bytes_per_event": bpe, "bytes_per_neuron_step": bpn,
                "launches_timed": kt["steps"], "replay_identical": bool(replay_ok)}
    result = {
        "metric": "synaptic events/s + sim-s per wall-s, 24x24 exp grid; served-job p50/p99",
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
        "solver": "exact-time event-driven" if exact else "1 ms step",
        # two-level networks: the scatter slot is k_seg_emit, the second pass k_seg_bin
        "kernels_avg_ms": {"k_update": round(kt["update_ms"], 6), "k_compact": round(kt["compact_ms"], 6),
                           "k_scatter": round(kt["scatter_ms"], 6), "k_sub": round(kt["sub_ms"], 6),
                           "k_tile": round(kt["tile_ms"], 6),
                           "deliver": round(kt["deliver_ms"], 6), "kernels_per_step": round(kt["step_ms"], 6)},
        "deliver_mode": stf["deliver_mode"],
        "bin_overflow_events": stf["bin_overflow"],
        "roofline": roofline,
        "served": None,
        "cpu_baseline": None,
    }
    g.close()
    if args.serve_jobs:
        from paper_1803_08833_amd import serve

        say = lambda *a: print(*a, file=sys.stderr, flush=True)
        result["served"] = serve.bench_served(args.serve_jobs, args.serve_plain, args.serve_capacity, log=say,
                                              gen=args.serve_gen, tune_jobs=args.serve_tune)
        result["served"]["generator"] = "binomial + Floyd" if args.serve_gen else "one trial per pair"
    if not args.no_cpu_baseline and not exact:
        sps = spikes / max(1, args.steps * 1000)
        result["cpu_baseline"] = cpu_baseline(net, max(1, int(round(sps))))
    if args.copy_mib:
        n = args.copy_mib << 18
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    print(json.dumps(result), flush=True)
    if result["served"] and result["served"]["failed"]:
        print(f"# {result['served']['failed']} served jobs failed", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
