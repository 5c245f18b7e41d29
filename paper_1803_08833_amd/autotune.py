"""Schedule autotuners.

Single network: the candidates are the delivery schedules and their knobs
exposed by the C ABI (direct atomics vs tile-binned delivery, the per-step
binning threshold, the scatter grid, the number of steps per captured HIP
graph).  Every candidate is timed on the identical workload: the network is
reset to its initial state (snn_reset), stepped through a warm-up, then timed;
all candidates give bit-identical results (integer delivery is order-free), so
the choice affects speed only.  The winner is cached in a JSON file keyed by
the network description and applied with snn_set_option.

Batches (continuous batching of many jobs): the candidates are the steps per
batched call (the length of a captured chunk, which is also the admission
granularity), the batched scatter grid, binned vs direct delivery and the
binning threshold (snn_batch_set_option).  Each is timed on the same closed
loop, a sample of the job mix all queued at once and served to completion, so
construction overlap and admission granularity count as they do when serving;
the schedule with the highest jobs/s wins.  Rasters do not depend on it.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import snn

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "snn_mi355x_autotune.json")


def key(net: dict) -> str:
    items = sorted((k, v) for k, v in net.items() if k != "seed")
    return hashlib.sha1(json.dumps(items).encode()).hexdigest()[:16]


def candidates(stats: dict):
    """Option sets to try (list of {option: value})."""
    out = []
    auto_thr = stats["bin_threshold"]
    for chunk in (32, 64, 128):
        out.append({snn.OPT_DELIVER_MODE: 0, snn.OPT_GRAPH_CHUNK: chunk})
    binned = 1 if stats["binned_ok"] & 1 else (2 if stats["binned_ok"] & 2 else 0)
    if binned:
        for thr in (auto_thr // 2, auto_thr, auto_thr * 2):
            for blocks in (256, 512):
                out.append({snn.OPT_DELIVER_MODE: binned, snn.OPT_BIN_THRESHOLD: int(thr),
                            snn.OPT_SCATTER_BLOCKS: blocks, snn.OPT_GRAPH_CHUNK: 64})
    return out


def apply(g: "snn.Net", opts: dict):
    for k, v in opts.items():
        g.set_option(int(k), int(v))


def tune(g: "snn.Net", warmup: int = 200, steps: int = 600, cache: str | None = DEFAULT_CACHE,
         sync=None) -> dict:
    """Time every candidate on `g` (built), keep the fastest, apply it and
    return {"options": ..., "ms_per_step": ..., "trials": [...]}; the
    network is reset afterwards."""
    import torch

    sync = sync or torch.cuda.synchronize
    st = g.stats()
    trials = []
    for opts in candidates(st):
        g.reset()
        apply(g, opts)
        g.step(warmup)
        sync()
        t0 = time.perf_counter()
        g.step(steps)
        sync()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        trials.append(dict(options={str(k): v for k, v in opts.items()}, ms_per_step=ms))
    best = min(trials, key=lambda r: r["ms_per_step"])
    g.reset()
    apply(g, {int(k): v for k, v in best["options"].items()})
    result = dict(options=best["options"], ms_per_step=best["ms_per_step"], trials=trials)
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key(g.net)] = dict(options=best["options"], ms_per_step=best["ms_per_step"])
        with open(cache + ".tmp", "w") as f:
            json.dump(data, f, indent=1)
        os.replace(cache + ".tmp", cache)
    return result


def load(g: "snn.Net", cache: str = DEFAULT_CACHE) -> bool:
    """Apply a cached choice for this network description, if any."""
    if not os.path.exists(cache):
        return False
    with open(cache) as f:
        data = json.load(f)
    ent = data.get(key(g.net))
    if not ent:
        return False
    apply(g, {int(k): v for k, v in ent["options"].items()})
    return True


def batch_key(jobs) -> str:
    """Key of a job mix: its jobs' descriptions without seeds, drives and
    durations (the shapes the batched kernels see)."""
    shapes = sorted(json.dumps(sorted((k, v) for k, v in j["net"].items() if k not in ("seed", "ext_rate_hz")))
                    for j in jobs)
    return "batch-" + hashlib.sha1(json.dumps(shapes).encode()).hexdigest()[:16]


def batch_candidates():
    """Batch schedules to try: {"chunk_ms": steps per call, "options": {...}}.
    The default (50 ms chunks, 256 scatter workgroups, binned where the job
    allows it, each job's own threshold) comes first."""
    out = [dict(chunk_ms=50, options={snn.OPT_SCATTER_BLOCKS: 256, snn.OPT_DELIVER_MODE: 1,
                                      snn.OPT_BIN_THRESHOLD_PPM: 0})]
    for chunk in (25, 50, 100):
        for blocks, mode, ppm in ((256, 1, 0), (512, 1, 0), (256, 0, 0), (256, 1, 19500), (256, 1, 78000)):
            c = dict(chunk_ms=chunk, options={snn.OPT_SCATTER_BLOCKS: blocks, snn.OPT_DELIVER_MODE: mode,
                                              snn.OPT_BIN_THRESHOLD_PPM: ppm})
            if c not in out:
                out.append(c)
    return out


def tune_batch(jobs, hbm_budget: int, max_neurons: int, candidates=None, finalists: int = 3,
               cache: str | None = DEFAULT_CACHE, log=None) -> dict:
    """Serve `jobs` (all queued at once) with every candidate schedule, time
    the best `finalists` once more, and return {"schedule": fastest by mean
    jobs/s, "trials": [...]}; cached under batch_key(jobs) when cache is set."""
    import numpy as np

    from . import serve

    say = log or (lambda *a: None)
    cands = list(candidates or batch_candidates())
    arrivals = np.zeros(len(jobs))
    walls = [[] for _ in cands]

    def trial(i):
        r = serve.serve_batched(jobs, arrivals, hbm_budget, max_neurons, schedule=cands[i])
        if r["failed"]:
            raise RuntimeError(f"batch autotuner: {len(r['failed'])} jobs failed under {cands[i]}")
        walls[i].append(r["wall"])

    for i in range(len(cands)):
        trial(i)
    order = sorted(range(len(cands)), key=lambda i: walls[i][0])
    for i in order[:finalists]:
        trial(i)
    mean = [sum(w) / len(w) for w in walls]
    best = min(order[:finalists] if finalists else order, key=lambda i: mean[i])
    trials = [dict(chunk_ms=c["chunk_ms"], options={str(k): v for k, v in c["options"].items()},
                   jobs_per_s=[len(jobs) / w for w in walls[i]]) for i, c in enumerate(cands)]
    schedule = dict(chunk_ms=cands[best]["chunk_ms"], options={str(k): v for k, v in cands[best]["options"].items()})
    say(f"# batch autotuner ({len(jobs)} jobs, {len(cands)} schedules): {schedule}, "
        f"{len(jobs) / mean[best]:.2f} jobs/s (default {len(jobs) / mean[0]:.2f})")
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[batch_key(jobs)] = dict(schedule=schedule, jobs_per_s=len(jobs) / mean[best])
        with open(cache + ".tmp", "w") as f:
            json.dump(data, f, indent=1)
        os.replace(cache + ".tmp", cache)
    return dict(schedule=schedule, trials=trials)


def load_batch(jobs, cache: str = DEFAULT_CACHE):
    """The cached schedule for this job mix, or None."""
    if not os.path.exists(cache):
        return None
    with open(cache) as f:
        ent = json.load(f).get(batch_key(jobs))
    return ent["schedule"] if ent else None
