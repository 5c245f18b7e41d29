"""Schedule autotuner for the single-network path.

Candidates are the delivery schedules and their knobs exposed by the C ABI
(direct atomics vs tile-binned delivery, the per-step binning threshold, the
scatter grid, the number of steps per captured HIP graph).  Every candidate is
timed on the identical workload: the network is reset to its initial state
(snn_reset), stepped through a warm-up, then timed; all candidates give
bit-identical results (integer delivery is order-free), so the choice affects
speed only.  The winner is cached in a JSON file keyed by the network
description and applied with snn_set_option.
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
    if stats["binned_ok"]:
        for thr in (auto_thr // 2, auto_thr, auto_thr * 2):
            for blocks in (256, 512):
                out.append({snn.OPT_DELIVER_MODE: 1, snn.OPT_BIN_THRESHOLD: int(thr),
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
