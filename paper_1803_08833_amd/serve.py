"""Serving of simulation jobs on one GPU: a request loop with continuous
batching (jobs are admitted into the running batch as slots and HBM free up,
and their steps overlap with the jobs already running), and the plain
one-job-at-a-time server it is compared with.  Latency of a job = time from
its arrival to its spike raster being readable on the host."""
from __future__ import annotations

import time

import numpy as np

from . import snn


class Result(dict):
    pass


def serve_batched(jobs, arrivals, hbm_budget=96 << 30, max_neurons=4 << 20, chunk_ms=50,
                  keep_spikes=False, clock=time.perf_counter, schedule=None):
    """Continuous batching.  jobs: list of {"net": desc, "steps": duration};
    arrivals: seconds after start (sorted).  schedule: a batch schedule
    {"chunk_ms": steps per batched call, "options": {option: value}} (the
    batch autotuner's choice), which replaces chunk_ms.  Returns per-job
    latency and events, wall time, and the rasters when keep_spikes."""
    if schedule:
        chunk_ms = int(schedule["chunk_ms"])
    n = len(jobs)
    lat = np.full(n, np.nan)
    events = np.zeros(n, dtype=np.int64)
    rasters = [None] * n
    slot_job = {}
    failed = []
    nxt = 0
    queue = []
    t0 = clock()
    with snn.Batch(hbm_budget, max_neurons, stream=snn.current_stream_handle()) as b:
        for opt, v in ((schedule or {}).get("options") or {}).items():
            b.set_option(int(opt), int(v))
        done_count = 0
        while done_count < n:
            now = clock() - t0
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            # the next chunk of the running jobs goes out first, so that the
            # admissions' synapse construction overlaps with it on the GPU
            stepped = bool(slot_job)
            if stepped:
                b.step(chunk_ms)
            while queue:
                j = queue[0]
                try:
                    slot = b.admit(jobs[j]["net"], jobs[j]["steps"])
                except snn.SNNError as e:   # can never be admitted: fails, the queue moves on
                    failed.append((j, str(e)))
                    queue.pop(0)
                    done_count += 1
                    continue
                if slot is None:            # no room now: wait for running jobs to finish
                    break
                slot_job[slot] = j
                queue.pop(0)
            if not stepped:
                if not slot_job:
                    # nothing running: wait for the next arrival, or for memory
                    # of finished jobs to be handed back
                    wait = arrivals[nxt] - (clock() - t0) if nxt < n else 0.01
                    time.sleep(max(0.0, min(wait, 0.01)))
                continue
            for slot in b.poll():
                j = slot_job.pop(slot)
                try:
                    events[j] = b.job_stats(slot)["rec_events"]
                    sp = b.read_spikes(slot)
                except snn.SNNError as e:   # the job's construction failed
                    try:
                        b.read_spikes(slot)   # reports the build error and frees the slot
                    except snn.SNNError as e2:
                        e = e2
                    failed.append((j, str(e)))
                    done_count += 1
                    continue
                lat[j] = clock() - t0 - arrivals[j]
                if keep_spikes:
                    rasters[j] = sp
                done_count += 1
    wall = clock() - t0
    return Result(latency=lat, events=events, wall=wall, rasters=rasters, failed=failed)


def serve_plain(jobs, arrivals, keep_spikes=False, clock=time.perf_counter):
    """One job at a time, each built and stepped alone with the plain path."""
    n = len(jobs)
    lat = np.full(n, np.nan)
    events = np.zeros(n, dtype=np.int64)
    rasters = [None] * n
    t0 = clock()
    for j in range(n):
        wait = arrivals[j] - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        net = jobs[j]["net"]
        N = net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])
        with snn.Net(net, hist_cap=int(N * jobs[j]["steps"] * 0.15) + 65536,
                     stream=snn.current_stream_handle()) as g:
            g.build_synapses()
            g.step(jobs[j]["steps"])
            sp = g.read_spikes()
            events[j] = g.stats()["rec_events"]
        lat[j] = clock() - t0 - arrivals[j]
        if keep_spikes:
            rasters[j] = sp
    wall = clock() - t0
    return Result(latency=lat, events=events, wall=wall, rasters=rasters)


def poisson_arrivals(n, rate_per_s, seed=4):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def summary(res, jobs):
    """Throughput and latency of a served run.  Jobs that failed (never
    admitted, or their build failed) have no latency and no simulated time:
    they are counted in `failed` and left out of every other figure."""
    lat = res["latency"]
    ok = ~np.isnan(lat)
    n_ok = int(ok.sum())
    sim_s = sum(j["steps"] for j, k in zip(jobs, ok) if k) * 1e-3
    pct = (lambda q: float(np.percentile(lat[ok], q))) if n_ok else (lambda q: float("nan"))
    return dict(jobs=len(jobs), failed=len(jobs) - n_ok, wall_s=res["wall"], jobs_per_s=n_ok / res["wall"],
                p50_s=pct(50), p99_s=pct(99),
                events_per_s=float(res["events"].sum() / res["wall"]), sim_s_per_wall_s=sim_s / res["wall"])


def bench_served(n_jobs=512, plain_jobs=128, capacity_jobs=64, load=0.8, seed=4, log=None,
                 hbm_budget=160 << 30, max_neurons=6 << 20, chunk_ms=50, gen=0, tune_jobs=16):
    """The served workload: the seeded stream of simulation jobs (grids
    2x2..16x16, Gaussian/exponential, 0.5-5 s), Poisson arrivals at `load`
    times the capacity measured by a saturated closed-loop batched run, served
    with continuous batching; the plain one-job-at-a-time server is run on the
    first `plain_jobs` jobs of the same stream with the same arrival process,
    and both servers' closed-loop capacities (throughput with every job
    queued at once) are measured on the first `capacity_jobs` jobs.  With
    tune_jobs > 0 the batch schedule is first chosen by the batch autotuner on
    the stream's first tune_jobs jobs (otherwise chunk_ms and the defaults)."""
    from . import workloads as W

    say = log or (lambda *a: None)
    jobs = W.serving_stream(n_jobs, seed=seed, gen=gen)
    schedule, tuning = None, None
    if tune_jobs:
        from . import autotune

        tuning = autotune.tune_batch(jobs[:tune_jobs], hbm_budget, max_neurons, cache=None, log=say)
        schedule = tuning["schedule"]
    cap_jobs = jobs[:capacity_jobs]
    rc = serve_batched(cap_jobs, np.zeros(len(cap_jobs)), hbm_budget, max_neurons, chunk_ms, schedule=schedule)
    capacity = len(cap_jobs) / rc["wall"]
    rcp = serve_plain(cap_jobs, np.zeros(len(cap_jobs)))
    capacity_plain = len(cap_jobs) / rcp["wall"]
    say(f"# capacity (closed loop, {len(cap_jobs)} jobs): batched {capacity:.2f} jobs/s, "
        f"plain {capacity_plain:.2f} jobs/s")
    arrivals = poisson_arrivals(n_jobs, load * capacity, seed=seed)
    rb = serve_batched(jobs, arrivals, hbm_budget, max_neurons, chunk_ms, schedule=schedule)
    sb = summary(rb, jobs)
    say(f"# served batched: {sb}")
    out = dict(jobs=n_jobs, arrival_rate_jobs_per_s=load * capacity, capacity_jobs_per_s=capacity,
               capacity_plain_jobs_per_s=capacity_plain,
               capacity_events_per_s=dict(batched=float(rc["events"].sum() / rc["wall"]),
                                          plain=float(rcp["events"].sum() / rcp["wall"])),
               p50_s=sb["p50_s"], p99_s=sb["p99_s"], jobs_per_s=sb["jobs_per_s"],
               events_per_s=sb["events_per_s"], sim_s_per_wall_s=sb["sim_s_per_wall_s"],
               failed=sb["failed"] + summary(rc, cap_jobs)["failed"],
               schedule=schedule or dict(chunk_ms=chunk_ms, options={}))
    if tuning:
        out["tuning"] = dict(jobs=tune_jobs, trials=tuning["trials"])
    if plain_jobs:
        pj = jobs[:plain_jobs]
        rp = serve_plain(pj, arrivals[:plain_jobs])
        sp = summary(rp, pj)
        rb2 = serve_batched(pj, arrivals[:plain_jobs], hbm_budget, max_neurons, chunk_ms, schedule=schedule)
        sb2 = summary(rb2, pj)
        say(f"# first {plain_jobs} jobs: plain {sp} | batched {sb2}")
        out["failed"] += sb2["failed"]
        out["same_stream_first_jobs"] = dict(
            jobs=plain_jobs,
            plain=dict(p50_s=sp["p50_s"], p99_s=sp["p99_s"], wall_s=sp["wall_s"], events_per_s=sp["events_per_s"]),
            batched=dict(p50_s=sb2["p50_s"], p99_s=sb2["p99_s"], wall_s=sb2["wall_s"],
                         events_per_s=sb2["events_per_s"]))
    return out
