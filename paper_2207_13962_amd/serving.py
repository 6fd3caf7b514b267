"""Request driver for batched serving: Poisson arrivals of independent runs,
served either by one fslbm server (continuous batching: runs that arrive while
others are on the GPU join the resident batch as slots and pool memory free
up) or one at a time (FIFO, each run alone in its own context with replayed
step graphs). Reports runs/s over the makespan and p50/p99 time to solution
(completion minus arrival, queueing included).

Every GPU step runs in libfslbm; this module only schedules submissions and
collects results.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import inputs as I


def _build(r):
    return I.build_request(r)


def make_mix(n_requests=48, seed=1234, l_min=32, l_max=64, steps_min=200, steps_max=800, workers=1):
    """A request mix shaped like the serving workload (drop impacts and
    standing-wave slabs, variant uniform; FP64 populations for the drops, FP32
for the waves, see inputs.build_request), with setups built
    up front (in `workers` processes); arrival times are assigned by
    `poisson_arrivals`."""
    reqs = I.serving_mix(n_requests=n_requests, seed=seed, l_min=l_min, l_max=l_max,
                         steps_min=steps_min, steps_max=steps_max)
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            setups = pool.map(_build, reqs, chunksize=1)
    else:
        setups = [_build(r) for r in reqs]
    for r, st in zip(reqs, setups):
        r["setup"] = st
    print("serving mix: %d setups built" % len(reqs), file=sys.stderr, flush=True)
    return reqs


def poisson_arrivals(reqs, rate, seed=99):
    """Arrival times (s) of a Poisson process of the given rate (runs/s);
    rate None or <= 0 puts every arrival at t = 0."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in reqs:
        if rate and rate > 0:
            t += float(rng.exponential(1.0 / rate))
        out.append(t)
    return out


def _summary(arrival, done, t_end, label):
    lat = np.array([done[i] - arrival[i] for i in range(len(arrival))])
    return {
        "mode": label,
        "runs": len(arrival),
        "makespan_s": t_end,
        "runs_per_s": len(arrival) / t_end if t_end > 0 else float("nan"),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
    }


def run_batched(reqs, arrival, budget_bytes, max_slots=64, ticks=16, device="cuda:0", keep_phi=False,
                progress=32):
    """Serve the requests with one fslbm server. Returns (summary, results):
    results[i] = (status, mass report, phi or None)."""
    import torch
    from .fslbm import Server

    srv = Server(budget_bytes, max_slots=max_slots, device=device)
    order = np.argsort(arrival, kind="stable")
    n = len(reqs)
    done_t = [None] * n
    results = [None] * n
    id2idx = {}
    nxt = 0
    peak_resident = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    finished = 0
    occupancy = []  # (s, pool bytes in use, resident runs, queued runs) after each advance
    while finished < n:
        now = time.perf_counter() - t0
        while nxt < n and arrival[order[nxt]] <= now:
            i = int(order[nxt])
            id2idx[srv.submit(reqs[i]["setup"], reqs[i]["steps"])] = i
            nxt += 1
        st = srv.stats()
        peak_resident = max(peak_resident, st["resident"])
        if st["resident"] == 0 and st["queued"] == 0:
            # idle until the next arrival
            if nxt < n:
                time.sleep(max(0.0, arrival[order[nxt]] - (time.perf_counter() - t0)))
            continue
        srv.advance(ticks)
        st = srv.stats()
        occupancy.append((time.perf_counter() - t0, st["bytes_in_use"], st["resident"], st["queued"]))
        for rid, status in srv.poll():
            i = id2idx.pop(rid)
            rep, phi = srv.result(rid, phi=keep_phi)
            done_t[i] = time.perf_counter() - t0
            results[i] = (status, rep, phi)
            finished += 1
            if progress and finished % progress == 0:
                print("batched: %d of %d done at %.1f s" % (finished, n, done_t[i]), file=sys.stderr,
                      flush=True)
    t_end = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = _summary(arrival, done_t, t_end, "batched")
    out.update(peak_resident=peak_resident, peak_pool_bytes=st["peak_bytes_in_use"],
               budget_bytes=st["budget_bytes"], ticks=st["ticks"],
               occupancy=occupancy_timeline(occupancy, t_end))
    return out, results


def occupancy_timeline(samples, t_end, points=24):
    """Pool use over time: for each of `points` equal time bins the largest
    bytes in use, resident and queued runs seen in it (GB, counts), and the
    time-weighted mean pool use."""
    if not samples:
        return {}
    edges = np.linspace(0.0, t_end, points + 1)
    rows = []
    for a, b in zip(edges[:-1], edges[1:]):
        sel = [x for x in samples if a <= x[0] < b]
        if sel:
            rows.append([round(float(b), 3), round(max(x[1] for x in sel) / 1e9, 3), max(x[2] for x in sel),
                         max(x[3] for x in sel)])
    ts = np.array([x[0] for x in samples])
    used = np.array([x[1] for x in samples], dtype=np.float64)
    dt = np.diff(np.concatenate([[0.0], ts]))
    return {"bins_t_end_s_peak_GB_resident_queued": rows,
            "mean_GB": float((used * dt).sum() / max(dt.sum(), 1e-12) / 1e9),
            "peak_GB": float(used.max() / 1e9)}


def run_sequential(reqs, arrival, device="cuda:0", keep_phi=False, progress=32):
    """One run at a time, in arrival order, each alone in its own context."""
    import torch
    from .fslbm import Simulation

    order = np.argsort(arrival, kind="stable")
    n = len(reqs)
    done_t = [None] * n
    results = [None] * n
    stream = torch.cuda.Stream(device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in order:
            i = int(i)
            wait = arrival[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            sim = Simulation(reqs[i]["setup"], device=device, stream=stream)
            sim.step(reqs[i]["steps"])
            rep = sim.mass(check=False)
            phi = sim.fields(pdf=False, check=False)["phi"] if keep_phi else None
            sim.close()
            done_t[i] = time.perf_counter() - t0
            results[i] = (rep["status"], rep, phi)
            if progress and sum(r is not None for r in results) % progress == 0:
                print("one at a time: %d of %d done" % (sum(r is not None for r in results), n),
                      file=sys.stderr, flush=True)
    t_end = time.perf_counter() - t0
    return _summary(arrival, done_t, t_end, "one-at-a-time"), results
