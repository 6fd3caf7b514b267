"""Throughput of the free-surface LBM step on one MI355X.

Workload (default): the 3D rectangular dam break, 256 x 128 x 64 cells, D3Q19
TRT (Lambda = 3/16), FP32 populations (stored shifted by the lattice weights),
FP64 mass, no-slip walls, liquid column 64 x 96 x 64 at rest in the corner,
g = 2e-5, nu = 1e-3, Smagorinsky LES with C_S = 0.1 (the paper's turbulence
model for its dam breaks, Sec. 2.1 and Sec. 4.2), run with all four
reconstruction variants in turn: one bench step advances each of the four
variant runs by one time step.

The timed window (steps 100-1100 after the untimed warm-up, then 200 steps of
kernel timing) lies inside the phase in which all four variants stay stable;
later in the collapse the NBKC, OM and OM3 runs of this no-slip 3D setup
develop velocities above the lattice speed of sound (the paper reports the
same failure mode for NBKC, Sec. 4.2), so a longer window would time NaN
states. The status of every variant run is reported with the result.

Prints one JSON line: fluid+interface cell updates per second (MLUPS) over the
timed steps, the roofline of the dominant kernel (the streaming kernel: pull
streaming, walls, free-surface condition, mass exchange and collision of every
liquid and interface cell; HBM bound) from HIP events around its launches, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SOURCES = ["paper_2207_13962_amd/csrc/fslbm_kernels.h", "paper_2207_13962_amd/csrc/fslbm_device.h",
                  "paper_2207_13962_amd/csrc/fslbm_ops.h"]
LAYOUTS = ("two_grid", "in_place")


def traffic_file(layout="two_grid"):
    """Committed counter summary of the streaming kernel on dam256 for one
    population layout."""
    name = "k_stream_dam256_traffic.txt" if layout == "two_grid" else "k_stream_dam256_inplace_traffic.txt"
    return os.path.join(ROOT, "profiles", name)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(layout="two_grid"):
    """HBM bytes per launch of the streaming kernel from the committed rocprofv3
    counter summary, or None if it is missing or was taken on other kernel code."""
    path = traffic_file(layout)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bytes_per_update(q, storage_bytes):
    """Algorithmic bytes of one fluid cell update: read q populations, write q
    populations, read the cell's flag byte (interface cells move a few more
    bytes - mass, fill level, mark - which are not counted)."""
    return 2 * q * storage_bytes + 1


# rocprofv3 FETCH_SIZE / WRITE_SIZE are in KiB per dispatch and count L2
# traffic in units that differ from bytes moved; each is scaled by what the
# same counter reads for a plain copy kernel of known size (--copy-calibration
# run under the same counters).
COPY_BYTES = 1 << 30  # bytes read and bytes written by one calibration copy


def _counter_rows(path, counter, kernel_prefix):
    import csv
    vals = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter and row["Kernel_Name"].startswith(kernel_prefix):
                vals.append((int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    vals.sort()
    return [v for _, v in vals]


def _copy_counter(path, counter):
    """Counter value (KiB) of the calibration copies: the median of the five
    largest dispatches (the 1 GiB copies) of the calibration run."""
    import csv
    vals = sorted(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"] == counter)
    top = vals[-5:]
    return top[len(top) // 2]


def write_traffic(fetch_csv, write_csv, cfetch_csv, cwrite_csv, last, command, layout="two_grid"):
    """Turns two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of the
    benchmark, and the same two counters over the copy calibration, into the
    traffic summary read back by measured_traffic(): the mean over the last
    `last` streaming-kernel dispatches (the kernel-timing region)."""
    fe = _counter_rows(fetch_csv, "FETCH_SIZE", "void fslbm::k_stream<")
    wr = _counter_rows(write_csv, "WRITE_SIZE", "void fslbm::k_stream<")
    if not fe or not wr:
        raise SystemExit("no k_stream dispatches in the counter files")
    fe, wr = fe[-last:], wr[-last:]
    f_kib = sum(fe) / len(fe)
    w_kib = sum(wr) / len(wr)
    cf, cw = _copy_counter(cfetch_csv, "FETCH_SIZE"), _copy_counter(cwrite_csv, "WRITE_SIZE")
    fscale, wscale = COPY_BYTES / (1024.0 * cf), COPY_BYTES / (1024.0 * cw)
    hbm = fscale * 1024 * f_kib + wscale * 1024 * w_kib
    path = traffic_file(layout)
    with open(path, "w") as fh:
        fh.write("# HBM traffic of the streaming kernel (k_stream), dam256 workload (D3Q19 TRT + LES,\n")
        fh.write("# FP32 populations, %s), from rocprofv3 counters.\n"
                 % ("two population grids" if layout == "two_grid" else "one grid updated in place"))
        fh.write("# Commands (run from the repository root):\n")
        for c in command:
            fh.write("#   %s\n" % c)
        fh.write("# dispatches averaged: the last %d of each benchmark run (kernel-timing region)\n" % len(fe))
        fh.write("# calibration: a 1 GiB copy reads FETCH_SIZE = %.0f KiB and writes WRITE_SIZE = %.0f KiB,\n"
                 % (cf, cw))
        fh.write("# so HBM bytes = %.3f*1024*FETCH_SIZE + %.3f*1024*WRITE_SIZE\n" % (fscale, wscale))
        fh.write("kernel_source_sha256_16: %s\n" % kernel_source_hash())
        fh.write("fetch_size_kib_per_launch: %.1f\n" % f_kib)
        fh.write("write_size_kib_per_launch: %.1f\n" % w_kib)
        fh.write("fetch_scale: %.4f\n" % fscale)
        fh.write("write_scale: %.4f\n" % wscale)
        fh.write("hbm_bytes_per_launch: %.0f\n" % hbm)
    print(open(path).read())


def write_trace_summary(trace_dir, out_path, last, command,
                        title="rocprofv3 kernel trace of the benchmark, dam256 workload (4 variant runs)."):
    """Short text summary of a rocprofv3 --kernel-trace --stats run of the
    benchmark: per-kernel calls and mean duration, plus the streaming kernel's
    mean over the last `last` launches (the kernel-timing region)."""
    import csv
    import glob
    stats = list(csv.DictReader(open(glob.glob(os.path.join(trace_dir, "*_kernel_stats.csv"))[0])))
    trace = list(csv.DictReader(open(glob.glob(os.path.join(trace_dir, "*_kernel_trace.csv"))[0])))
    ks = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
          if r["Kernel_Name"].startswith("void fslbm::k_stream<")]
    with open(out_path, "w") as fh:
        fh.write("# %s\n" % title)
        fh.write("# command (from the repository root):\n")
        for c in command:
            fh.write("#   %s\n" % c)
        fh.write("%-72s %8s %12s %7s\n" % ("kernel", "calls", "mean_us", "pct"))
        for r in stats:
            fh.write("%-72s %8s %12.2f %7.2f\n" % (r["Name"][:72], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                   float(r["Percentage"])))
        if ks:
            tail = ks[-last:]
            fh.write("k_stream mean over the last %d launches (kernel-timing region): %.2f us\n"
                     % (len(tail), sum(tail) / len(tail)))
    print(open(out_path).read())


def scale_point(args, variant=3, warm=200, timed=200):
    """The streaming kernel on the dam break scaled 2x per axis (512x256x128,
    8.4x the fluid cells, a working set well beyond the Infinity Cache): its
    algorithmic HBM rate where bandwidth and not latency bounds the step.
    Context for the roofline above, not the headline workload."""
    import torch
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.fslbm import Simulation

    s = I.workload("dam512", **({"smagorinsky": args.les} if args.les else {}))
    p = s.params
    sb = {I.F64: 8, I.F32: 4, I.F16S: 2}[p.storage]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = Simulation(s, variant=variant, device="cuda:0", stream=stream)
        sim.set_graphs(not args.no_graphs)
        sim.step(warm)
        stream.synchronize()
        b = sim.mass(check=False)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(timed)
        ev1.record(stream)
        stream.synchronize()
        ms = ev0.elapsed_time(ev1)
        sim.set_timing(timed)
        kb = sim.mass(check=False)
        sim.step(timed)
        stream.synchronize()
        ka = sim.mass(check=False)
        n, kms = sim.kernel_time()
        sim.set_timing(0)
        sim.close()
    nfl = 0.5 * (kb["n_liquid"] + kb["n_interface"] + ka["n_liquid"] + ka["n_interface"])
    per_launch = nfl * bytes_per_update(p.q, sb)
    achieved = per_launch / (kms / n * 1e-3) / 1e9
    step_updates = 0.5 * (b["n_liquid"] + b["n_interface"] + kb["n_liquid"] + kb["n_interface"]) * timed
    return {
        "workload": "dam512: rectangular dam break %dx%dx%d, D3Q%d TRT%s, variant %s, steps %d-%d"
                    % (p.nx, p.ny, p.nz, p.q, " + LES" if args.les else "", I.VARIANT_NAMES[variant],
                       warm, warm + 2 * timed),
        "fluid_cells": int(ka["n_liquid"] + ka["n_interface"]),
        "mlups": step_updates / (ms * 1e-3) / 1e6,
        "kernel": "k_stream",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "avg_launch_ms": kms / n,
        "bytes_per_launch": per_launch,
        "status": "ok" if ka["status"] == 0 else "unstable (%d)" % ka["status"],
    }


# Algorithmic bytes per grid cell of one tracked-bubble update (seven passes):
# init 42 (flags; parent, volumes, target, flag written), union 5 (flags,
# parent), volume 21 (flags, parent, phi, old label; root written), amount 17
# (flags, parent, old label, phi), target 4, pressure 4, cells 17 (flags,
# parent; label and gas density written). Per-bubble entries are cached.
BUBBLE_BYTES_PER_CELL = 110


def bubbles_bench(args, warm=100, timed=200):
    """Cost of the tracked-bubble model (bubble model 2): the same closed box
    of rising bubbles stepped with a constant volume pressure and with every
    bubble tracked; the difference per step is the bubble update."""
    import torch
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.fslbm import Simulation

    out = {}
    s2 = I.bubbly_column(nx=192, ny=128, nz=128, n_bubbles=80, radius=(3.0, 9.0), fill=0.8, g=2e-5,
                         seed=11, storage=I.F32, bubble_model=2, sub=2)
    print("bubbles bench: setup built", file=sys.stderr, flush=True)
    for model in (0, 2):
        s = I.Setup(s2.params.with_(bubble_model=model), s2.type, s2.phi, s2.rho, s2.ux, s2.uy, s2.uz)
        p = s.params
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim = Simulation(s, device="cuda:0", stream=stream)
            sim.set_graphs(not args.no_graphs)
            sim.step(warm)
            stream.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sim.step(timed)
            ev1.record(stream)
            stream.synchronize()
            ms = ev0.elapsed_time(ev1) / timed
            m = sim.mass(check=False)
            nb = len(sim.bubbles(check=False)[0]) if model == 2 else None
            sim.close()
        out[model] = dict(ms=ms, fluid=int(m["n_liquid"] + m["n_interface"]), status=m["status"], bubbles=nb)
        print("bubbles bench: model %d %.4f ms per step" % (model, ms), file=sys.stderr, flush=True)
    n = p.n
    over_us = (out[2]["ms"] - out[0]["ms"]) * 1e3
    return {
        "workload": "closed box %dx%dx%d of liquid (80%% full) with 80 rising bubbles (radius 3-9), D3Q19 SRT "
                    "FP32, variant OM, steps %d-%d" % (p.nx, p.ny, p.nz, warm, warm + timed),
        "cells": n,
        "fluid_cells": out[2]["fluid"],
        "bubbles_tracked": out[2]["bubbles"],
        "ms_per_step_constant_pressure": out[0]["ms"],
        "ms_per_step_tracked_bubbles": out[2]["ms"],
        "bubble_update_us": over_us,
        "bubble_bytes_per_cell": BUBBLE_BYTES_PER_CELL,
        "bubble_update_GBps": BUBBLE_BYTES_PER_CELL * n / (over_us * 1e-6) / 1e9 if over_us > 0 else None,
        "status": ["ok" if out[k]["status"] == 0 else "unstable (%d)" % out[k]["status"] for k in (0, 2)],
    }


def validate_taylor(D=32, variants=(1, 2, 3, 4)):
    """The paper's Taylor-bubble setup at tube diameter D, all four variants:
    the Reynolds number of the rising bubble beside the paper's values."""
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.validation import PAPER_TAYLOR_RE, taylor_reynolds

    out = {"setup": "paper Taylor bubble, D = %d (%dx%dx%d, D3Q19 SRT, omega 1.8, Mo 0.015, Bo 100)"
                    % (D, D, D, 10 * D), "variants": {}}
    for v in variants:
        r = taylor_reynolds(D, variant=v, progress=lambda k: print(
            "taylor D=%d %s: step %d" % (D, I.VARIANT_NAMES[v], k), file=sys.stderr, flush=True))
        paper = PAPER_TAYLOR_RE.get(D, {}).get(v)
        r["Re_paper"] = paper
        r["rel_diff"] = (r["Re"] - paper) / paper if paper else None
        r["status"] = "ok" if r["status"] == 0 else "unstable (%d)" % r["status"]
        out["variants"][I.VARIANT_NAMES[v]] = r
        print("taylor D=%d %s: Re %.2f (paper %s)" % (D, I.VARIANT_NAMES[v], r["Re"], paper), file=sys.stderr,
              flush=True)
    return out


def validate_wave(L=200, variants=(1, 2, 3, 4)):
    """The paper's gravity wave at wavelength L, all four variants: the
    surface elevation at x = 0 against the analytic model (errors over the
    first t* = 6, 12 and 24), sampled every t* = 0.05 up to t* = 40."""
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.validation import gravity_wave_elevation, paper_curve_distances, wave_errors

    golden = os.path.join(ROOT, "tests", "golden", "gravity_wave_paper_curves.json")
    curves = json.load(open(golden))["variants"] if os.path.exists(golden) else None

    out = {"setup": "paper gravity wave, L = %d (%dx%dx1, D3Q19 SRT, omega 1.8, Re 10, a0 0.01 L, d L/2)"
                    % (L, L, L), "variants": {}}
    for v in variants:
        name = I.VARIANT_NAMES[v]
        t0 = time.perf_counter()
        r = gravity_wave_elevation(L, variant=v, progress=lambda ts: print(
            "wave L=%d %s: t* = %.1f" % (L, name, ts), file=sys.stderr, flush=True))
        e = wave_errors(r)
        e["steps"] = r["steps"]
        e["seconds"] = round(time.perf_counter() - t0, 1)
        e["status"] = "ok" if r["status"] == 0 else "unstable (%d)" % r["status"]
        # the elevation at every t* = 1 for plotting against the model
        e["a_sim_every_t1"] = [round(float(x), 4) for x in r["a_sim"][::20]]
        if curves:
            e["vs_paper_runs"] = {"t%g" % tm: paper_curve_distances(r, v, L, curves, t_max=tm)
                                  for tm in (12.0, 24.0) if tm <= r["t_star"][-1] + 1e-9}
        out["variants"][name] = e
        print("wave L=%d %s: max err to t*=12 %.3f, to t*=24 %.3f" % (
            L, name, e["max_abs_err_t12"], e["max_abs_err_t24"]), file=sys.stderr, flush=True)
    out["a_model_every_t1"] = [round(float(x), 4) for x in r["a_model"][::20]]
    return out


def copy_calibration():
    """A plain device copy of COPY_BYTES, five times (run under rocprofv3
    counters to calibrate FETCH_SIZE and WRITE_SIZE)."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 5}))


def copy_rate():
    """Device-to-device copy rate of a 1 GiB buffer (read + write bytes per
    second, best of five), the bandwidth a plain streaming kernel reaches."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * COPY_BYTES / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads for the host leg: OMP_NUM_THREADS when set (the share of the
    host this process is meant to use), else the CPU affinity."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(setup_fn, steps, threads):
    """FP64 oracle on the host: fluid+interface updates per second over `steps`
    steps of the same workload on `threads` OpenMP threads (the oracle's
    per-cell loops; results do not depend on the count). Only the steps are
    timed; the cell counts come from mass reports taken between them."""
    from oracle import Oracle
    s = setup_fn()
    s.params = s.params.with_(storage=0)
    o = Oracle(s)
    o.set_threads(threads)
    upd, dt, done = 0, 0.0, 0
    for _ in range(steps):
        r = o.mass()
        t0 = time.perf_counter()
        st = o.step(1)
        dt += time.perf_counter() - t0
        if st != 0:
            break
        a = o.mass()
        upd += 0.5 * (r.n_liquid + r.n_interface + a.n_liquid + a.n_interface)
        done += 1
    return upd / dt / 1e6, dt, done


def time_runs(setup, variants, steps, warmup, ksteps, graphs=True):
    """One run per variant of the same setup on a non-default stream (step
    graphs are replayed on it, captured before the warm-up): `warmup` untimed
    steps, then `steps` timed steps of every run (HIP events around the whole
    window), then `ksteps` steps with the streaming kernel's own launches
    timed. Returns the window's duration, the fluid+interface updates in it,
    per-run state, and the streaming kernel's mean launch time and
    algorithmic bytes per launch."""
    import torch
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.fslbm import Simulation

    p = setup.params
    sb = {I.F64: 8, I.F32: 4, I.F16S: 2}[p.storage]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sims = [Simulation(setup, variant=v, device="cuda:0", stream=stream) for v in variants]
        for s in sims:
            s.set_graphs(graphs)  # captures the step graph now
        # warmup, in the same interleaving as the timed region
        for s in sims:
            s.step(warmup)
        stream.synchronize()
        before = [s.mass(check=False) for s in sims]
        chunk = 48
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream.synchronize()
        ev0.record(stream)
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            for s in sims:
                s.step(n)
            done += n
        ev1.record(stream)
        stream.synchronize()
        ms = ev0.elapsed_time(ev1)
        after = [s.mass(check=False) for s in sims]
        # dominant kernel: the streaming launches of a second region, each
        # launch recording its own start/stop timestamps
        for s in sims:
            s.set_timing(ksteps)
        kb = [s.mass(check=False) for s in sims]
        for s in sims:
            s.step(ksteps)
        stream.synchronize()
        ka = [s.mass(check=False) for s in sims]
        launches, kms, liq_bytes = 0, 0.0, 0.0
        for s, b, a in zip(sims, kb, ka):
            n, t = s.kernel_time()
            launches += n
            kms += t
            nfl = 0.5 * (b["n_liquid"] + b["n_interface"] + a["n_liquid"] + a["n_interface"])
            liq_bytes += n * nfl * bytes_per_update(p.q, sb)
            s.set_timing(0)
        for s in sims:
            s.close()
    updates = 0.0
    per_variant = {}
    for v, b, a, k in zip(variants, before, after, ka):
        nb = b["n_liquid"] + b["n_interface"]
        na = a["n_liquid"] + a["n_interface"]
        updates += 0.5 * (nb + na) * steps
        per_variant[I.VARIANT_NAMES[v]] = dict(
            fluid_cells=int(na), interface_cells=int(a["n_interface"]),
            mass_drift=(a["total_mass"] - b["total_mass"]) / b["total_mass"],
            status="ok" if k["status"] == 0 else "unstable (%d)" % k["status"])
    return dict(ms=ms, updates=updates, per_variant=per_variant, launches=launches,
                avg_launch_ms=kms / max(launches, 1), bytes_per_launch=liq_bytes / max(launches, 1),
                bytes_per_update=bytes_per_update(p.q, sb))


def concurrent_runs(setup, variants, steps, warmup):
    """The variant runs of `time_runs` stepped side by side, each on a stream
    of its own (default priority), so that one run's latency-bound launches
    (re-typing, compaction) overlap another run's streaming launch: the same
    work as the headline window (steps warmup..warmup+steps of every run),
    timed by events on a joining stream. Returns fluid+interface MLUPS and the
    window's duration."""
    import torch
    from paper_2207_13962_amd.fslbm import Simulation

    streams = [torch.cuda.Stream() for _ in variants]
    sims = [Simulation(setup, variant=v, device="cuda:0", stream=st) for v, st in zip(variants, streams)]
    for s in sims:
        s.set_graphs(True)
    for s in sims:
        s.step(warmup)
    torch.cuda.synchronize()
    before = [s.mass(check=False) for s in sims]
    main = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(main)
    for st in streams:
        st.wait_event(ev0)
    chunk, done = 48, 0
    while done < steps:
        n = min(chunk, steps - done)
        for s in sims:
            s.step(n)
        done += n
    for st in streams:
        e = torch.cuda.Event()
        e.record(st)
        main.wait_event(e)
    ev1.record(main)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    after = [s.mass(check=False) for s in sims]
    for s in sims:
        s.close()
    updates = sum(0.5 * (b["n_liquid"] + b["n_interface"] + a["n_liquid"] + a["n_interface"]) * steps
                  for b, a in zip(before, after))
    ok = all(a["status"] == 0 for a in after)
    return {"value": updates / (ms * 1e-3) / 1e6, "unit": "MLUPS", "ms": ms,
            "ms_per_time_step": ms / (steps * len(variants)), "streams": len(variants),
            "all_runs_stable": ok}


def _line(name, setup, variants, steps, warmup, ksteps, graphs):
    from paper_2207_13962_amd import inputs as I
    p = setup.params
    r = time_runs(setup, variants, steps, warmup, ksteps, graphs)
    achieved = r["bytes_per_launch"] / (r["avg_launch_ms"] * 1e-3) / 1e9
    return {
        "workload": name,
        "lattice": "D3Q%d %s" % (p.q, "TRT" if p.collision else "SRT"),
        "dtype": {I.F64: "f64", I.F32: "f32", I.F16S: "f16-shifted/f32"}[p.storage],
        "variants": "/".join(I.VARIANT_NAMES[v] for v in variants),
        "steps": "%d-%d of each run" % (warmup, warmup + steps),
        "value": r["updates"] / (r["ms"] * 1e-3) / 1e6,
        "unit": "MLUPS",
        "ms_per_time_step": r["ms"] / (steps * len(variants)),
        "roofline": {"kernel": "k_stream", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "bytes_per_update": r["bytes_per_update"], "bytes_per_launch": r["bytes_per_launch"],
                     "avg_launch_ms": r["avg_launch_ms"]},
        "per_variant": r["per_variant"],
    }


def extra_lines(args):
    """Throughput of the other measured workloads (each within its stable
    window): the dam break in FP64 (the paper's precision) and with one
    population grid updated in place (FP32 and FP16-shifted), the cylindrical
    dam break (D3Q27, free-slip walls, conversion-heavy) and the Taylor bubble
    (D3Q27, surface tension, single-bubble volume pressure) in its three
    storage formats. Context for the headline line."""
    from paper_2207_13962_amd import inputs as I
    graphs = not args.no_graphs
    les = {"smagorinsky": args.les} if args.les else {}
    out = {}
    cache = {}

    def taylor(st):
        if "t" not in cache:
            cache["t"] = I.workload("taylor512", storage=I.F64)
        t = cache["t"]
        return I.Setup(t.params.with_(storage=st), t.type, t.phi, t.rho, t.ux, t.uy, t.uz)

    def inplace(st):
        d = I.workload("dam256", storage=st, **les)
        return I.Setup(d.params.with_(layout=I.AA), d.type, d.phi, d.rho, d.ux, d.uy, d.uz)

    todo = [
        ("dam256_fp64", lambda: I.workload("dam256", storage=I.F64, **les), [1, 2, 3, 4], 200, 100),
        ("dam256_inplace_fp32", lambda: inplace(I.F32), [1, 2, 3, 4], 200, 100),
        ("dam256_inplace_f16s", lambda: inplace(I.F16S), [1, 2, 3, 4], 200, 100),
        ("cyl256_fp32", lambda: I.workload("cyl256", **les), [1, 2, 3, 4], 200, 100),
        ("taylor512_fp64", lambda: taylor(I.F64), [3], 200, 50),
        ("taylor512_fp32", lambda: taylor(I.F32), [3], 200, 50),
        ("taylor512_f16s", lambda: taylor(I.F16S), [3], 200, 50),
    ]
    for name, fn, variants, steps, warm in todo:
        try:
            s = fn()
            p = s.params
            desc = "%s: %dx%dx%d%s%s%s" % (name.split("_")[0], p.nx, p.ny, p.nz,
                                           ", Smagorinsky C_S = %g" % p.smagorinsky if p.smagorinsky else "",
                                           ", surface tension %g, single-bubble volume pressure" % p.sigma
                                           if p.sigma else "",
                                           ", one population grid updated in place (AA pattern)"
                                           if p.layout == I.AA else "")
            out[name] = _line(desc, s, variants, steps, warm, min(steps, 100), graphs)
            if p.layout == I.AA:
                from paper_2207_13962_amd.fslbm import workspace_bytes
                two = workspace_bytes(p.with_(layout=I.TWO_GRID))
                out[name]["device_bytes"] = {"in_place": workspace_bytes(p), "two_grid": two}
            print("line %s: %.0f MLUPS, k_stream %.2f of peak" % (
                name, out[name]["value"], out[name]["roofline"]["frac"]), file=sys.stderr, flush=True)
        except Exception as e:  # context only: never hides the headline result
            out[name] = {"error": repr(e)}
    return out


def serving_density(args, reqs):
    """What the in-place layout buys a server: the same closed batch (every run
    submitted at t = 0) served with two population grids and in place, under
    the same pool budget (--budget-gb): peak resident runs, peak pool use and
    runs/s. With a pool smaller than the mix, more resident runs share each
    batched launch. Fill levels must agree bitwise between the layouts."""
    import numpy as np
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd import serving as SV
    from paper_2207_13962_amd.fslbm import workspace_bytes

    budget = int(args.budget_gb * (1 << 30))
    zero = [0.0] * len(reqs)
    out = {"workload": "%d runs: drop impacts (L^3, FP64) and wave slabs (L x L/2 x L/4, FP32), L in [%d, %d], "
                       "%d-%d steps, closed batch, pool %.2f GiB" % (
                           len(reqs), args.l_min, args.l_max, args.steps_min, args.steps_max, args.budget_gb)}
    phis = {}
    for name, lay in (("two_grid", I.TWO_GRID), ("in_place", I.AA)):
        for r in reqs:
            r["setup"].params = r["setup"].params.with_(layout=lay)
        SV.run_batched(reqs[:4], zero[:4], budget, max_slots=args.slots)  # warm-up (code load)
        res, runs = SV.run_batched(reqs, zero, budget, max_slots=args.slots, keep_phi=True)
        phis[name] = runs
        out[name] = {"runs_per_s": res["runs_per_s"], "makespan_s": res["makespan_s"],
                     "peak_resident": res["peak_resident"], "peak_pool_GB": res["peak_pool_bytes"] / 1e9,
                     "mix_bytes_GB": sum(workspace_bytes(r["setup"].params) for r in reqs) / 1e9}
        print("serving density: %s %.1f runs/s, peak resident %d" % (name, res["runs_per_s"], res["peak_resident"]),
              file=sys.stderr, flush=True)
    out["identical_results"] = all(a[0] == b[0] and np.array_equal(a[2], b[2], equal_nan=True)
                                   for a, b in zip(phis["two_grid"], phis["in_place"]))
    out["speedup_runs_per_s"] = out["in_place"]["runs_per_s"] / out["two_grid"]["runs_per_s"]
    return out


def serving_section(args, reqs=None):
    """Batched serving against one-at-a-time solves on a request mix shaped
    like the serving workload (drop impacts with FP64 populations and wave
    slabs with FP32, variants uniform): closed batches (every run arriving at t = 0) give each mode's
    capacity in runs/s; then Poisson arrivals at `load` times the batched
    capacity are served both ways: runs/s over the makespan, p50/p99 time to
    solution (queueing included). The fill levels of every run must agree
    bitwise between the two modes."""
    import numpy as np
    from paper_2207_13962_amd import serving as SV

    if reqs is None:
        reqs = SV.make_mix(n_requests=args.requests, l_min=args.l_min, l_max=args.l_max,
                           steps_min=args.steps_min, steps_max=args.steps_max)
    budget = int(args.budget_gb * (1 << 30))
    zero = [0.0] * len(reqs)
    SV.run_batched(reqs[:4], zero[:4], budget, max_slots=args.slots)  # warm-up (code load)
    closed, _ = SV.run_batched(reqs, zero, budget, max_slots=args.slots)
    print("serving: closed batch %.1f runs/s" % closed["runs_per_s"], file=sys.stderr, flush=True)
    closed_single, _ = SV.run_sequential(reqs, zero)
    print("serving: closed, one at a time %.1f runs/s" % closed_single["runs_per_s"], file=sys.stderr,
          flush=True)
    rate = args.load * closed["runs_per_s"]
    arrival = SV.poisson_arrivals(reqs, rate)
    batched, rb = SV.run_batched(reqs, arrival, budget, max_slots=args.slots, keep_phi=True)
    print("serving: batched %.1f runs/s" % batched["runs_per_s"], file=sys.stderr, flush=True)
    single, rs = SV.run_sequential(reqs, arrival, keep_phi=True)
    print("serving: one at a time %.1f runs/s" % single["runs_per_s"], file=sys.stderr, flush=True)
    # (a run that became unstable holds non-finite fill levels; NaN == NaN here)
    same = all(a[0] == b[0] and np.array_equal(a[2], b[2], equal_nan=True) for a, b in zip(rb, rs))
    cells = [r["L"] ** 3 if r["kind"] == "drop" else r["L"] * (r["L"] // 2) * max(r["L"] // 4, 1)
             for r in reqs]
    return {
        "workload": "%d runs: drop impacts (L^3) and wave slabs (L x L/2 x L/4), L in [%d, %d], "
                    "%d-%d steps, D3Q19 (drops TRT with FP64 populations, waves SRT with FP32), variants uniform" % (
                        len(reqs), args.l_min, args.l_max, args.steps_min, args.steps_max),
        "cells_total": int(sum(cells)),
        "steps_total": int(sum(r["steps"] for r in reqs)),
        "capacity_runs_per_s": {"batched": closed["runs_per_s"],
                                "one_at_a_time": closed_single["runs_per_s"],
                                "speedup": closed["runs_per_s"] / closed_single["runs_per_s"]},
        "poisson_rate_runs_per_s": rate,
        "batched": batched,
        "one_at_a_time": single,
        "speedup_runs_per_s": batched["runs_per_s"] / single["runs_per_s"],
        "identical_results": bool(same),
        "unstable_runs": int(sum(1 for r in rb if r[0] != 0)),
    }


def precision_study(args):
    """FP32 and FP16-shifted population storage against FP64 (the FP64 mode is
    parity-checked against the oracle): front position and mass drift on the
    rectangular dam break (all four variants), rise velocity and mass drift of
    the Taylor bubble (surface tension, bubble model)."""
    import numpy as np
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.fslbm import Simulation

    names = {I.F64: "f64", I.F32: "f32", I.F16S: "f16s"}
    out = {"dam_break": {}, "taylor_bubble": {}}
    every = 100
    for v in (1, 2, 3, 4):
        res = {}
        for st in (I.F64, I.F32, I.F16S):
            s = I.workload("dam256", smagorinsky=args.les, storage=st, variant=v)
            sim = Simulation(s)
            m0 = sim.mass()["total_mass"]
            fronts, status = [], 0
            for n in range(0, args.dam_steps + 1, every):
                if n:
                    sim.step(every)
                r = sim.mass(check=False)
                if r["status"] != 0:
                    status = r["status"]
                    break
                t = sim.fields(pdf=False, check=False)["type"].reshape(s.params.nz, s.params.ny, s.params.nx)
                floor = ((t[:, 0, :] == 1) | (t[:, 0, :] == 2)).any(axis=0)
                fronts.append(int(np.nonzero(floor)[0].max()))
            res[names[st]] = dict(front=fronts, status=status,
                                  mass_drift=(r["total_mass"] - m0) / m0)
            sim.close()
            print("precision: dam break %s %s done" % (I.VARIANT_NAMES[v], names[st]), file=sys.stderr,
                  flush=True)
        ref = res["f64"]["front"]
        for k in ("f32", "f16s"):
            f = res[k]["front"]
            n = min(len(f), len(ref))
            res[k]["max_front_diff_cells"] = int(max(abs(a - b) for a, b in zip(f[:n], ref[:n]))) if n else None
        out["dam_break"][I.VARIANT_NAMES[v]] = res
    # Taylor bubble: centroid of the gas (1 - phi over gas and interface cells)
    every = args.taylor_steps // 10
    for st in (I.F64, I.F32, I.F16S):
        s = I.workload("taylor512", storage=st)
        p = s.params
        zc = np.repeat(np.arange(p.nz) + 0.5, p.nx * p.ny)
        sim = Simulation(s)
        m0 = sim.mass()["total_mass"]
        cz, status = [], 0
        for n in range(0, args.taylor_steps + 1, every):
            if n:
                sim.step(every)
            r = sim.mass(check=False)
            if r["status"] != 0:
                status = r["status"]
                break
            f = sim.fields(pdf=False, check=False)
            w = np.where((f["type"] == 0) | (f["type"] == 1), 1.0 - f["phi"], 0.0)
            cz.append(float((w * zc).sum() / w.sum()))
        half = len(cz) // 2
        vel = (cz[-1] - cz[half]) / ((len(cz) - 1 - half) * every) if len(cz) > 2 else None
        out["taylor_bubble"][names[st]] = dict(centroid_z=cz, rise_velocity=vel, status=status,
                                                 mass_drift=(r["total_mass"] - m0) / m0,
                                                 bubble_volume=r["bubble_volume"])
        sim.close()
        print("precision: Taylor bubble %s done" % names[st], file=sys.stderr, flush=True)
    ref = out["taylor_bubble"]["f64"]["rise_velocity"]
    for k in ("f32", "f16s"):
        v = out["taylor_bubble"][k]["rise_velocity"]
        out["taylor_bubble"][k]["rise_velocity_rel_err"] = (v - ref) / ref if (v and ref) else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="dam256")
    ap.add_argument("--variants", default="1,2,3,4")
    ap.add_argument("--layout", choices=LAYOUTS, default="two_grid",
                    help="population layout of the main run: two grids, or one grid updated in place")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle steps, single-thread CPU baseline")
    ap.add_argument("--cpu-steps-all", type=int, default=100,
                    help="oracle steps, CPU baseline on all host threads")
    ap.add_argument("--no-lines", action="store_true",
                    help="skip the FP64 dam break, cylindrical dam break and Taylor-bubble lines")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the variant runs stepped side by side on four streams")
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="time steps per variant run of the kernel-timing region")
    ap.add_argument("--les", type=float, default=0.1, help="Smagorinsky constant (0: off)")
    ap.add_argument("--no-graphs", action="store_true", help="launch kernel by kernel")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to calibrate the HBM counters")
    ap.add_argument("--write-traffic", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="summarise rocprofv3 counter runs into the traffic file and exit")
    ap.add_argument("--write-trace-summary", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--trace-title", default=None, help="first line of a trace summary")
    ap.add_argument("--trace-out", default=None, help="file a trace summary is written to")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line recorded in a profile summary (repeat per run)")
    ap.add_argument("--precision-study", action="store_true",
                    help="only the storage-precision study (FP32/FP16-shifted against FP64)")
    ap.add_argument("--dam-steps", type=int, default=1500, help="precision study: dam-break steps")
    ap.add_argument("--taylor-steps", type=int, default=10000, help="precision study: Taylor-bubble steps")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-scale-point", action="store_true",
                    help="skip the streaming kernel on the dam break scaled 2x per axis")
    ap.add_argument("--validate-taylor", type=int, default=0, metavar="D",
                    help="the paper's Taylor-bubble runs at tube diameter D (32, 64 or 128), four variants")
    ap.add_argument("--bubbles", action="store_true",
                    help="only the cost of the tracked-bubble model on a closed box of rising bubbles")
    ap.add_argument("--validate-wave", type=int, default=0, metavar="L",
                    help="the paper's gravity wave at wavelength L (200, 400 or 800), four variants")
    ap.add_argument("--scale-only", action="store_true",
                    help="only the streaming kernel on the dam break scaled 2x per axis (kernel by kernel)")
    ap.add_argument("--serving-only", action="store_true", help="only the serving measurement")
    ap.add_argument("--serving-density", action="store_true",
                    help="only the same closed batch served with two grids and in place under --budget-gb")
    ap.add_argument("--requests", type=int, default=48, help="serving: runs in the mix")
    ap.add_argument("--l-min", type=int, default=32, help="serving: smallest domain edge")
    ap.add_argument("--l-max", type=int, default=64, help="serving: largest domain edge")
    ap.add_argument("--steps-min", type=int, default=200, help="serving: fewest steps of a run")
    ap.add_argument("--steps-max", type=int, default=800, help="serving: most steps of a run")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: device pool (GiB)")
    ap.add_argument("--slots", type=int, default=64, help="serving: resident runs at most")
    ap.add_argument("--build-workers", type=int, default=1,
                    help="serving: host processes building the request setups")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving: Poisson rate as a fraction of the batched capacity")
    args = ap.parse_args()
    last = len(args.variants.split(",")) * min(args.steps, args.kernel_steps)
    if args.write_traffic:
        write_traffic(*args.write_traffic, last, args.profile_command, args.layout)
        return
    if args.write_trace_summary:
        kw = {"title": args.trace_title} if args.trace_title else {}
        write_trace_summary(args.write_trace_summary,
                            args.trace_out or os.path.join(ROOT, "profiles", "k_stream_dam256_%strace.txt"
                                                           % ("" if args.layout == "two_grid" else "inplace_")),
                            last,
                            args.profile_command, **kw)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the free-surface LBM step here runs on a single "
              "MI355X (no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    reqs = None
    if args.serving_only or args.serving_density:
        # the request setups are built on the host before the GPU is touched
        # (worker processes are forked from a process without GPU state)
        from paper_2207_13962_amd import serving as SV
        reqs = SV.make_mix(n_requests=args.requests, l_min=args.l_min, l_max=args.l_max,
                           steps_min=args.steps_min, steps_max=args.steps_max,
                           workers=args.build_workers)

    import torch
    from paper_2207_13962_amd import inputs as I
    from paper_2207_13962_amd.fslbm import Simulation

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serving_only:
        print(json.dumps(serving_section(args, reqs)))
        return
    if args.serving_density:
        print(json.dumps(serving_density(args, reqs)))
        return
    if args.precision_study:
        print(json.dumps(precision_study(args)))
        return
    if args.scale_only:
        print(json.dumps(scale_point(args)))
        return
    if args.validate_taylor:
        print(json.dumps(validate_taylor(args.validate_taylor, [int(v) for v in args.variants.split(",")])))
        return
    if args.bubbles:
        print(json.dumps(bubbles_bench(args)))
        return
    if args.validate_wave:
        print(json.dumps(validate_wave(args.validate_wave, [int(v) for v in args.variants.split(",")])))
        return
    # serving first: its small runs are latency-bound and measured lower
    # after the long bandwidth-bound runs below (224-315 against 389-414
    # runs/s on the same kind of box)
    serving = None
    if not args.no_serving:
        try:
            serving = serving_section(args)
        except Exception as e:  # the serving figures must never hide the step result
            serving = {"error": repr(e)}
    variants = [int(v) for v in args.variants.split(",")]
    setup_fn = lambda: I.workload(args.workload, **({"smagorinsky": args.les} if args.les else {}))  # noqa: E731
    base = setup_fn()
    if args.layout == "in_place":
        base.params = base.params.with_(layout=I.AA)
    p = base.params
    sb = {I.F64: 8, I.F32: 4, I.F16S: 2}[p.storage]
    # the runs side by side first, so that the kernel-timing region stays the
    # last streaming launches of the process (the profiles average those)
    concurrent = None
    if not args.no_concurrent:
        try:
            concurrent = concurrent_runs(base, variants, args.steps, args.warmup)
            concurrent["effective_GBps_whole_step"] = (concurrent["value"] * 1e6 * bytes_per_update(p.q, sb)
                                                       / 1e9)
            concurrent["effective_whole_step_frac_of_peak"] = concurrent["effective_GBps_whole_step"] / HBM_PEAK_GBS
            concurrent["note"] = ("the same runs and steps as the headline window, the four runs stepped side "
                                  "by side on four streams instead of in turn on one")
        except Exception as e:  # context only: never hides the headline result
            concurrent = {"error": repr(e)}
    r = time_runs(base, variants, args.steps, args.warmup, min(args.steps, args.kernel_steps),
                  not args.no_graphs)
    ms, updates, per_variant = r["ms"], r["updates"], r["per_variant"]
    mlups = updates / (ms * 1e-3) / 1e6
    avg_ms, bytes_per_launch, launches = r["avg_launch_ms"], r["bytes_per_launch"], r["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.layout)
    whole_gbs = updates * bytes_per_update(p.q, sb) / (ms * 1e-3) / 1e9
    try:
        copy_gbs = copy_rate()
    except Exception:  # context only
        copy_gbs = None

    cpu = None
    if not args.no_cpu:
        try:
            threads = host_threads()
            v1, dt1, n1 = cpu_baseline(setup_fn, args.cpu_steps, 1)
            vn, dtn, nn = cpu_baseline(setup_fn, args.cpu_steps_all, threads)
            cpu = {"value": vn, "unit": "MLUPS", "cores": threads, "kind": "oracle",
                   "sample": "steps 1-%d of the %s workload (%dx%dx%d, FP64 oracle, variant OM) on %d "
                             "OpenMP threads, %.1f s; fluid+interface updates counted outside the timer"
                             % (nn, args.workload, p.nx, p.ny, p.nz, threads, dtn),
                   "single_thread": {"value": v1, "cores": 1,
                                     "sample": "steps 1-%d, %.1f s" % (n1, dt1)},
                   "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model()}
        except Exception as e:  # the baseline must never hide the GPU result
            cpu = {"value": None, "error": repr(e)}

    out = {
        "metric": "fluid+interface MLUPS (free-surface LBM step)",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "ms_per_time_step": ms / (args.steps * len(variants)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {I.F64: "f64", I.F32: "f32", I.F16S: "f16-shifted/f32"}[p.storage],
        "data": "synthetic",
        "config": {
            "workload": "%s: rectangular dam break %dx%dx%d, D3Q%d %s, variants %s, %d steps per variant run%s"
                        % (args.workload, p.nx, p.ny, p.nz, p.q, "TRT" if p.collision else "SRT",
                           "/".join(I.VARIANT_NAMES[v] for v in variants), args.steps,
                           "" if args.layout == "two_grid" else ", one population grid updated in place"),
            "layout": args.layout,
            "cells": p.n,
            "parallelism": "single GPU",
            "effective_GBps_whole_step": whole_gbs,
            "effective_whole_step_frac_of_peak": whole_gbs / HBM_PEAK_GBS,
            "copy_GBps_measured": copy_gbs,
            "smagorinsky": args.les,
            "bench_step": "one time step of each of the %d variant runs (ms_per_time_step: one run's "
                          "time step)" % len(variants),
            "step_launches": "kernel by kernel" if args.no_graphs else
                             "replayed HIP graphs of 8 and 2 steps, both step parities (captured before the warm-up)",
            "per_variant": per_variant,
        },
        "roofline": {
            "kernel": "k_stream (pull streaming, walls, free-surface condition, mass exchange, TRT%s "
                      "collision; all fluid cells)" % (" + LES" if args.les else ""),
            "bytes_model": "%d B per fluid cell update (read and write %d populations of %d B, one flag byte)"
                           % (bytes_per_update(p.q, sb), p.q, sb),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "launches": launches,
            "bytes_per_launch": bytes_per_launch,
            "frac_of_measured_copy": achieved / copy_gbs if copy_gbs else None,
        },
        "cpu_baseline": cpu,
    }
    if concurrent is not None:
        out["concurrent_variants"] = concurrent
    if not args.no_lines:
        out["lines"] = extra_lines(args)
    if not args.no_scale_point:
        try:
            out["roofline_dam512"] = scale_point(args)
        except Exception as e:  # context only: never hides the headline result
            out["roofline_dam512"] = {"error": repr(e)}
    if serving is not None:
        out["serving"] = serving
    print(json.dumps(out))
    bad = [k for k, v in per_variant.items() if v["status"] != "ok"]
    if bad:
        print("warning: variant runs %s became unstable inside the timed window; their later "
              "steps ran on non-finite states" % ",".join(bad), file=sys.stderr)


if __name__ == "__main__":
    main()
