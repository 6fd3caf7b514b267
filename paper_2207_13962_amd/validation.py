"""Validation against the paper's own results: the Taylor-bubble runs of
Sec. 4.4 (tube diameter D, all four boundary-condition variants), whose
Reynolds numbers the paper tabulates, and the gravity wave of Sec. 4.1 at the
paper's resolutions against the analytic model the paper compares with. Every
step runs in libfslbm; this module builds the setups, samples the fill levels
and reduces them to the rise velocity or the surface elevation."""
from __future__ import annotations

import math

import numpy as np

from . import inputs as I

# Reynolds numbers of the paper's Taylor-bubble runs (Sec. 4.4, table of Re by
# tube diameter), by D and variant (1..4).
PAPER_TAYLOR_RE = {32: {1: 21.92, 2: 20.98, 3: 24.12, 4: 22.68},
                   64: {1: 23.77, 2: 22.86, 3: 25.35, 4: 23.96},
                   128: {1: 25.12, 2: 24.27, 3: 25.89, 4: 24.74}}


def taylor_reynolds(D=32, variant=I.OM, storage=I.F64, device="cuda:0", progress=None):
    """Re = D u / nu of the paper's Taylor bubble, u the rise velocity of the
    bubble's centre of mass (gas weight 1 - phi over gas and interface cells)
    between t* = 10 and t* = 15 (t* = t sqrt(g / D)). Returns a dict with Re,
    the two centroid heights, the steps and the run's status."""
    import torch

    from .fslbm import Simulation

    s = I.taylor_bubble_paper(D, variant=variant, storage=storage)
    p = s.params
    g = -p.gravity[2]
    nu = (p.tau - 0.5) / 3.0
    t10, t15 = (int(round(t / math.sqrt(g / D))) for t in (10.0, 15.0))
    z = (np.arange(p.n) // (p.nx * p.ny)).astype(np.float64) + 0.5
    stream = torch.cuda.Stream(device=device)
    with torch.cuda.stream(stream):
        sim = Simulation(s, device=device, stream=stream)

        def centroid():
            f = sim.fields(pdf=False, check=False)
            gas = (f["type"] == I.GAS) | (f["type"] == I.INTERFACE)
            w = np.where(gas, 1.0 - f["phi"], 0.0)
            return float((w * z).sum() / w.sum()), int(f["status"])

        def advance(n, done):
            chunk = 10000
            while n > 0:
                k = min(chunk, n)
                sim.step(k)
                n -= k
                done += k
                if progress:
                    progress(done)
            return done

        try:
            done = advance(t10, 0)
            z10, _ = centroid()
            advance(t15 - t10, done)
            z15, status = centroid()
        finally:
            sim.close()
    u = (z15 - z10) / (t15 - t10)
    return dict(Re=D * u / nu, z_centroid_t10=z10, z_centroid_t15=z15, steps=t15, status=status)


def wave_model(t_star, nu, k, omega0):
    """The paper's analytic surface elevation at x = 0 (Sec. 4.1): a*(0, t*) =
    exp(-2 nu k^2 t) cos(t*), t = t* / omega0."""
    t = np.asarray(t_star, dtype=np.float64) / omega0
    return np.exp(-2.0 * nu * k * k * t) * np.cos(np.asarray(t_star, dtype=np.float64))


def gravity_wave_elevation(L=200, variant=I.OM, storage=I.F64, t_end=40.0, dt_star=0.05,
                           device="cuda:0", progress=None):
    """The paper's gravity wave of wavelength L (Sec. 4.1) run to t* = t_end
    (t* = t omega0); every dt_star the surface elevation at the left border
    x = 0: the liquid height of a column (sum of fill levels over y) averaged
    over the two columns next to x = 0 (cells 0 and L - 1 of the periodic
    domain), minus the depth, over a0. Returns t*, the simulated and the
    model's a*, and the run's status."""
    import torch

    from .fslbm import Simulation

    s = I.gravity_wave_paper(L, variant=variant, storage=storage)
    p, m = s.params, s.meta
    omega0, nu, k = m["omega0"], m["nu"], m["k"]
    d, a0 = m["depth"], m["amp"]
    n_samples = int(round(t_end / dt_star))
    steps = [int(round(i * dt_star / omega0)) for i in range(n_samples + 1)]
    stream = torch.cuda.Stream(device=device)
    a_sim = np.zeros(n_samples + 1)
    status = 0
    with torch.cuda.stream(stream):
        sim = Simulation(s, device=device, stream=stream)

        def elevation():
            f = sim.fields(pdf=False, check=False)
            phi = np.where(f["type"] == I.LIQUID, 1.0,
                           np.where(f["type"] == I.INTERFACE, f["phi"], 0.0)).reshape(p.ny, p.nx)
            h = 0.5 * (phi[:, 0].sum() + phi[:, p.nx - 1].sum())
            return (h - d) / a0, int(f["status"])

        try:
            done = 0
            for i, st in enumerate(steps):
                if st > done:
                    sim.step(st - done)
                    done = st
                a_sim[i], status = elevation()
                if status:
                    a_sim[i + 1:] = np.nan
                    break
                if progress and i % max(1, n_samples // 8) == 0:
                    progress(i * dt_star)
        finally:
            sim.close()
    t_star = np.arange(n_samples + 1) * dt_star
    return dict(t_star=t_star, a_sim=a_sim, a_model=wave_model(t_star, nu, k, omega0),
                steps=steps[-1], status=status)


def wave_errors(r, windows=(6.0, 12.0, 24.0)):
    """Max and RMS of a*_sim - a*_model over t* in [0, w] for each window w."""
    out = {}
    for w in windows:
        sel = r["t_star"] <= w + 1e-9
        e = r["a_sim"][sel] - r["a_model"][sel]
        out["max_abs_err_t%g" % w] = float(np.max(np.abs(e)))
        out["rms_err_t%g" % w] = float(np.sqrt(np.mean(e * e)))
    return out


def paper_curve_distances(r, variant, L, curves, t_max=12.0):
    """Distances of a simulated elevation series r (gravity_wave_elevation) to
    the paper's own simulated series of the same variant and L (curves: the
    plotted series of the paper's convergence figures, {variant name: {L:
    [(t*, a*)]}}), and, for scale, the largest distance between the paper's
    series of this variant and of any other variant at the same L, each as the
    max and RMS over t* in (0, t_max]."""
    name = I.VARIANT_NAMES[variant]
    sel = (r["t_star"] > 0) & (r["t_star"] <= t_max + 1e-9) & np.isfinite(r["a_sim"])
    t = r["t_star"][sel]

    def on_t(v):
        p = np.asarray(curves[v][str(L)], dtype=np.float64)
        return np.interp(t, p[:, 0], p[:, 1])

    mine = on_t(name)
    d = r["a_sim"][sel] - mine
    others = [on_t(v) - mine for v in curves if v != name]
    return dict(max_to_paper=float(np.abs(d).max()), rms_to_paper=float(np.sqrt(np.mean(d * d))),
                paper_variant_spread_max=float(max(np.abs(o).max() for o in others)),
                paper_variant_spread_rms=float(max(np.sqrt(np.mean(o * o)) for o in others)))
