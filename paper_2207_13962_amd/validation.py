"""Validation against the paper's own results: the Taylor-bubble runs of
Sec. 4.4 (tube diameter D, all four boundary-condition variants), whose
Reynolds numbers the paper tabulates. Every step runs in libfslbm; this module
builds the setup, samples the fill levels and reduces them to the rise
velocity."""
from __future__ import annotations

import math

import numpy as np

from . import inputs as I

# Reynolds numbers of the paper's Taylor-bubble runs (Sec. 4.4, table of Re by
# tube diameter), by D and variant (1..4).
PAPER_TAYLOR_RE = {32: {1: 21.92, 2: 20.98, 3: 24.12, 4: 22.68},
                   64: {1: 23.77, 2: 22.86, 3: 25.35, 4: 23.96},
                   128: {1: 25.12, 2: 24.27, 3: 25.89, 4: 24.74}}


def taylor_reynolds(D=32, variant=I.OM, storage=I.F64, device="cuda:0"):
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

        try:
            sim.step(t10)
            z10, _ = centroid()
            sim.step(t15 - t10)
            z15, status = centroid()
        finally:
            sim.close()
    u = (z15 - z10) / (t15 - t10)
    return dict(Re=D * u / nu, z_centroid_t10=z10, z_centroid_t15=z15, steps=t15, status=status)
