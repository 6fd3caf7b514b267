"""The paper's Taylor-bubble runs (Sec. 4.4) at tube diameters 32 and 64, all
four variants: the Reynolds number of the rising bubble against the paper's table,
and the variants in the paper's order (OM > OM3 > NBRC > NBKC). The paper's
gravity wave (Sec. 4.1) at wavelength 200: the surface elevation at x = 0
against the analytic model the paper compares with and against the paper's
own simulated series (tests/golden/gravity_wave_paper_curves.json)."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_taylor_bubble_reynolds_as_in_the_paper():
    from paper_2207_13962_amd.validation import PAPER_TAYLOR_RE, taylor_reynolds
    re = {}
    for v in (I.NBRC, I.NBKC, I.OM, I.OM3):
        r = taylor_reynolds(32, variant=v)
        assert r["status"] == 0
        re[v] = r["Re"]
        paper = PAPER_TAYLOR_RE[32][v]
        # the paper's own runs differ from each other by up to 15 % across
        # variants; the same setup here lands within 5 % of each
        assert abs(re[v] - paper) <= 0.05 * paper, (I.VARIANT_NAMES[v], re[v], paper)
    assert re[I.OM] > re[I.OM3] > re[I.NBRC] > re[I.NBKC]


@pytest.mark.timeout(900)
def test_taylor_bubble_reynolds_at_d64():
    """The same at tube diameter 64 (2.6 M cells, about 37 000 steps per
    variant): within 3 % of the paper's Re for every variant (measured: within
    1.9 %), and the paper's order of the variants."""
    from paper_2207_13962_amd.validation import PAPER_TAYLOR_RE, taylor_reynolds
    re = {}
    for v in (I.NBRC, I.NBKC, I.OM, I.OM3):
        r = taylor_reynolds(64, variant=v)
        assert r["status"] == 0
        re[v] = r["Re"]
        paper = PAPER_TAYLOR_RE[64][v]
        assert abs(re[v] - paper) <= 0.03 * paper, (I.VARIANT_NAMES[v], re[v], paper)
    assert re[I.OM] > re[I.OM3] > re[I.NBRC] > re[I.NBKC]


def test_gravity_wave_follows_the_analytic_model_and_the_papers_runs():
    """Besides the analytic model: the paper's own simulated elevation series
    of the same variant and L (its Sec. 4.1 convergence figures, golden
    fixture) lies closer to this run than the paper's series of the other
    variants lie to it (RMS and max over t* in (0, 12])."""
    import json
    import os
    from paper_2207_13962_amd.validation import gravity_wave_elevation, paper_curve_distances, wave_errors
    curves = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                         "gravity_wave_paper_curves.json")))["variants"]
    for v in (I.NBRC, I.NBKC, I.OM, I.OM3):
        r = gravity_wave_elevation(200, variant=v, t_end=12.0)
        dp = paper_curve_distances(r, v, 200, curves, t_max=12.0)
        # measured: RMS 0.046-0.064 against spreads of 0.12-0.19
        assert dp["rms_to_paper"] < dp["paper_variant_spread_rms"], (I.VARIANT_NAMES[v], dp)
        assert dp["max_to_paper"] < dp["paper_variant_spread_max"], (I.VARIANT_NAMES[v], dp)
        assert r["status"] == 0
        assert abs(r["a_sim"][0] - 1.0) < 1e-3
        e = wave_errors(r, windows=(12.0,))
        # at L = 200 the four variants stay within 0.16-0.30 of the model up
        # to t* = 12 (RMS 0.08-0.12); the error shrinks with L (0.10-0.15 at
        # L = 400, 0.08-0.13 at L = 800)
        assert e["max_abs_err_t12"] < 0.35 and e["rms_err_t12"] < 0.15, (I.VARIANT_NAMES[v], e)
        # the wave reverses: its first trough lies near t* = pi
        t, a = r["t_star"], r["a_sim"]
        trough = t[np.argmin(np.where(t < 2 * np.pi, a, np.inf))]
        assert abs(trough - np.pi) < 0.5, (I.VARIANT_NAMES[v], trough)
