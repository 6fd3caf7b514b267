"""Tracked bubbles (bubble model 2) on the GPU against the oracle: the
bubbles (labels identical; volumes and pressures within 1e-12) and the full
state, through coalescence, segmentation, periodic faces and a closed box
of rising bubbles spanning many blocks."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

from ._parity import compare_state

pytestmark = pytest.mark.gpu


def _pair(setup):
    from oracle import Oracle
    from paper_2207_13962_amd.fslbm import Simulation
    return Simulation(setup), Oracle(setup)


# Volumes and pressures to the FP64 state tolerance (the amounts are handed
# over exactly where bubbles neither merge nor split, volumes are sums of
# 1 - phi); labels are integers: identical.
RTOL_BUBBLE = 1e-12


def _same_bubbles(g, o, what):
    lg, vg, pg = g.bubbles()
    lo, vo, po = o.bubbles()
    assert list(lg) == list(lo), (what, list(lg), list(lo))
    np.testing.assert_allclose(vg, vo, rtol=RTOL_BUBBLE, atol=1e-12, err_msg=what)
    np.testing.assert_allclose(pg, po, rtol=RTOL_BUBBLE, err_msg=what)
    return len(lo)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("kind,periodic,count", [("apart", False, (2, 2)), ("merge", False, (2, 1)),
                                                 ("split", False, (1, 2)), ("straddle", True, (1, 1)),
                                                 ("straddle", False, (2, 2))])
def test_bubble_events_match_oracle(q, kind, periodic, count):
    s = I.bubble_pair(kind, q=q, periodic_x=periodic, g=1e-4)
    g, o = _pair(s)
    assert _same_bubbles(g, o, "init") == count[0]
    g.step(1)
    assert o.step(1) == 0
    assert _same_bubbles(g, o, "step 1") == count[1]
    compare_state(g, o, what="%s q%d step 1" % (kind, q))
    g.step(29)
    o.step(29)
    _same_bubbles(g, o, "step 30")
    compare_state(g, o, what="%s q%d step 30" % (kind, q))


def test_bubbles_at_rest_keep_their_labels():
    # a flat interface at rest marks no cell in any step: the labelling
    # passes are skipped and the bubble (the gas above) carried over
    s = I.flat_interface_rest(nx=16, ny=12, nz=8)
    s.params = s.params.with_(bubble_model=2)
    g, o = _pair(s)
    lab0, v0, p0 = g.bubbles()
    g.step(30)
    assert o.step(30) == 0
    lab, v, p = g.bubbles()
    assert list(lab) == list(lab0)
    np.testing.assert_allclose(p * v, p0 * v0, rtol=1e-14)
    _same_bubbles(g, o, "step 30")
    compare_state(g, o, what="flat rest step 30")


@pytest.mark.parametrize("variant", [I.NBRC, I.OM])
def test_bubbly_column_matches_oracle(variant):
    # 48 x 40 x 56 cells (420 blocks per pass), six bubbles including the gas
    # above the surface of the closed box
    s = I.bubbly_column(variant=variant)
    g, o = _pair(s)
    assert _same_bubbles(g, o, "init") == 6
    for k in range(3):
        g.step(20)
        o.step(20)
        _same_bubbles(g, o, "step %d" % (20 * (k + 1)))
        compare_state(g, o, what="bubbly column step %d" % (20 * (k + 1)))
    lab, v, p = g.bubbles()
    assert np.all(p > 0.333) and np.all(p < 0.34)


def test_one_bubble_is_the_single_bubble_model_on_gpu():
    from paper_2207_13962_amd.fslbm import Simulation
    s2 = I.bubble_pair("straddle", periodic_x=True, g=2e-4)
    s1 = I.Setup(s2.params.with_(bubble_model=1), s2.type, s2.phi, s2.rho, s2.ux, s2.uy, s2.uz)
    g1, g2 = Simulation(s1), Simulation(s2)
    g1.step(30)
    g2.step(30)
    lab, v, p = g2.bubbles()
    assert len(lab) == 1
    assert p[0] == pytest.approx(g1.mass()["p_volume"], rel=1e-12)
    f1, f2 = g1.fields(), g2.fields()
    assert np.array_equal(f1["type"], f2["type"])
    np.testing.assert_allclose(f2["pdf"], f1["pdf"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("case", ["taylor", "column"])
def test_tracked_bubbles_with_surface_tension(case):
    # the curvature pass adds the Laplace term to each interface cell's own
    # bubble pressure: D3Q27 TRT rising bubble in a tube of obstacle cells,
    # and the box of rising bubbles, both with sigma = 1e-3
    if case == "taylor":
        s = I.taylor_bubble(nx=24, ny=24, nz=64, tube_radius=10.5, bubble_radius=6.0, z0=16.0, length=16.0,
                            g=1e-5, nu=0.01, sigma=1e-3, storage=I.F64, variant=I.OM)
        s.params = s.params.with_(bubble_model=2)
    else:
        s = I.bubbly_column(variant=I.NBKC)
        s.params = s.params.with_(sigma=1e-3)
    g, o = _pair(s)
    _same_bubbles(g, o, "init")
    for k in range(2):
        g.step(25)
        assert o.step(25) == 0
        _same_bubbles(g, o, "step %d" % (25 * (k + 1)))
        compare_state(g, o, what="%s sigma step %d" % (case, 25 * (k + 1)))


def test_tracked_bubbles_are_reproducible():
    """The per-bubble totals are built from atomic adds of many waves, as
    integer parts and 2^-64 fractions added exactly, so two runs of the same
    bubbly column (six bubbles, 420 blocks per pass, rising and deforming)
    agree bitwise: labels, volumes, pressures, populations, fill levels."""
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.bubbly_column(variant=I.OM)
    runs = []
    for _ in range(2):
        g = Simulation(s)
        g.step(60)
        f = g.fields(pdf=True)
        runs.append((g.bubbles(), f))
        g.close()
    (b0, f0), (b1, f1) = runs
    for x, y in zip(b0, b1):
        assert np.array_equal(x, y)
    for key in ("type", "phi", "mass", "pdf"):
        assert np.array_equal(f0[key], f1[key]), key
