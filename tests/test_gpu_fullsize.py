"""Parity and properties at the measured workloads' full sizes.

* dam256 with the Smagorinsky model, as the benchmark runs it (graph replay on
  a non-default stream), in FP64 mode against the oracle, all four variants;
* taylor512 (D3Q27, surface tension, bubble model) in FP64 mode against the
  oracle;
* cyl256 (D3Q27 TRT, free-slip walls, 8.4 M cells) in FP32: mass conservation,
  the interface list, and the mirror symmetries of the setup (in bulk); the
  same run in FP64: the symmetries to rounding, and 24 steps against the oracle;
* dam256 in FP64 after 600 steps against the oracle, then 20 more steps from
  the oracle's own state loaded through the resume path."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

from ._parity import compare_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [I.NBRC, I.NBKC, I.OM, I.OM3])
def test_dam256_fp64_les_parity(variant):
    import torch
    from oracle import Oracle
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("dam256", smagorinsky=0.1, storage=I.F64, variant=variant)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = Simulation(s, stream=stream)
        g.step(16)  # two replays of the 8-step graph
        stream.synchronize()
        o = Oracle(s)
        assert o.step(16) == 0
        compare_state(g, o, what="dam256 v%d" % variant)
        g.close()


def test_taylor512_fp64_parity():
    from oracle import Oracle
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("taylor512", storage=I.F64)
    g, o = Simulation(s), Oracle(s)
    g.step(4)
    assert o.step(4) == 0
    compare_state(g, o, what="taylor512")
    rg, ro = g.mass(), o.mass()
    assert abs(rg["bubble_volume"] - ro.bubble_volume) <= 1e-12 * ro.bubble_volume
    assert abs(rg["p_volume"] - ro.p_volume) <= 1e-12 * ro.p_volume
    g.close()


def _mirror_diffs(f, p):
    """(share of cells whose type differs, |phi| differences over the cells
    that are interface on both sides) for the x mirror, the y mirror and the
    x <-> y swap."""
    t3 = f["type"].reshape(p.nz, p.ny, p.nx)
    phi = f["phi"].reshape(p.nz, p.ny, p.nx)
    out = []
    for mt, mp in ((t3[:, :, ::-1], phi[:, :, ::-1]), (t3[:, ::-1, :], phi[:, ::-1, :]),
                   (t3.transpose(0, 2, 1), phi.transpose(0, 2, 1))):
        same = mt == t3
        both_if = same & (t3 == I.INTERFACE)
        out.append((1.0 - same.mean(), np.abs(mp[both_if] - phi[both_if])))
    return out


def test_cyl256_fp32_properties():
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("cyl256")
    g = Simulation(s)
    m0 = g.mass()["total_mass"]
    g.step(300)
    r = g.mass()
    f = g.fields(pdf=False)
    lst = g.interface_list()
    g.close()
    assert r["status"] == 0
    assert abs(r["total_mass"] - m0) / m0 < 1e-6
    assert np.array_equal(lst, np.nonzero(f["type"] == I.INTERFACE)[0])
    assert r["n_interface"] == lst.size
    # the column is centred between cells, so the run is mirror symmetric in
    # x and y and symmetric under x <-> y up to rounding. In FP32 the sums on
    # the two sides run in different orders; a conversion that one rounding
    # puts a step earlier on one side then perturbs its neighbourhood, so the
    # bound is on the bulk (99 % of the interface cells) and on how many cells
    # are off (the FP64 run below is symmetric to rounding everywhere).
    for differ, dphi in _mirror_diffs(f, s.params):
        assert differ < 1e-5
        assert np.quantile(dphi, 0.99) < 2e-5
        assert (dphi > 1e-3).mean() < 5e-3


def test_cyl256_fp64_symmetry():
    """The same run with FP64 populations: types identical and fill levels
    equal to 1e-11 under both mirrors and the swap."""
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("cyl256", storage=I.F64)
    g = Simulation(s)
    m0 = g.mass()["total_mass"]
    g.step(300)
    r = g.mass()
    f = g.fields(pdf=False)
    g.close()
    assert r["status"] == 0
    assert abs(r["total_mass"] - m0) / m0 < 1e-12
    for differ, dphi in _mirror_diffs(f, s.params):
        assert differ == 0.0
        assert dphi.max() < 1e-11


def test_cyl256_fp32_against_fp64():
    """The conversion-heavy cylindrical collapse in FP32 against the same run
    in FP64 (which matches the oracle: test_cyl256_fp64_oracle_parity), after
    300 steps. Where a fill level lies within rounding of a conversion
    threshold the two runs convert that cell a step apart, and in the
    spreading film such differences grow (measured: 0.007 % of the cells of
    another type, 186 of 28 600 interface cells; the cells interface in both
    have a median |phi difference| of 2e-5 but a 99th percentile of 0.14), so
    the comparison is on what such shifts leave alone: the front on the floor
    within one cell (measured 0.03), at least 99.9 % of the cells of the same
    type, the median fill-level difference below 1e-3, and the total mass
    within 1e-6 relative (measured 1.5e-9)."""
    from paper_2207_13962_amd.fslbm import Simulation
    out = {}
    for st in (I.F64, I.F32):
        s = I.workload("cyl256", storage=st)
        g = Simulation(s)
        g.step(300)
        out[st] = (g.fields(pdf=False), g.mass())
        g.close()
    p = I.workload("cyl256").params
    (f64, r64), (f32, r32) = out[I.F64], out[I.F32]
    assert r64["status"] == r32["status"] == 0

    def front(f):
        t = f["type"].reshape(p.nz, p.ny, p.nx)[0]
        y, x = np.nonzero((t == I.LIQUID) | (t == I.INTERFACE))
        return np.sqrt((x + 0.5 - p.nx / 2.0) ** 2 + (y + 0.5 - p.ny / 2.0) ** 2).max()
    assert abs(front(f32) - front(f64)) <= 1.0, (front(f32), front(f64))
    assert (f32["type"] == f64["type"]).mean() >= 0.999
    assert abs(r32["total_mass"] - r64["total_mass"]) <= 1e-6 * r64["total_mass"]
    both = (f32["type"] == I.INTERFACE) & (f64["type"] == I.INTERFACE)
    assert np.median(np.abs(f32["phi"][both] - f64["phi"][both])) < 1e-3


@pytest.mark.timeout(900)
def test_cyl256_fp64_oracle_parity():
    """cyl256 (D3Q27 TRT, free-slip sides and ceiling, no-slip floor, 8.4 M
    cells) in FP64 mode against the oracle: 24 steps (three replays of the
    8-step graph), identical types, populations, masses and fill levels within
    1e-12."""
    from oracle import Oracle
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("cyl256", storage=I.F64, variant=I.NBRC)
    g = Simulation(s)
    o = Oracle(s)
    g.step(24)
    assert o.step(24) == 0
    compare_state(g, o, what="cyl256")
    rg, ro = g.mass(), o.mass()
    assert abs(rg["total_mass"] - ro.total_mass) <= 1e-12 * ro.total_mass
    g.close()


@pytest.mark.timeout(1200)
def test_dam256_collapse_parity_and_resume():
    """dam256 as the benchmark runs it (Smagorinsky model, graph replay on a
    non-default stream) in FP64 mode: after 600 steps, deep into the
    collapse with tens of conversions per step, the GPU run and the oracle
    agree (identical types, populations, masses, fill levels within 1e-12).
    Then the oracle's own state at step 600 - post-collision populations,
    masses, fill levels, types, lost mass - is loaded into a new GPU context
    (fslbm_create with pdf and mass, fslbm_set_scalars) and both codes take 20
    more steps: again identical within 1e-12."""
    import torch
    from oracle import Oracle
    from paper_2207_13962_amd.fslbm import Simulation
    s = I.workload("dam256", smagorinsky=0.1, storage=I.F64, variant=I.OM)
    o = Oracle(s)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = Simulation(s, stream=stream)
        g.step(600)
        assert o.step(600) == 0
        compare_state(g, o, what="dam256 step 600")
        mg, mo = g.mass(), o.mass()
        assert abs(mg["total_mass"] - mo.total_mass) <= 1e-12 * mo.total_mass
        g.close()
        st = o.export_state()
        f = o.fields()
        init = I.Setup(s.params, st["type"], st["phi"], f["rho"], f["ux"], f["uy"], f["uz"])
        r = Simulation(init, pdf=o.post_collision(), mass=st["mass"], stream=stream)
        r.set_scalars(st["lost_mass"], st["p_volume"], st["p_volume0"], st["volume0"])
        r.step(20)
        assert o.step(20) == 0
        compare_state(r, o, what="dam256 resumed from the oracle at step 600, +20")
        mr, mo = r.mass(), o.mass()
        assert abs(mr["total_mass"] - mo.total_mass) <= 1e-12 * mo.total_mass
        r.close()
