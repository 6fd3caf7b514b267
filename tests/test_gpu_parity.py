"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs. FP64 mode: identical cell types, populations, mass and fill
levels within 1e-12 relative."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

from ._parity import compare_state, mass_tol

pytestmark = pytest.mark.gpu

VARIANTS = [I.NBRC, I.NBKC, I.OM, I.OM3]


def _sim(setup, **kw):
    from paper_2207_13962_amd.fslbm import Simulation
    return Simulation(setup, **kw)


def _oracle(setup, **kw):
    from oracle import Oracle
    return Oracle(setup, **kw)


def test_initial_state_matches():
    s = I.gravity_wave()
    g, o = _sim(s), _oracle(s)
    compare_state(g, o, what="init")


@pytest.mark.parametrize("variant", VARIANTS)
def test_wave64_1000_steps(variant):
    """Standing wave 64x64x1, D3Q19 SRT FP64, 1000 steps: types identical every
    10 steps, full state within 1e-12 every 100 steps."""
    s = I.gravity_wave(variant=variant)
    g, o = _sim(s), _oracle(s)
    for block in range(10):
        for _ in range(10):
            g.step(10)
            assert o.step(10) == 0
            tg = g.fields(pdf=False)["type"]
            assert np.array_equal(tg, o.fields()["type"]), "types differ near step %d" % (
                o.mass().step)
        compare_state(g, o, what="variant %d step %d" % (variant, (block + 1) * 100))
    mg, mo = g.mass(), o.mass()
    assert abs(mg["total_mass"] - mo.total_mass) <= 1e-12 * mo.total_mass


MINI_CASES = [
    # (q, collision, side walls)
    (19, I.SRT, I.WALL_NOSLIP),
    (19, I.TRT, I.WALL_FREESLIP),
    (27, I.TRT, I.WALL_NOSLIP),
    (27, I.SRT, I.WALL_FREESLIP),
]


def _lockstep(g, o, steps, what, every=100):
    """Steps both codes one step at a time: cell types compared after every
    step, the full state (populations, masses, fill levels) every `every`."""
    for n in range(1, steps + 1):
        g.step(1)
        assert o.step(1) == 0, "%s: oracle unstable at step %d" % (what, n)
        tg, to = g.types(), o.types()
        if not np.array_equal(tg, to):
            c = int(np.nonzero(tg != to)[0][0])
            raise AssertionError("%s: types differ at step %d, first cell %d (gpu %d, oracle %d)"
                                 % (what, n, c, tg[c], to[c]))
        if n % every == 0:
            compare_state(g, o, what="%s step %d" % (what, n), mtol=mass_tol(n))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("q,coll,wall", MINI_CASES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_mini_dam_break(q, coll, wall, variant):
    """3D dam break 48x32x16 with many conversions, every lattice/collision/wall
    combination and every variant, 1000 steps: identical types after every
    step, populations within 1e-12 every 100 steps (masses and fill levels
    within the accumulation bound mass_tol)."""
    b = (wall, wall, I.WALL_NOSLIP, I.WALL_NOSLIP, wall, wall)
    s = I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=0.005, q=q, collision=coll,
                         storage=I.F64, boundary=b, variant=variant)
    g, o = _sim(s), _oracle(s)
    o.set_threads(8)
    g.set_graphs(False)  # one step per call: plain launches
    _lockstep(g, o, 1000, "q%d c%d w%d v%d" % (q, coll, wall, variant))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("variant", VARIANTS)
def test_droplet_impact_40(variant):
    """Drop impact 40^3 (periodic x, y): conversions around a moving drop,
    1000 steps, types after every step, full state every 100."""
    s = I.droplet_impact(L=40, velocity=0.04, storage=I.F64, variant=variant)
    g, o = _sim(s), _oracle(s)
    o.set_threads(8)
    g.set_graphs(False)
    _lockstep(g, o, 1000, "drop v%d" % variant)


def test_interface_list_sorted_and_complete():
    s = I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=0.005, storage=I.F64)
    g = _sim(s)
    for _ in range(5):
        g.step(37)
        lst = g.interface_list()
        t = g.fields(pdf=False)["type"]
        assert np.array_equal(lst, np.nonzero(t == I.INTERFACE)[0])


def test_lists_large_ragged_domain():
    """A domain of 8.6 M cells (525 compaction tiles; N is not a multiple of
    the tile or of the 64-cell chunk): after conversion-heavy steps the
    interface list equals the interface cells in ascending order and mass is
    conserved (a chunk missing from the liquid list would leave its cells
    unwritten)."""
    s = I.rect_dam_break(nx=515, ny=130, nz=129, wx=160, hy=100, g=2e-4, nu=2e-3, storage=I.F32,
                         variant=I.OM)
    g = _sim(s)
    m0 = g.mass()["total_mass"]
    for _ in range(3):
        g.step(40)
        r = g.mass()
        lst = g.interface_list()
        t = g.fields(pdf=False)["type"]
        assert np.array_equal(lst, np.nonzero(t == I.INTERFACE)[0])
        assert r["n_interface"] == lst.size
        assert abs(r["total_mass"] - m0) / m0 < 1e-6
    g.close()


def test_compaction_tile_sizes_identical():
    """Compaction tiles of 16, 32, 64 and 128 cells per thread - the packed
    and the separate scans of the list counts, one and two flag batches per
    thread, chunks shared by threads or held by one - give bitwise the same
    run on a ragged domain: types, fill levels, populations, interface list.
    Sizes below the library's choice or not 16 times a power of two are
    refused."""
    from paper_2207_13962_amd.fslbm import FslbmError
    s = I.rect_dam_break(nx=133, ny=70, nz=37, wx=40, hy=50, g=2e-4, nu=2e-3, storage=I.F32,
                         variant=I.OM)
    ref = None
    for per in (16, 32, 64, 128):
        g = _sim(s)
        if per == 16:
            for bad in (8, 48, 8192):
                with pytest.raises(FslbmError):
                    g.set_compaction_tile(bad)
        else:
            g.set_compaction_tile(per)
        g.step(60)
        f = g.fields(pdf=True)
        lst = g.interface_list()
        g.close()
        assert np.array_equal(lst, np.nonzero(f["type"] == I.INTERFACE)[0]), per
        if ref is None:
            ref = f
            continue
        for k in ("type", "phi", "mass", "pdf"):
            assert np.array_equal(f[k], ref[k]), (per, k)


def test_flat_rest_all_variants():
    for v in VARIANTS:
        for q in (19, 27):
            s = I.flat_interface_rest(q=q, variant=v)
            g, o = _sim(s), _oracle(s)
            g.step(20)
            assert o.step(20) == 0
            compare_state(g, o, what="rest q%d v%d" % (q, v))


@pytest.mark.parametrize("q,coll", [(19, I.TRT), (27, I.SRT)])
def test_mini_dam_break_smagorinsky(q, coll):
    """Dam break with the Smagorinsky model on (C_S = 0.1, as used for the
    paper's dam breaks, Sec. 2.1) at low viscosity: 1e-12 parity, 300 steps."""
    s = I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=1e-4, q=q, collision=coll,
                         storage=I.F64, variant=I.OM)
    s.params = s.params.with_(smagorinsky=0.1)
    g, o = _sim(s), _oracle(s)
    for k in range(6):
        g.step(50)
        assert o.step(50) == 0
        compare_state(g, o, what="les q%d c%d step %d" % (q, coll, 50 * (k + 1)))


@pytest.mark.parametrize("layout", [I.TWO_GRID, I.AA])
def test_variant_switch_mid_run(layout):
    """fslbm_set_variant between steps: a dam break that changes its variant
    three times (after step counts of both parities, with replayed graphs)
    against the oracle switching at the same steps."""
    s = I.rect_dam_break(nx=40, ny=28, nz=12, wx=14, hy=20, g=2e-4, nu=5e-3, storage=I.F64, variant=I.NBRC)
    s.params = s.params.with_(layout=layout)
    g, o = _sim(s), _oracle(s)
    done = 0
    for n, v in ((37, I.OM3), (24, I.NBKC), (51, I.OM), (40, None)):
        g.step(n)
        assert o.step(n) == 0
        done += n
        compare_state(g, o, what="switch step %d" % done, mtol=mass_tol(done))
        if v is not None:
            g.set_variant(v)
            o.set_variant(v)
    g.close()
