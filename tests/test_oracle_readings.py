"""Pins of the oracle's readings of what the paper delegates to cited work.

The paper states the forced fill/empty modification of the mass flux, the
reinitialisation of new interface cells, the excess-mass fallback and the
free-slip condition only by intent or by reference (Sec. 2.1 walls; Sec. 2.2
mass flux, conversion, reinitialisation and excess-mass equation). Each test
below checks the oracle against a consequence of that stated intent which a
plausible mistake in the reading would break:

* forced fill/empty: a cell that should empty only gives mass to interface
  neighbours of another class, one that should fill only receives, and the
  modification moves no mass in total (swapping the two roles keeps the
  table antisymmetric, so conservation alone cannot see it);
* reinitialisation: a new interface cell from gas carries the equilibrium at
  the mean density and mean (half-force shifted) velocity of its liquid and
  old interface neighbours after streaming, and of no other cells;
* excess mass with no interface neighbour: booked exactly into the lost-mass
  counter, total mass unchanged;
* free-slip walls (faces and edges): tangential momentum of a liquid sliding
  along them is conserved to round-off (no-slip walls must lose it);
* a flat free surface at rest under gravity with hydrostatic initialisation
  stays at rest (velocities of order g) and at the gas density, all variants.

Plus properties of the oracle as a program: the same result for any thread
count, a verbatim export/import that continues a run bitwise, and a clean run
under AddressSanitizer and UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import Oracle, equilibrium, lattice
from oracle.oracle import GCC_FLAGS, _HERE as ORACLE_DIR
from paper_2207_13962_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
P = I.PERIODIC


def _setup(p, t, phi, rho, u):
    n = p.n
    ux, uy, uz = (np.ascontiguousarray(a, dtype=np.float64) for a in u)
    return I.Setup(p, np.ascontiguousarray(t, dtype=np.uint8), np.ascontiguousarray(phi, dtype=np.float64),
                   np.ascontiguousarray(rho, dtype=np.float64), ux.reshape(n), uy.reshape(n), uz.reshape(n))


def _grid(p):
    k, j, i = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def _stencil(p, q):
    """Neighbour index arrays (q-1, N) of the velocity set on a periodic box."""
    c, _ = lattice(q)
    i, j, k = _grid(p)
    nb = []
    for d in c[1:]:
        nb.append(((i + d[0]) % p.nx) + p.nx * (((j + d[1]) % p.ny) + p.ny * ((k + d[2]) % p.nz)))
    return np.array(nb)


# ----------------------------------------------------------------------------
# forced fill/empty (Sec. 2.2: the mass flux is modified so that interface
# cells without liquid neighbours empty and those without gas neighbours fill)
# ----------------------------------------------------------------------------

def _random_surface(q, seed, n=12):
    """A periodic box with a random, closed interface layer: every class of
    interface cell occurs (no liquid neighbour, no gas neighbour, both).
    Conversions are switched off (eps_phi huge) so that one step changes the
    masses by the flux alone."""
    rng = np.random.default_rng(seed)
    p = I.Params(n, n, n, q=q, collision=I.SRT, tau=0.8, boundary=(P,) * 6, variant=I.OM,
                 thurey_flux=1, eps_phi=50.0)
    i, j, k = _grid(p)
    a = rng.uniform(0, 2 * np.pi, 3)
    phi = (0.45 + 0.9 * np.sin(2 * np.pi * i / n + a[0]) * np.cos(2 * np.pi * j / n + a[1])
           + 0.6 * np.sin(2 * np.pi * k / n + a[2]) + rng.uniform(-0.5, 0.5, p.n))
    t, phi = I.types_from_fill(phi, p)
    phi = np.where(t == I.INTERFACE, np.maximum(phi, 0.05), np.where(t == I.LIQUID, 1.0, 0.0))
    rho = rng.uniform(0.98, 1.02, p.n)
    u = rng.uniform(-0.02, 0.02, (3, p.n))
    return _setup(p, t, phi, rho, u)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_forced_fill_empty_direction(q, seed):
    s = _random_surface(q, seed)
    p = s.params
    on, off = Oracle(s), Oracle(_setup(p.with_(thurey_flux=0), s.type, s.phi, s.rho, (s.ux, s.uy, s.uz)))
    i, j, k = _grid(p)
    t0 = s.type
    cls = np.full(p.n, -1)
    for c in np.nonzero(t0 == I.INTERFACE)[0]:
        cls[c] = on.flux_class(int(i[c]), int(j[c]), int(k[c]))
    # the classes follow their definition (liquid / gas neighbours at t)
    nb = _stencil(p, q)
    has_liq = (t0[nb] == I.LIQUID).any(axis=0)
    has_gas = (t0[nb] == I.GAS).any(axis=0)
    ifc = t0 == I.INTERFACE
    want = np.where(has_gas & ~has_liq, 1, np.where(has_liq & ~has_gas, 2, 0))
    assert np.array_equal(cls[ifc], want[ifc])
    assert on.step(1) == 0 and off.step(1) == 0
    a, b = on.export_state(), off.export_state()
    assert np.array_equal(a["type"], t0) and np.array_equal(b["type"], t0)  # no conversion
    diff = a["mass"] - b["mass"]
    NOLIQ, NOGAS, STD = 1, 2, 0
    checked = {"empty": 0, "fill": 0, "std_recv": 0, "std_give": 0, "zero": 0}
    for c in np.nonzero(ifc)[0]:
        nbc = {int(cls[x]) for x in nb[:, c] if t0[x] == I.INTERFACE}
        other = nbc - {int(cls[c])}
        if not other:
            assert diff[c] == 0.0  # equal classes exchange as without the rule
            checked["zero"] += 1
        elif cls[c] == NOLIQ:
            assert diff[c] < 0.0  # should empty: only gives
            checked["empty"] += 1
        elif cls[c] == NOGAS:
            assert diff[c] > 0.0  # should fill: only receives
            checked["fill"] += 1
        elif other == {NOLIQ}:
            assert diff[c] > 0.0  # neighbours that empty give to it
            checked["std_recv"] += 1
        elif other == {NOGAS}:
            assert diff[c] < 0.0  # neighbours that fill take from it
            checked["std_give"] += 1
    assert min(checked.values()) > 0, checked
    # the modification moves no mass in total (antisymmetric in the pair)
    assert abs(diff.sum()) < 1e-13


# ----------------------------------------------------------------------------
# reinitialisation of new interface cells from gas (Sec. 2.2)
# ----------------------------------------------------------------------------

def _filling_layer(q, seed, g=1e-3):
    """Liquid below y = 4, an interface layer at y = 4 in which most cells are
    over-full (they convert to liquid in the first step) and some are half
    full (they stay interface), gas above; random densities and velocities so
    that neighbours differ."""
    rng = np.random.default_rng(seed)
    n = 8
    p = I.Params(n, n, n, q=q, collision=I.SRT, tau=0.9, boundary=(P, P, I.WALL_NOSLIP, I.WALL_NOSLIP, P, P),
                 variant=I.OM, gravity=(0.0, -g, 0.0))
    i, j, k = _grid(p)
    t = np.where(j < 4, I.LIQUID, np.where(j == 4, I.INTERFACE, I.GAS)).astype(np.uint8)
    full = rng.uniform(0, 1, p.n) < 0.75
    phi = np.where(j < 4, 1.0, np.where(j == 4, np.where(full, 1.3, 0.5), 0.0))
    rho = rng.uniform(0.95, 1.05, p.n)
    u = rng.uniform(-0.03, 0.03, (3, p.n))
    return _setup(p, t, phi, rho, u)


@pytest.mark.parametrize("q", [19, 27])
def test_reinit_from_gas_averages(q):
    g = 1e-3
    s = _filling_layer(q, 5, g)
    p = s.params
    o = Oracle(s)
    t0 = s.type.copy()
    assert o.step(1) == 0
    f = o.fields()
    t1 = f["type"]
    c, _ = lattice(q)
    i, j, k = _grid(p)
    new_gas = (t0 == I.GAS) & (t1 == I.INTERFACE)
    assert new_gas.sum() > 0
    contrast = 0
    for cell in np.nonzero(new_gas)[0]:
        allowed, excluded = [], []
        for d in c[1:]:
            y = j[cell] + d[1]
            if y < 0 or y >= p.ny:
                continue  # wall
            nbi = ((i[cell] + d[0]) % p.nx) + p.nx * (y + p.ny * ((k[cell] + d[2]) % p.nz))
            if t1[nbi] in (I.LIQUID, I.INTERFACE):
                (excluded if t0[nbi] == I.GAS else allowed).append(nbi)
        allowed = np.array(allowed)
        assert allowed.size > 0
        # neighbour moments after streaming, velocity with the half-force shift
        pdf = f["pdf"][:, allowed]
        r = pdf.sum(axis=0)
        uu = ((c.T @ pdf) + 0.5 * r * np.array([0.0, -g, 0.0])[:, None]) / r
        rbar, ubar = r.mean(), uu.mean(axis=1)
        assert abs(f["rho"][cell] - rbar) < 1e-14
        # pre-collision velocity of an equilibrium at ubar is ubar + g/2
        got = np.array([f["ux"][cell], f["uy"][cell], f["uz"][cell]])
        assert np.allclose(got, ubar + 0.5 * np.array([0.0, -g, 0.0]), rtol=0, atol=1e-15)
        assert np.allclose(f["pdf"][:, cell], equilibrium(q, rbar, ubar), rtol=0, atol=1e-15)
        # the excluded new neighbours would have changed the result
        if len(excluded):
            pe = f["pdf"][:, np.concatenate([allowed, excluded])]
            if abs(pe.sum(axis=0).mean() - rbar) > 1e-6:
                contrast += 1
    assert contrast > 0


# ----------------------------------------------------------------------------
# excess mass without an interface neighbour (Sec. 2.2, excess-mass equation)
# ----------------------------------------------------------------------------

def _box(q, n=7, t_fill=I.GAS):
    p = I.Params(n, n, n, q=q, collision=I.SRT, tau=0.8, boundary=(P,) * 6, variant=I.OM)
    t = np.full(p.n, t_fill, dtype=np.uint8)
    phi = np.where(t == I.LIQUID, 1.0, 0.0)
    return p, t, phi


@pytest.mark.parametrize("q", [19, 27])
def test_lost_mass_emptied_cell_without_interface_neighbour(q):
    """An interface cell alone in gas whose fill level is below -eps empties;
    no interface cell is left around it, so its whole mass m goes to the lost
    mass, exactly."""
    p, t, phi = _box(q)
    c0 = p.n // 2
    t[c0] = I.INTERFACE
    phi[c0] = -0.05
    rho = np.full(p.n, 1.0)
    rho[c0] = 1.01
    s = _setup(p, t, phi, rho, np.zeros((3, p.n)))
    o = Oracle(s)
    m0 = o.export_state()["mass"][c0]
    assert m0 == -0.05 * 1.01
    assert o.step(1) == 0
    r = o.mass()
    assert (o.fields()["type"] == I.GAS).all()
    assert r.lost_mass == m0          # booked exactly
    assert r.total_mass == m0         # nothing else holds mass


@pytest.mark.parametrize("q", [19, 27])
def test_lost_mass_filled_cell_inside_liquid(q):
    """An over-full interface cell with only liquid around it fills; no
    interface neighbour receives its excess, which goes to the lost mass:
    total mass is unchanged and the lost mass is m - rho of the cell."""
    p, t, phi = _box(q, t_fill=I.LIQUID)
    c0 = p.n // 2
    t[c0] = I.INTERFACE
    phi[c0] = 1.5
    s = _setup(p, t, phi, np.full(p.n, 1.0), np.zeros((3, p.n)))
    o = Oracle(s)
    M0 = o.mass().total_mass
    assert o.step(1) == 0
    r = o.mass()
    assert (o.fields()["type"] == I.LIQUID).all()
    assert 0.45 < r.lost_mass < 0.55
    assert abs(r.total_mass - M0) < 1e-13 * M0


def test_excess_goes_to_interface_neighbour_not_lost():
    """The same emptying cell with one interface neighbour: nothing is lost,
    the neighbour ends with both cells' mass."""
    p, t, phi = _box(19)
    c0 = p.n // 2
    t[c0], t[c0 + 1] = I.INTERFACE, I.INTERFACE
    phi[c0], phi[c0 + 1] = -0.05, 0.4
    s = _setup(p, t, phi, np.ones(p.n), np.zeros((3, p.n)))
    o = Oracle(s)
    m = o.export_state()["mass"]
    assert o.step(1) == 0
    st, r = o.export_state(), o.mass()
    assert st["type"][c0] == I.GAS and st["type"][c0 + 1] == I.INTERFACE
    assert r.lost_mass == 0.0
    assert abs(st["mass"][c0 + 1] - (m[c0] + m[c0 + 1])) < 1e-15


# ----------------------------------------------------------------------------
# free-slip walls (Sec. 2.1: the wall-normal velocity component is reversed)
# ----------------------------------------------------------------------------

def _momentum(o, q):
    c, _ = lattice(q)
    f = o.fields()["pdf"]
    return c.T @ f.sum(axis=1)


@pytest.mark.parametrize("q,coll,walls", [
    (19, I.SRT, "y"),        # two free-slip faces
    (19, I.TRT, "yz"),       # four faces, edges where two meet
    (27, I.TRT, "yz"),       # D3Q27: corner directions reflected at both faces of an edge
])
def test_free_slip_keeps_tangential_momentum(q, coll, walls):
    nx, ny, nz = 8, 6, 5
    b = [P, P, P, P, P, P]
    for a in walls:
        ax = "xyz".index(a)
        b[2 * ax] = b[2 * ax + 1] = I.WALL_FREESLIP
    p = I.Params(nx, ny, nz, q=q, collision=coll, tau=0.8, boundary=tuple(b), variant=I.OM)
    rng = np.random.default_rng(11)
    u = np.zeros((3, p.n))
    u[0] = 0.04 + 0.005 * rng.standard_normal(p.n)   # along x: tangential to every wall
    if "z" not in walls:
        u[2] = 0.01
    s = _setup(p, np.full(p.n, I.LIQUID), np.ones(p.n), 1.0 + 0.01 * rng.standard_normal(p.n), u)
    o = Oracle(s)
    P0 = _momentum(o, q)
    assert o.step(200) == 0
    P1 = _momentum(o, q)
    assert abs(P1[0] - P0[0]) < 1e-12 * abs(P0[0])
    if "z" not in walls:
        assert abs(P1[2] - P0[2]) < 1e-12 * abs(P0[2])
    # the same box with no-slip walls loses its momentum to the walls
    s2 = _setup(p.with_(boundary=tuple(I.WALL_NOSLIP if x == I.WALL_FREESLIP else x for x in b)),
                s.type, s.phi, s.rho, (s.ux, s.uy, s.uz))
    o2 = Oracle(s2)
    assert o2.step(200) == 0
    assert _momentum(o2, q)[0] < 0.8 * P0[0]


# ----------------------------------------------------------------------------
# flat free surface at rest under gravity
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [I.NBRC, I.NBKC, I.OM, I.OM3])
@pytest.mark.parametrize("q", [19, 27])
def test_flat_surface_under_gravity_stays_at_rest(variant, q):
    """Liquid below a flat interface layer (fill level 1/2), gas above,
    g = 1e-5 towards -y, densities hydrostatic with the gas pressure at the
    surface (y = 12.5): over 1000 steps the velocities stay of the order of g
    (a wrong condition or force would set the surface moving with velocities
    of order sqrt(g h) ~ 1e-2) and the interface density stays at rho^G."""
    g = 1e-5
    nx, ny, nz, level = 12, 24, 2, 12
    p = I.Params(nx, ny, nz, q=q, collision=I.SRT, tau=0.8,
                 boundary=(P, P, I.WALL_NOSLIP, I.WALL_NOSLIP, P, P), variant=variant,
                 gravity=(0.0, -g, 0.0))
    i, j, k = _grid(p)
    t = np.where(j < level, I.LIQUID, np.where(j == level, I.INTERFACE, I.GAS)).astype(np.uint8)
    phi = np.where(j < level, 1.0, np.where(j == level, 0.5, 0.0))
    rho = I.hydrostatic_rho(p, level + 0.5, 1, g)
    o = Oracle(_setup(p, t, phi, rho, np.zeros((3, p.n))))
    umax, drho = 0.0, 0.0
    for _ in range(10):
        assert o.step(100) == 0
        f = o.fields()
        fl = (f["type"] == I.LIQUID) | (f["type"] == I.INTERFACE)
        umax = max(umax, float(np.sqrt(f["ux"] ** 2 + f["uy"] ** 2 + f["uz"] ** 2)[fl].max()))
        ifc = f["type"] == I.INTERFACE
        drho = max(drho, float(np.abs(f["rho"][ifc] - 1.0).max()))
        assert np.array_equal(f["type"], t)  # the surface stays in its layer
    assert umax < 2.0 * g
    assert drho < 5.0 * g


# ----------------------------------------------------------------------------
# the oracle as a program
# ----------------------------------------------------------------------------

def test_thread_count_does_not_change_the_result():
    s = I.rect_dam_break(nx=40, ny=24, nz=12, wx=12, hy=18, g=2e-4, nu=5e-3, collision=I.TRT,
                         storage=I.F64, variant=I.NBKC)
    a, b = Oracle(s), Oracle(s)
    a.set_threads(1)
    b.set_threads(4)
    assert a.step(80) == 0 and b.step(80) == 0
    sa, sb = a.export_state(), b.export_state()
    for key in ("type", "pdf", "mass", "phi"):
        assert np.array_equal(sa[key], sb[key]), key
    assert sa["lost_mass"] == sb["lost_mass"]


@pytest.mark.parametrize("bubble", [0, 1])
def test_export_import_continues_bitwise(bubble):
    s = I.rect_dam_break(nx=40, ny=24, nz=12, wx=12, hy=18, g=2e-4, nu=5e-3, collision=I.TRT,
                         storage=I.F64, variant=I.OM3)
    s.params = s.params.with_(bubble_model=bubble)
    ref = Oracle(s)
    assert ref.step(60) == 0
    part = Oracle(s)
    assert part.step(30) == 0
    st = part.export_state()
    fresh = Oracle(s)
    fresh.import_state(st, step=30)
    assert fresh.step(30) == 0
    a, b = ref.export_state(), fresh.export_state()
    for key in ("type", "pdf", "mass", "phi"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("lost_mass", "p_volume", "p_volume0", "volume0"):
        assert a[key] == b[key], key
    assert fresh.mass().step == 60


def _write_case(d, name, s, steps):
    p = s.params
    ints = [p.nx, p.ny, p.nz, p.q, p.collision, *p.boundary, p.variant, p.thurey_flux, p.bubble_model, steps]
    dbl = [p.tau, p.trt_lambda, *p.gravity, p.rho_gas, p.sigma, p.eps_phi, p.tie_delta or 1e-9,
           p.smagorinsky]
    with open(os.path.join(d, name), "wb") as fh:
        fh.write(np.array(ints, dtype=np.int32).tobytes())
        fh.write(np.array(dbl, dtype=np.float64).tobytes())
        fh.write(s.type.astype(np.uint8).tobytes())
        for a in (s.phi, s.rho, s.ux, s.uy, s.uz):
            fh.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    """The oracle built with -fsanitize=address,undefined runs cases that
    touch every rule (conversions, free-slip and no-slip walls, surface
    tension with a volume pressure, tracked bubbles through a merge) without
    a sanitizer report."""
    exe = str(tmp_path / "orc_asan")
    flags = [f for f in GCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = ["gcc", *flags, "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", ORACLE_DIR, "-o", exe,
           os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ORACLE_DIR, "fslbm_oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    cases = [
        (I.rect_dam_break(nx=32, ny=20, nz=8, wx=10, hy=14, g=2e-4, nu=5e-3, collision=I.TRT, storage=I.F64,
                          variant=I.NBKC), 60),
        (I.rect_dam_break(nx=24, ny=16, nz=8, wx=8, hy=12, g=2e-4, nu=5e-3, q=27, collision=I.SRT,
                          storage=I.F64, variant=I.OM3,
                          boundary=(I.WALL_FREESLIP,) * 4 + (I.WALL_NOSLIP, I.WALL_FREESLIP)), 60),
        (I.sphere_drop_static(L=16, radius=4.0, q=19, sigma=1e-3, bubble=True), 20),
        (I.bubble_pair("merge"), 10),
    ]
    for n, (s, steps) in enumerate(cases):
        _write_case(tmp_path, "case%d.bin" % n, s, steps)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + [str(tmp_path / ("case%d.bin" % n)) for n in range(len(cases))],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("ok") == len(cases), r.stdout


# ----------------------------------------------------------------------------
# near-obstacle normal and smoothing (Sec. 2.2 cites the rule that keeps
# obstacle cells out of the fill-level gradient, and the K8 smoothing)
# ----------------------------------------------------------------------------

def _flat_layer_with_walls(q=19, sigma=0.0):
    """A flat interface layer (fill level 1/2) at y = 6 over liquid, no-slip
    walls on the x and z faces (so the layer meets walls along faces and
    edges) and a block of obstacle cells standing in the layer."""
    nx, ny, nz = 10, 12, 7
    W = I.WALL_NOSLIP
    p = I.Params(nx, ny, nz, q=q, collision=I.SRT, tau=0.8, boundary=(W, W, W, W, W, W), variant=I.NBRC,
                 sigma=sigma)
    i, j, k = _grid(p)
    t = np.where(j < 6, I.LIQUID, np.where(j == 6, I.INTERFACE, I.GAS)).astype(np.uint8)
    block = (i >= 4) & (i < 6) & (k >= 2) & (k < 4)
    t[block] = I.NOSLIP
    phi = np.where(t == I.LIQUID, 1.0, np.where(t == I.INTERFACE, 0.5, 0.0))
    return _setup(p, t, phi, np.ones(p.n), np.zeros((3, p.n)))


def test_normal_of_flat_interface_stays_along_walls():
    """Obstacle points of the 3x3x3 stencil take the cell's own fill level, so
    a flat surface meeting walls or obstacles keeps its normal exactly
    perpendicular to the surface (reading 0 or 1 there would tilt it)."""
    s = _flat_layer_with_walls()
    o = Oracle(s)
    i, j, k = _grid(s.params)
    for c in np.nonzero(s.type == I.INTERFACE)[0]:
        n = o.normal(int(i[c]), int(j[c]), int(k[c]))
        assert n[0] == 0.0 and n[2] == 0.0, (i[c], k[c], n)
        assert n[1] < 0.0  # towards the liquid below


def test_flat_interface_has_zero_curvature_next_to_walls():
    """The smoothing leaves obstacle cells out and renormalises its weights, so
    a flat surface stays flat after smoothing up to walls and obstacles: zero
    curvature in every interface cell (unrenormalised weights would bend it
    down next to every wall)."""
    s = _flat_layer_with_walls(sigma=1e-3)
    o = Oracle(s)
    i, j, k = _grid(s.params)
    for c in np.nonzero(s.type == I.INTERFACE)[0]:
        kap = o.curvature(int(i[c]), int(j[c]), int(k[c]))
        assert abs(kap) < 1e-14, (i[c], k[c], kap)
