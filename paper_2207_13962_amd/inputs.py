"""Seeded, synthetic initial conditions for free-surface LBM runs.

This module builds the initial cell types, fill levels, densities and velocities
that both the GPU library and the CPU oracle consume. It holds geometry only
(fill levels of planes, cosines, boxes, cylinders, spheres and capsules, plus the
hydrostatic density profile) and none of the time step's arithmetic.

Setups follow the shapes of the paper's experiments (Sec. 4: standing gravity
wave, rectangular and cylindrical dam break, rising Taylor bubble, drop impact)
at the sizes and parameters of the workloads this library is measured on.
Cell (i, j, k) covers [i, i+1] x [j, j+1] x [k, k+1]; index = i + nx*(j + ny*k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

GAS, INTERFACE, LIQUID, NOSLIP, FREESLIP = 0, 1, 2, 3, 4
PERIODIC, WALL_NOSLIP, WALL_FREESLIP = 0, 1, 2
NBRC, NBKC, OM, OM3 = 1, 2, 3, 4
SRT, TRT = 0, 1
F64, F32, F16S = 0, 1, 2
# population layout: two grids, or one grid updated in place (AA pattern)
TWO_GRID, AA = 0, 1
VARIANT_NAMES = {NBRC: "NBRC", NBKC: "NBKC", OM: "OM", OM3: "OM3"}


def tau_from_nu(nu: float) -> float:
    """Relaxation time of a kinematic viscosity, nu = (tau - 1/2) / 3 (Sec. 2.1)."""
    return 3.0 * nu + 0.5


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    q: int = 19
    collision: int = SRT
    storage: int = F64
    boundary: tuple = (PERIODIC,) * 6
    variant: int = OM
    thurey_flux: int = 1
    bubble_model: int = 0
    tau: float = 0.55
    trt_lambda: float = 3.0 / 16.0
    gravity: tuple = (0.0, 0.0, 0.0)
    rho_gas: float = 1.0
    sigma: float = 0.0
    eps_phi: float = 1e-2
    tie_delta: float = 0.0
    smagorinsky: float = 0.0
    layout: int = TWO_GRID

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


@dataclass
class Setup:
    """Initial state of one run: parameters plus N-arrays (x fastest)."""

    params: Params
    type: np.ndarray
    phi: np.ndarray
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    name: str = ""
    steps: int = 0
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _grid(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def supersampled_fill(nx, ny, nz, inside, sub=8):
    """Fill level = fraction of sub^3 sample points of each cell for which
    inside(x, y, z) holds. Only cells whose corners disagree are sampled."""
    i, j, k = _grid(nx, ny, nz)
    corners = []
    for dx in (0.0, 1.0):
        for dy in (0.0, 1.0):
            for dz in (0.0, 1.0):
                corners.append(inside(i + dx, j + dy, k + dz))
    corners = np.stack(corners)
    allin = corners.all(axis=0)
    anyin = corners.any(axis=0)
    phi = np.where(allin, 1.0, 0.0)
    # cells whose corners disagree, plus a safety band (curved shapes can cut a
    # cell whose corners all lie outside); test the cell centre's neighbourhood
    centre_in = inside(i + 0.5, j + 0.5, k + 0.5)
    mixed = (anyin & ~allin) | (centre_in != allin)
    idx = np.nonzero(mixed | _near_boundary(nx, ny, nz, inside))[0]
    if idx.size:
        off = (np.arange(sub) + 0.5) / sub
        ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
        ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
        for start in range(0, idx.size, 4096):
            sl = idx[start:start + 4096]
            xs = i[sl][:, None] + ox[None, :]
            ys = j[sl][:, None] + oy[None, :]
            zs = k[sl][:, None] + oz[None, :]
            phi[sl] = inside(xs, ys, zs).mean(axis=1)
    return phi


def _near_boundary(nx, ny, nz, inside):
    """Cells whose centre lies within one cell of the shape's boundary: the
    centre test disagrees with the test at one of the 6 face centres."""
    i, j, k = _grid(nx, ny, nz)
    c = inside(i + 0.5, j + 0.5, k + 0.5)
    out = np.zeros_like(c)
    for d in ((0.5, 0, 0), (-0.5, 0, 0), (0, 0.5, 0), (0, -0.5, 0), (0, 0, 0.5), (0, 0, -0.5)):
        out |= inside(i + 0.5 + d[0], j + 0.5 + d[1], k + 0.5 + d[2]) != c
    return out


def cosine_column_fill(nx, ny, depth, amp, wavelength):
    """Exact fill levels of the cells below the surface y = depth + amp cos(2 pi x / wavelength):
    phi(i, j) = integral over x in [i, i+1] of clamp(eta(x) - j, 0, 1)."""
    k = 2.0 * math.pi / wavelength
    phi = np.zeros((ny, nx))

    def eta(x):
        return depth + amp * math.cos(k * x)

    def crossings(a, b, level):
        # x in (a, b) with eta(x) = level
        if amp == 0.0:
            return []
        v = (level - depth) / amp
        if v < -1.0 or v > 1.0:
            return []
        base = math.acos(v)
        out = []
        n0 = int(math.floor(k * a / (2 * math.pi))) - 1
        n1 = int(math.ceil(k * b / (2 * math.pi))) + 1
        for n in range(n0, n1 + 1):
            for th in (base + 2 * math.pi * n, -base + 2 * math.pi * n):
                x = th / k
                if a < x < b:
                    out.append(x)
        return out

    for j in range(ny):
        for i in range(nx):
            a, b = float(i), float(i + 1)
            pts = sorted(set([a, b] + crossings(a, b, j) + crossings(a, b, j + 1)))
            total = 0.0
            for x0, x1 in zip(pts[:-1], pts[1:]):
                e = eta(0.5 * (x0 + x1)) - j
                if e <= 0.0:
                    continue
                if e >= 1.0:
                    total += x1 - x0
                    continue
                # integral of (depth - j + amp cos(k x)) over [x0, x1]
                total += (depth - j) * (x1 - x0) + amp / k * (math.sin(k * x1) - math.sin(k * x0))
            phi[j, i] = min(max(total, 0.0), 1.0)
    return phi


def _neighbour_offsets(q):
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                n2 = dx * dx + dy * dy + dz * dz
                if n2 == 0 or (q == 19 and n2 == 3):
                    continue
                offs.append((dx, dy, dz))
    return offs


def types_from_fill(phi, params: Params, obstacle=None):
    """Cell types from fill levels: phi >= 1 liquid, phi <= 0 gas, interface
    otherwise; then every liquid cell with a gas cell in its velocity-set
    neighbourhood becomes interface with phi = 1, so that the interface layer
    is closed. Obstacle cells (boolean mask) keep their obstacle type."""
    nx, ny, nz, q = params.nx, params.ny, params.nz, params.q
    t = np.where(phi >= 1.0, LIQUID, np.where(phi <= 0.0, GAS, INTERFACE)).astype(np.uint8)
    phi = np.clip(phi, 0.0, 1.0).copy()
    if obstacle is not None:
        t[obstacle] = NOSLIP
        phi[obstacle] = 0.0
    t3 = t.reshape(nz, ny, nx)
    gas3 = t3 == GAS
    touch = np.zeros_like(gas3)
    b = params.boundary
    for dx, dy, dz in _neighbour_offsets(q):
        sh = gas3
        for axis, d, lo, hi in ((2, dx, b[0], b[1]), (1, dy, b[2], b[3]), (0, dz, b[4], b[5])):
            if d == 0:
                continue
            sh = np.roll(sh, -d, axis=axis)
            # a rolled-in slab across a wall face is not a neighbour
            face_periodic = (hi if d > 0 else lo) == PERIODIC
            if not face_periodic:
                idx = [slice(None)] * 3
                idx[axis] = slice(-1, None) if d > 0 else slice(0, 1)
                sh = sh.copy()
                sh[tuple(idx)] = False
        touch |= sh
    promote = (t3 == LIQUID) & touch
    t3[promote] = INTERFACE
    return t3.ravel().copy(), phi


def hydrostatic_rho(params: Params, h_ref: float, axis: int, g: float):
    """rho = 1 + 3 g (h_ref - y_c) along the gravity axis, y_c = cell centre;
    the lattice pressure p = rho/3 then equals p0 = 1/3 at height h_ref."""
    i, j, k = _grid(params.nx, params.ny, params.nz)
    yc = (i, j, k)[axis] + 0.5
    return 1.0 + 3.0 * g * (h_ref - yc)


def _finish(params, phi, rho, name, steps, obstacle=None, u=None, meta=None):
    t, phi = types_from_fill(phi, params, obstacle)
    n = params.n
    ux = np.zeros(n)
    uy = np.zeros(n)
    uz = np.zeros(n)
    if u is not None:
        ux, uy, uz = u
    fluid = (t == LIQUID) | (t == INTERFACE)
    rho = np.where(fluid, rho, 1.0)
    ux = np.where(fluid, ux, 0.0)
    uy = np.where(fluid, uy, 0.0)
    uz = np.where(fluid, uz, 0.0)
    phi = np.where(t == INTERFACE, phi, np.where(t == LIQUID, 1.0, 0.0))
    return Setup(params, t, phi.astype(np.float64), rho.astype(np.float64), ux.astype(np.float64),
                 uy.astype(np.float64), uz.astype(np.float64), name, steps, meta or {})


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def gravity_wave(nx=64, ny=64, nz=1, depth=32.0, amp=0.64, g=1e-5, tau=0.55, q=19,
                 collision=SRT, storage=F64, variant=OM, steps=1000, wavelength=None) -> Setup:
    """Standing gravity wave (Sec. 4.1 shape): periodic in x and z, no-slip
    walls below and above (y), surface depth + amp cos(2 pi x / nx), gravity -y."""
    b = (PERIODIC, PERIODIC, WALL_NOSLIP, WALL_NOSLIP, PERIODIC, PERIODIC)
    p = Params(nx, ny, nz, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=tau, gravity=(0.0, -g, 0.0))
    col = cosine_column_fill(nx, ny, depth, amp, wavelength or nx)  # (ny, nx)
    phi = np.broadcast_to(col[None, :, :], (nz, ny, nx)).ravel().copy()
    rho = hydrostatic_rho(p, depth, 1, g)
    return _finish(p, phi, rho, "gravity_wave", steps,
                   meta=dict(depth=depth, amp=amp, g=g, wavelength=wavelength or nx))


def gravity_wave_paper(L=200, variant=OM, storage=F64, steps=0) -> Setup:
    """The paper's gravity wave (Sec. 4.1): L x L x 1, liquid depth L/2,
    amplitude 0.01 L, one wavelength across x, D3Q19 SRT with relaxation rate
    1.8; Re = a0 omega0 L / nu = 10 fixes the wave's angular frequency
    omega0 = 1000 nu / L^2, and the dispersion relation omega0^2 =
    g k tanh(k d) with k = 2 pi / L fixes g."""
    tau = 1.0 / 1.8
    nu = (tau - 0.5) / 3.0
    k = 2.0 * math.pi / L
    d = 0.5 * L
    omega0 = 10.0 * nu / (0.01 * L * L)
    g = omega0 * omega0 / (k * math.tanh(k * d))
    s = gravity_wave(nx=L, ny=L, nz=1, depth=d, amp=0.01 * L, g=g, tau=tau, q=19, collision=SRT,
                     storage=storage, variant=variant, steps=steps, wavelength=L)
    s.meta.update(omega0=omega0, nu=nu, k=k)
    return s


def bubble_pair(kind="apart", q=19, storage=F64, variant=OM, periodic_x=False, g=0.0, steps=0) -> Setup:
    """Gas bubbles (5 x 4 x 4 gas cells, each inside a one-cell interface shell
    with phi = 0.5) in liquid at rest, 28 x 10 x 10 cells, no-slip walls (x
    periodic if periodic_x), tracked-bubble model. kind "apart": two bubbles,
    shells five liquid cells apart; "merge": one liquid cell between the
    shells, and the first bubble's shell face next to it holds phi = -0.05, so
    it empties in the first step and the film cell turns interface, joining
    the bubbles; "split": the shells five cells apart, joined by a one-cell
    line of interface cells with phi = 1.05, which fill in the first step and
    separate the bubbles; "straddle": one bubble across the x faces (two
    halves when x has walls)."""
    nx, ny, nz = 28, 10, 10
    wall = WALL_NOSLIP
    b = ((PERIODIC, PERIODIC) if periodic_x else (wall, wall)) + (wall, wall, wall, wall)
    p = Params(nx, ny, nz, q=q, collision=SRT, storage=storage, boundary=b, variant=variant, tau=0.6,
               bubble_model=2, gravity=(0.0, 0.0, -g))
    t = np.full((nz, ny, nx), LIQUID, dtype=np.uint8)
    phi = np.ones((nz, ny, nx))

    def bubble(xs):
        for x in xs:
            t[2:8, 2:8, x] = INTERFACE
            phi[2:8, 2:8, x] = 0.5
        for x in xs[1:-1]:
            t[3:7, 3:7, x] = GAS
            phi[3:7, 3:7, x] = 0.0

    if kind == "straddle":
        bubble([(nx - 3 + i) % nx for i in range(7)])
    else:
        bubble(list(range(2, 9)))
        x0 = 10 if kind == "merge" else 14
        bubble(list(range(x0, x0 + 7)))
    if kind == "merge":
        face = t[2:8, 2:8, 8] == INTERFACE
        phi[2:8, 2:8, 8] = np.where(face, -0.05, phi[2:8, 2:8, 8])
    elif kind == "split":
        t[5, 5, 9:14] = INTERFACE
        phi[5, 5, 9:14] = 1.05
    rho = np.ones(p.n)
    z = np.zeros(p.n)
    tt = t.ravel().copy()
    ph = np.where(tt == LIQUID, 1.0, np.where(tt == GAS, 0.0, phi.ravel()))
    return Setup(p, tt, ph, rho, z.copy(), z.copy(), z.copy(), "bubble_pair_" + kind, steps)


def bubbly_column(nx=48, ny=40, nz=56, n_bubbles=14, radius=(2.5, 6.0), fill=0.75, g=1e-4, seed=7, q=19,
                  storage=F64, variant=OM, bubble_model=2, steps=0, sub=4) -> Setup:
    """Closed box (no-slip walls) filled with liquid up to fill * nz, gas
    above, and n_bubbles spherical gas bubbles of random radius (seeded) in
    the liquid, some overlapping; gravity -z, D3Q19 SRT, tracked-bubble model
    (the gas above the surface is a bubble too: the box is closed)."""
    rng = np.random.default_rng(seed)
    b = (WALL_NOSLIP,) * 6
    p = Params(nx, ny, nz, q=q, collision=SRT, storage=storage, boundary=b, variant=variant, tau=0.6,
               bubble_model=bubble_model, gravity=(0.0, 0.0, -g))
    h = fill * nz
    centres = []
    for _ in range(n_bubbles):
        r = rng.uniform(*radius)
        c = (rng.uniform(r + 1, nx - r - 1), rng.uniform(r + 1, ny - r - 1), rng.uniform(r + 2, h - r - 2))
        centres.append((c, r))

    def inside(x, y, z):  # liquid
        liq = z < h
        for (cx, cy, cz), r in centres:
            liq &= (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 > r * r
        return liq

    phi = supersampled_fill(nx, ny, nz, inside, sub=sub)
    rho = hydrostatic_rho(p, h, 2, g)
    return _finish(p, phi, rho, "bubbly_column", steps, meta=dict(g=g, fill=fill, bubbles=centres))


def rect_dam_break(nx=256, ny=128, nz=64, wx=64, hy=96, g=2e-5, nu=1e-3, q=19, collision=TRT,
                   storage=F32, variant=OM, steps=5000, boundary=None) -> Setup:
    """Rectangular dam break (Sec. 4.2 shape): a liquid column wx x hy x nz in
    the left corner at rest, gravity -y, no-slip walls on every face."""
    b = boundary or (WALL_NOSLIP,) * 6
    p = Params(nx, ny, nz, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=tau_from_nu(nu), gravity=(0.0, -g, 0.0))
    i, j, k = _grid(nx, ny, nz)
    phi = ((i < wx) & (j < hy)).astype(np.float64)
    rho = hydrostatic_rho(p, float(hy), 1, g)
    return _finish(p, phi, rho, "rect_dam_break", steps, meta=dict(wx=wx, hy=hy, g=g))


def cyl_dam_break(nx=256, ny=256, nz=128, radius=32.0, height=96.0, g=2e-5, nu=5e-4, q=27,
                  collision=TRT, storage=F32, variant=OM, steps=4000) -> Setup:
    """Cylindrical dam break (Sec. 4.3 shape): a liquid cylinder on the floor
    (z = 0, no-slip), free-slip side walls and ceiling, gravity -z."""
    b = (WALL_FREESLIP, WALL_FREESLIP, WALL_FREESLIP, WALL_FREESLIP, WALL_NOSLIP, WALL_FREESLIP)
    p = Params(nx, ny, nz, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=tau_from_nu(nu), gravity=(0.0, 0.0, -g))
    cx, cy = nx / 2.0, ny / 2.0

    def inside(x, y, z):
        return ((x - cx) ** 2 + (y - cy) ** 2 < radius * radius) & (z < height)

    phi = supersampled_fill(nx, ny, nz, inside)
    rho = hydrostatic_rho(p, height, 2, g)
    return _finish(p, phi, rho, "cyl_dam_break", steps, meta=dict(radius=radius, height=height, g=g))


def taylor_bubble(nx=64, ny=64, nz=512, tube_radius=30.0, bubble_radius=24.0, z0=64.0,
                  length=96.0, g=1e-6, nu=1e-3, sigma=1e-4, q=27, collision=TRT, storage=F64,
                  variant=OM, steps=2000, cap=True, z_ref=None) -> Setup:
    """Rising Taylor bubble (Sec. 4.4 shape): a tube along z inside no-slip
    walls (cells whose centre lies farther than tube_radius from the axis are
    obstacles), a gas cylinder of bubble_radius from z0 to z0 + length, capped
    by a hemisphere when `cap`, liquid elsewhere, gravity -z, surface tension
    on, one enclosed bubble with volume pressure. Hydrostatic density is
    referenced to z_ref (default: the bubble's centre height)."""
    b = (WALL_NOSLIP,) * 6
    p = Params(nx, ny, nz, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=tau_from_nu(nu), gravity=(0.0, 0.0, -g), sigma=sigma, bubble_model=1)
    cx, cy = nx / 2.0, ny / 2.0
    ztop = z0 + length

    def in_bubble(x, y, z):
        r2 = (x - cx) ** 2 + (y - cy) ** 2
        cyl = (r2 < bubble_radius ** 2) & (z >= z0) & (z < ztop)
        if not cap:
            return cyl
        top = (r2 + (z - ztop) ** 2 < bubble_radius ** 2) & (z >= ztop)
        return cyl | top

    phi = 1.0 - supersampled_fill(nx, ny, nz, in_bubble)
    i, j, k = _grid(nx, ny, nz)
    obstacle = (i + 0.5 - cx) ** 2 + (j + 0.5 - cy) ** 2 > tube_radius ** 2
    zc = z_ref if z_ref is not None else z0 + 0.5 * (length + bubble_radius)
    rho = hydrostatic_rho(p, zc, 2, g)
    return _finish(p, phi, rho, "taylor_bubble", steps, obstacle=obstacle,
                   meta=dict(g=g, z0=z0, length=length, bubble_radius=bubble_radius))


def taylor_bubble_paper(D=32, variant=OM, storage=F64) -> Setup:
    """The paper's Taylor-bubble setup (Sec. 4.4): tube of diameter D in a
    D x D x 10D domain, no-slip walls, gas cylinder of diameter 0.75 D and
    length 3 D starting D above the bottom, hydrostatic pressure equal to the
    volume pressure at height 5 D; D3Q19 SRT with relaxation rate 1.8;
    Mo = g mu^4 / (rho sigma^3) = 0.015 and Bo = g D^2 / sigma = 100 (liquid
    density 1) fix g and sigma."""
    tau = 1.0 / 1.8
    nu = (tau - 0.5) / 3.0
    g = nu * nu * 1000.0 / (math.sqrt(0.015) * D ** 3)
    sigma = g * D * D / 100.0
    return taylor_bubble(nx=D, ny=D, nz=10 * D, tube_radius=D / 2.0, bubble_radius=0.375 * D, z0=float(D),
                         length=3.0 * D, g=g, nu=nu, sigma=sigma, q=19, collision=SRT, storage=storage,
                         variant=variant, cap=False, z_ref=5.0 * D)


def droplet_impact(L=48, diameter=None, pool=None, velocity=0.03, g=1e-5, tau=None, q=19,
                   collision=SRT, storage=F32, variant=OM, steps=2000) -> Setup:
    """Drop impact on a thin pool (Sec. 4.5 shape): cubic domain of edge L,
    periodic in x and y, no-slip floor and ceiling (z), pool depth L/20, a
    drop of diameter L/5 touching the pool and moving down at `velocity`."""
    d = diameter if diameter is not None else L / 5.0
    h = pool if pool is not None else L / 20.0
    tau = tau if tau is not None else 1.0 / 1.989
    b = (PERIODIC, PERIODIC, PERIODIC, PERIODIC, WALL_NOSLIP, WALL_NOSLIP)
    p = Params(L, L, L, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=tau, gravity=(0.0, 0.0, -g))
    c = (L / 2.0, L / 2.0, h + d / 2.0)

    def inside(x, y, z):
        return ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < (d / 2.0) ** 2) | (z < h)

    phi = supersampled_fill(L, L, L, inside)
    i, j, k = _grid(L, L, L)
    drop = (i + 0.5 - c[0]) ** 2 + (j + 0.5 - c[1]) ** 2 + (k + 0.5 - c[2]) ** 2 < (d / 2.0 + 1.0) ** 2
    drop &= (k + 0.5) > h
    uz = np.where(drop, -velocity, 0.0)
    rho = hydrostatic_rho(p, h, 2, g)
    n = p.n
    return _finish(p, phi, rho, "droplet_impact", steps, u=(np.zeros(n), np.zeros(n), uz),
                   meta=dict(diameter=d, pool=h, velocity=velocity))


def wave_slab(L=64, amp_frac=0.01, g=1e-5, tau=0.55, q=19, storage=F32, variant=OM,
              steps=2000) -> Setup:
    """3D standing-wave slab L x L/2 x L/4: depth L/4 (half the y extent),
    periodic x and z, no-slip y walls, amplitude amp_frac * L."""
    return gravity_wave(nx=L, ny=L // 2, nz=max(L // 4, 1), depth=L / 4.0, amp=amp_frac * L, g=g,
                        tau=tau, q=q, storage=storage, variant=variant, steps=steps)


def sphere_drop_static(L=32, radius=8.0, q=19, sigma=1e-3, bubble=False, storage=F64) -> Setup:
    """A resting drop (or bubble) of the given radius centred in a periodic box
    with no gravity: the Laplace-pressure pin."""
    b = (PERIODIC,) * 6
    p = Params(L, L, L, q=q, collision=SRT, storage=storage, boundary=b, variant=OM, tau=0.8,
               sigma=sigma)
    c = L / 2.0

    def inside(x, y, z):
        r2 = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
        return (r2 > radius * radius) if bubble else (r2 < radius * radius)

    phi = supersampled_fill(L, L, L, inside)
    rho = np.ones(p.n)
    return _finish(p, phi, rho, "static_bubble" if bubble else "static_drop", 0,
                   meta=dict(radius=radius))


def flat_interface_rest(nx=8, ny=12, nz=4, level=6, q=19, variant=OM, storage=F64,
                        collision=SRT) -> Setup:
    """Liquid below y = level, one flat interface layer (phi = 1/2) at
    y = level, gas above; rho = 1, u = 0, no gravity: a resting interface."""
    b = (PERIODIC, PERIODIC, WALL_NOSLIP, WALL_NOSLIP, PERIODIC, PERIODIC)
    p = Params(nx, ny, nz, q=q, collision=collision, storage=storage, boundary=b, variant=variant,
               tau=0.7)
    i, j, k = _grid(nx, ny, nz)
    phi = np.where(j < level, 1.0, np.where(j == level, 0.5, 0.0))
    return _finish(p, phi, np.ones(p.n), "flat_rest", 0)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def workload(name: str, smagorinsky: float = 0.0, **kw) -> Setup:
    """The measured workloads, by name (optionally with the Smagorinsky model)."""
    if name == "wave64":       # 64x64x1 D3Q19 SRT FP64 standing wave, OM, 1000 steps
        s = gravity_wave(**kw)
    elif name == "dam256":     # 256x128x64 D3Q19 TRT FP32 rectangular dam break, 5000 steps
        s = rect_dam_break(**kw)
    elif name == "cyl256":     # 256x256x128 D3Q27 TRT FP32 cylindrical dam break, 4000 steps
        s = cyl_dam_break(**kw)
    elif name == "taylor512":  # 64x64x512 D3Q27 TRT Taylor bubble with surface tension
        s = taylor_bubble(**kw)
    elif name == "dam512":     # the dam break scaled x2 per axis (HBM-resident working set)
        s = rect_dam_break(nx=512, ny=256, nz=128, wx=128, hy=192, **kw)
    else:
        raise KeyError(name)
    if smagorinsky:
        s.params = s.params.with_(smagorinsky=smagorinsky)
    return s


def serving_mix(n_requests=512, seed=1234, rate=None, l_min=48, l_max=192, steps_min=2000,
                steps_max=10000):
    """Request mix of the serving workload: half drop impacts (cubic edge L,
    lognormal around sqrt(l_min l_max) (96 for the default range), clipped to
    [l_min, l_max], drop L/5, pool L/20, impact
    speed 0.02-0.05), half standing-wave slabs L x L/2 x L/4 with amplitude
    0.005-0.02 L; variant uniform over the four; FP32 populations; 2000-10000
    steps; Poisson arrivals. Returns a list of dicts (kind, L, variant, steps,
    arrival, extra) - setups are built lazily by build_request()."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(n_requests):
        L = float(np.exp(rng.normal(0.5 * math.log(l_min * l_max), math.log(2.0) / 2.0)))
        L = int(min(max(round(L / 4) * 4, l_min), l_max))
        kind = "drop" if r % 2 == 0 else "wave"
        variant = int(rng.integers(1, 5))
        steps = int(rng.integers(steps_min, steps_max + 1))
        extra = float(rng.uniform(0.02, 0.05)) if kind == "drop" else float(rng.uniform(0.005, 0.02))
        if rate is not None:
            t += float(rng.exponential(1.0 / rate))
        reqs.append(dict(id=r, kind=kind, L=L, variant=variant, steps=steps, arrival=t, extra=extra))
    return reqs


# Relaxation time of the serving mix's drop impacts. The drop case's own
# relaxation rate (tau = 1/1.989) leaves a drop of only L/5 cells unresolved:
# 10 of the 24 drops of the small mix and 12 of 64 of a larger one (L 48-128,
# 1000-4000 steps) went unstable even with the Smagorinsky model, none at
# tau = 0.52.
SERVING_DROP_TAU = 0.52


def build_request(req: dict, storage=F32, drop_storage=F64) -> Setup:
    """Setup of one serving request: drops run TRT at SERVING_DROP_TAU, waves
    SRT. Drops keep FP64 populations by default: of the 48 fastest drops of
    the 512-request mix (L up to 192, up to 10000 steps), 16 went unstable
    with FP32 storage (all OM or OM3, late in the splash; still 2 at tau 0.55
    and 2 at 0.53 with the Smagorinsky model), none with FP64."""
    if req["kind"] == "drop":
        return droplet_impact(L=req["L"], velocity=req["extra"], variant=req["variant"],
                              storage=drop_storage, steps=req["steps"], collision=TRT,
                              tau=SERVING_DROP_TAU)
    return wave_slab(L=req["L"], amp_frac=req["extra"], variant=req["variant"], storage=storage,
                     steps=req["steps"])
