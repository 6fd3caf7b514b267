"""ctypes binding of the FP64 CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fslbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fslbm.so")
GCC_FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall"]


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "fslbm_oracle.h"))):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("q", C.c_int32),
                ("collision", C.c_int32), ("boundary", C.c_int32 * 6), ("variant", C.c_int32),
                ("thurey_flux", C.c_int32), ("bubble_model", C.c_int32), ("tau", C.c_double),
                ("trt_lambda", C.c_double), ("gravity", C.c_double * 3), ("rho_gas", C.c_double),
                ("sigma", C.c_double), ("eps_phi", C.c_double), ("tie_delta", C.c_double),
                ("smagorinsky", C.c_double)]


class _Report(C.Structure):
    _fields_ = [("total_mass", C.c_double), ("liquid_mass", C.c_double),
                ("interface_mass", C.c_double), ("lost_mass", C.c_double),
                ("bubble_volume", C.c_double), ("p_volume", C.c_double),
                ("n_liquid", C.c_int64), ("n_interface", C.c_int64), ("n_gas", C.c_int64),
                ("step", C.c_int64)]


@dataclass
class OracleReport:
    total_mass: float
    liquid_mass: float
    interface_mass: float
    lost_mass: float
    bubble_volume: float
    p_volume: float
    n_liquid: int
    n_interface: int
    n_gas: int
    step: int


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = C.CDLL(build_oracle())
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        lib.orc_create.argtypes = [C.POINTER(_Params), u8, dp, dp, dp, dp, dp, C.POINTER(C.c_void_p)]
        lib.orc_create.restype = C.c_int
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_int64]
        lib.orc_step.restype = C.c_int
        lib.orc_set_variant.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_variant.restype = C.c_int
        lib.orc_fields.argtypes = [C.c_void_p, u8, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_post_collision.argtypes = [C.c_void_p, dp]
        lib.orc_mass.argtypes = [C.c_void_p, C.POINTER(_Report)]
        lib.orc_bubbles.argtypes = [C.c_void_p, C.POINTER(C.c_int64), dp, dp, C.c_int64]
        lib.orc_bubbles.restype = C.c_int64
        lib.orc_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        lib.orc_lattice.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), dp]
        lib.orc_opposite.argtypes = [C.c_int, C.c_int]
        lib.orc_opposite.restype = C.c_int
        lib.orc_collide_cell.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp,
                                         dp, dp, dp, dp]
        lib.orc_reconstruct_set.argtypes = [C.c_int, C.c_int, dp, C.c_uint32, C.c_double, u8]
        lib.orc_bc_value.argtypes = [C.c_int, C.c_int, C.c_double, dp, C.c_double]
        lib.orc_bc_value.restype = C.c_double
        lib.orc_normal.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp]
        lib.orc_curvature.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        lib.orc_curvature.restype = C.c_double
        lib.orc_thurey_class.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        lib.orc_thurey_class.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_threads.restype = C.c_int
        lib.orc_export_state.argtypes = [C.c_void_p, u8, dp, dp, dp, dp]
        lib.orc_import_state.argtypes = [C.c_void_p, u8, dp, dp, dp, dp, C.c_int64]
        lib.orc_import_state.restype = C.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def equilibrium(q, rho, u):
    out = np.zeros(q)
    _L().orc_equilibrium(q, rho, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(out))
    return out


def lattice(q):
    """(c, w): c is (q, 3) int, w is (q,) float, in the oracle's direction order."""
    c = np.zeros((q, 3), dtype=np.int64)
    w = np.zeros(q)
    cc = (C.c_int * 3)()
    ww = C.c_double()
    for i in range(q):
        _L().orc_lattice(q, i, cc, C.byref(ww))
        c[i] = list(cc)
        w[i] = ww.value
    return c, w


def opposite(q, i):
    return _L().orc_opposite(q, i)


def collide_cell(q, collision, tau, lam, g, f, cs=0.0, return_tau=False):
    fs = np.zeros(q)
    u = np.zeros(3)
    t = C.c_double()
    _L().orc_collide_cell(q, collision, tau, lam, cs, _dp(np.ascontiguousarray(g, dtype=np.float64)),
                          _dp(np.ascontiguousarray(f, dtype=np.float64)), _dp(fs), _dp(u),
                          C.cast(C.byref(t), C.POINTER(C.c_double)))
    if return_tau:
        return fs, u, t.value
    return fs, u


def reconstruct_set(q, variant, n, gas_mask, tie_delta=1e-9):
    R = np.zeros(q, dtype=np.uint8)
    _L().orc_reconstruct_set(q, variant, _dp(np.ascontiguousarray(n, dtype=np.float64)),
                             int(gas_mask), tie_delta, _u8(R))
    return R.astype(bool)


def bc_value(q, i, rho_g, u, fs_ibar):
    return _L().orc_bc_value(q, i, rho_g, _dp(np.ascontiguousarray(u, dtype=np.float64)), fs_ibar)


class Oracle:
    """One oracle simulation built from an inputs.Setup (or equivalent fields)."""

    def __init__(self, setup, variant=None):
        p = setup.params
        self.params = p
        self.q = p.q
        self.n = p.n
        cp = _Params()
        cp.nx, cp.ny, cp.nz, cp.q = p.nx, p.ny, p.nz, p.q
        cp.collision = p.collision
        for k in range(6):
            cp.boundary[k] = p.boundary[k]
        cp.variant = p.variant if variant is None else variant
        cp.thurey_flux = p.thurey_flux
        cp.bubble_model = p.bubble_model
        cp.tau, cp.trt_lambda = p.tau, p.trt_lambda
        for k in range(3):
            cp.gravity[k] = p.gravity[k]
        cp.rho_gas, cp.sigma, cp.eps_phi = p.rho_gas, p.sigma, p.eps_phi
        cp.tie_delta = p.tie_delta if p.tie_delta > 0 else 1e-9
        cp.smagorinsky = p.smagorinsky
        self._keep = [np.ascontiguousarray(a) for a in
                      (setup.type.astype(np.uint8), setup.phi, setup.rho, setup.ux, setup.uy, setup.uz)]
        t, phi, rho, ux, uy, uz = self._keep
        h = C.c_void_p()
        st = _L().orc_create(C.byref(cp), _u8(t), _dp(phi), _dp(rho), _dp(ux), _dp(uy), _dp(uz),
                             C.byref(h))
        if st != 0:
            raise ValueError("orc_create failed with status %d" % st)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def step(self, n=1):
        return _L().orc_step(self._h, int(n))

    def set_variant(self, v):
        return _L().orc_set_variant(self._h, int(v))

    def fields(self):
        n, q = self.n, self.q
        t = np.zeros(n, dtype=np.uint8)
        phi, rho, ux, uy, uz, m = (np.zeros(n) for _ in range(6))
        pdf = np.zeros(q * n)
        _L().orc_fields(self._h, _u8(t), _dp(phi), _dp(rho), _dp(ux), _dp(uy), _dp(uz), _dp(m),
                        _dp(pdf))
        return dict(type=t, phi=phi, rho=rho, ux=ux, uy=uy, uz=uz, mass=m, pdf=pdf.reshape(q, n))

    def set_threads(self, n):
        """OpenMP threads of the per-cell loops (results are bitwise the same
        for any count)."""
        if _L().orc_set_threads(self._h, int(n)) != 0:
            raise ValueError("threads must be >= 1")

    def export_state(self):
        """The state between steps, verbatim: types, pre-collision populations
        (q, N), raw mass array (interface m, 0 elsewhere), fill levels and the
        scalars (lost mass, p^V, p^V(0), V(0))."""
        n, q = self.n, self.q
        t = np.zeros(n, dtype=np.uint8)
        pdf, m, phi, sc = np.zeros(q * n), np.zeros(n), np.zeros(n), np.zeros(4)
        _L().orc_export_state(self._h, _u8(t), _dp(pdf), _dp(m), _dp(phi), _dp(sc))
        return dict(type=t, pdf=pdf.reshape(q, n), mass=m, phi=phi,
                    lost_mass=sc[0], p_volume=sc[1], p_volume0=sc[2], volume0=sc[3])

    def types(self):
        """Cell types of the current state (a copy, no arithmetic)."""
        t = np.zeros(self.n, dtype=np.uint8)
        _L().orc_export_state(self._h, _u8(t), None, None, None, None)
        return t

    def import_state(self, st, step=0):
        """Replaces the state verbatim by one exported from an oracle run of
        the same shape (see export_state)."""
        t = np.ascontiguousarray(st["type"], dtype=np.uint8)
        pdf = np.ascontiguousarray(st["pdf"], dtype=np.float64).reshape(-1)
        m = np.ascontiguousarray(st["mass"], dtype=np.float64)
        phi = np.ascontiguousarray(st["phi"], dtype=np.float64)
        sc = np.array([st["lost_mass"], st["p_volume"], st["p_volume0"], st["volume0"]], dtype=np.float64)
        if t.size != self.n or pdf.size != self.q * self.n or m.size != self.n or phi.size != self.n:
            raise ValueError("state of another shape")
        if _L().orc_import_state(self._h, _u8(t), _dp(pdf), _dp(m), _dp(phi), _dp(sc), int(step)) != 0:
            raise ValueError("orc_import_state failed")

    def post_collision(self):
        out = np.zeros(self.q * self.n)
        _L().orc_post_collision(self._h, _dp(out))
        return out.reshape(self.q, self.n)

    def mass(self) -> OracleReport:
        r = _Report()
        _L().orc_mass(self._h, C.byref(r))
        return OracleReport(**{k: getattr(r, k) for k, _ in _Report._fields_})

    def bubbles(self):
        """Tracked bubbles (bubble model 2): labels (smallest cell index),
        gas volumes and volume pressures, ascending by label."""
        cnt = _L().orc_bubbles(self._h, None, None, None, 0)
        lab = np.zeros(max(cnt, 1), dtype=np.int64)
        vol, pr = np.zeros(max(cnt, 1)), np.zeros(max(cnt, 1))
        _L().orc_bubbles(self._h, lab.ctypes.data_as(C.POINTER(C.c_int64)), _dp(vol), _dp(pr), cnt)
        return lab[:cnt], vol[:cnt], pr[:cnt]

    def normal(self, x, y, z):
        n = np.zeros(3)
        _L().orc_normal(self._h, x, y, z, _dp(n))
        return n

    def curvature(self, x, y, z):
        return _L().orc_curvature(self._h, x, y, z)

    def flux_class(self, x, y, z):
        return _L().orc_thurey_class(self._h, x, y, z)
