"""Python binding of libfslbm (argument marshalling only).

Every step of the method runs in the HIP kernels of libfslbm.so; this module
only converts arguments, owns a torch device tensor used as the library's
memory arena and passes torch's current HIP stream. It raises if the built
library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfslbm.so")

FSLBM_ABI_VERSION = 2
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE, EBUDGET = 0, -1, -2, -3, -4, -5, -6


class FslbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fslbm status %d: %s" % (status, msg))
        self.status = status


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("q", C.c_int32), ("collision", C.c_int32),
                ("storage", C.c_int32), ("boundary", C.c_int32 * 6), ("variant", C.c_int32),
                ("thurey_flux", C.c_int32), ("bubble_model", C.c_int32), ("tau", C.c_double),
                ("trt_lambda", C.c_double), ("gravity", C.c_double * 3), ("rho_gas", C.c_double),
                ("sigma", C.c_double), ("eps_phi", C.c_double), ("tie_delta", C.c_double),
                ("smagorinsky", C.c_double), ("layout", C.c_int32)]


class MassReport(C.Structure):
    _fields_ = [("total_mass", C.c_double), ("liquid_mass", C.c_double),
                ("interface_mass", C.c_double), ("lost_mass", C.c_double),
                ("bubble_volume", C.c_double), ("p_volume", C.c_double),
                ("n_liquid", C.c_int64), ("n_interface", C.c_int64), ("n_gas", C.c_int64),
                ("step", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

EXPORTED = ["fslbm_workspace_bytes", "fslbm_create", "fslbm_set_variant", "fslbm_step",
            "fslbm_mass", "fslbm_fields", "fslbm_interface_list", "fslbm_bubbles", "fslbm_set_timing",
            "fslbm_kernel_time", "fslbm_set_graphs", "fslbm_set_compaction_tile", "fslbm_destroy",
            "fslbm_strerror", "fslbm_last_error", "fslbm_server_create", "fslbm_server_submit",
            "fslbm_server_advance", "fslbm_server_poll", "fslbm_server_result",
            "fslbm_server_stats_get", "fslbm_server_destroy"]


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("resident", C.c_int64), ("completed", C.c_int64),
                ("ticks", C.c_int64), ("bytes_in_use", C.c_uint64),
                ("peak_bytes_in_use", C.c_uint64), ("budget_bytes", C.c_uint64)]


def load_library(path: str = LIB_PATH):
    """Load libfslbm.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libfslbm.so is not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    vp, dp, u8p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint8)
    lib.fslbm_workspace_bytes.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t)]
    lib.fslbm_workspace_bytes.restype = C.c_int
    lib.fslbm_create.argtypes = [C.POINTER(Params), u8p, dp, dp, dp, dp, dp, dp, dp, vp, C.c_size_t,
                                 vp, C.POINTER(vp)]
    lib.fslbm_create.restype = C.c_int
    lib.fslbm_set_variant.argtypes = [vp, C.c_int]
    lib.fslbm_set_variant.restype = C.c_int
    lib.fslbm_step.argtypes = [vp, C.c_int64]
    lib.fslbm_step.restype = C.c_int
    lib.fslbm_mass.argtypes = [vp, C.POINTER(MassReport)]
    lib.fslbm_mass.restype = C.c_int
    lib.fslbm_fields.argtypes = [vp, u8p, dp, dp, dp, dp, dp, dp, dp]
    lib.fslbm_fields.restype = C.c_int
    lib.fslbm_interface_list.argtypes = [vp, C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)]
    lib.fslbm_bubbles.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)]
    lib.fslbm_interface_list.restype = C.c_int
    lib.fslbm_set_timing.argtypes = [vp, C.c_int64]
    lib.fslbm_set_timing.restype = C.c_int
    lib.fslbm_kernel_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.fslbm_kernel_time.restype = C.c_int
    lib.fslbm_set_graphs.argtypes = [vp, C.c_int]
    lib.fslbm_set_graphs.restype = C.c_int
    lib.fslbm_set_compaction_tile.argtypes = [vp, C.c_int]
    lib.fslbm_set_compaction_tile.restype = C.c_int
    lib.fslbm_mass_noalloc.argtypes = [vp, dp]
    lib.fslbm_mass_noalloc.restype = C.c_int
    lib.fslbm_get_scalars.argtypes = [vp, dp]
    lib.fslbm_get_scalars.restype = C.c_int
    lib.fslbm_set_scalars.argtypes = [vp, dp]
    lib.fslbm_set_scalars.restype = C.c_int
    lib.fslbm_destroy.argtypes = [vp]
    lib.fslbm_destroy.restype = None
    lib.fslbm_strerror.argtypes = [C.c_int]
    lib.fslbm_strerror.restype = C.c_char_p
    lib.fslbm_last_error.argtypes = [vp]
    lib.fslbm_last_error.restype = C.c_char_p
    lib.fslbm_server_create.argtypes = [C.c_size_t, C.c_int, vp, C.POINTER(vp)]
    lib.fslbm_server_create.restype = C.c_int
    lib.fslbm_server_submit.argtypes = [vp, C.POINTER(Params), u8p, dp, dp, dp, dp, dp, C.c_int64,
                                        C.POINTER(C.c_uint64)]
    lib.fslbm_server_submit.restype = C.c_int
    lib.fslbm_server_advance.argtypes = [vp, C.c_int64]
    lib.fslbm_server_advance.restype = C.c_int
    lib.fslbm_server_poll.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_int), C.c_int,
                                      C.POINTER(C.c_int)]
    lib.fslbm_server_poll.restype = C.c_int
    lib.fslbm_server_result.argtypes = [vp, C.c_uint64, C.POINTER(MassReport), dp]
    lib.fslbm_server_result.restype = C.c_int
    lib.fslbm_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    lib.fslbm_server_stats_get.restype = C.c_int
    lib.fslbm_server_destroy.argtypes = [vp]
    lib.fslbm_server_destroy.restype = None
    _lib = lib
    return lib


def make_params(p) -> Params:
    """C parameter struct from an inputs.Params."""
    cp = Params()
    cp.abi_version = FSLBM_ABI_VERSION
    cp.nx, cp.ny, cp.nz, cp.q = p.nx, p.ny, p.nz, p.q
    cp.collision, cp.storage = p.collision, p.storage
    for k in range(6):
        cp.boundary[k] = p.boundary[k]
    cp.variant, cp.thurey_flux, cp.bubble_model = p.variant, p.thurey_flux, p.bubble_model
    cp.tau, cp.trt_lambda = p.tau, p.trt_lambda
    for k in range(3):
        cp.gravity[k] = p.gravity[k]
    cp.rho_gas, cp.sigma, cp.eps_phi, cp.tie_delta = p.rho_gas, p.sigma, p.eps_phi, p.tie_delta
    cp.smagorinsky = p.smagorinsky
    cp.layout = p.layout
    return cp


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint8))


def workspace_bytes(p) -> int:
    lib = load_library()
    n = C.c_size_t()
    st = lib.fslbm_workspace_bytes(C.byref(make_params(p)), C.byref(n))
    if st != OK:
        raise FslbmError(st, lib.fslbm_last_error(None).decode())
    return n.value


class Simulation:
    """One free-surface LBM run on the GPU.

    setup: an inputs.Setup (params + initial fields). The device memory arena is
    a torch uint8 tensor; all work goes to torch's current stream of `device`.
    """

    def __init__(self, setup, variant=None, device="cuda:0", pdf=None, mass=None, stream=None):
        import torch

        lib = load_library()
        p = setup.params
        if variant is not None:
            p = p.with_(variant=variant)
        self.params = p
        self.q, self.n = p.q, p.n
        self.device = torch.device(device)
        cp = make_params(p)
        nbytes = workspace_bytes(p)
        with torch.cuda.device(self.device):
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arrays = [np.ascontiguousarray(setup.type, dtype=np.uint8)]
        arrays += [np.ascontiguousarray(a, dtype=np.float64) for a in
                   (setup.phi, setup.rho, setup.ux, setup.uy, setup.uz)]
        pdf = None if pdf is None else np.ascontiguousarray(pdf, dtype=np.float64).reshape(-1)
        mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        h = C.c_void_p()
        st = lib.fslbm_create(C.byref(cp), _u8(arrays[0]), *[_dp(a) for a in arrays[1:]], _dp(pdf),
                              _dp(mass), C.c_void_p(self._arena.data_ptr()), nbytes,
                              C.c_void_p(self._stream.cuda_stream), C.byref(h))
        if st != OK:
            raise FslbmError(st, lib.fslbm_last_error(None).decode())
        self._h = h
        self._lib = lib

    def _check(self, st):
        if st not in (OK,):
            raise FslbmError(st, self._lib.fslbm_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._lib.fslbm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_variant(self, v):
        self._check(self._lib.fslbm_set_variant(self._h, int(v)))

    def step(self, n=1):
        """Enqueue n steps (asynchronous)."""
        self._check(self._lib.fslbm_step(self._h, int(n)))

    def mass(self, check=True):
        r = MassReport()
        st = self._lib.fslbm_mass(self._h, C.byref(r))
        if check:
            self._check(st)
        d = r.as_dict()
        d["status"] = st
        return d

    def mass_noalloc(self, out):
        """Enqueue the mass reduction into `out`, a torch float64 device tensor
        of 8 elements (total, liquid, interface, lost mass, bubble volume,
        n_liquid, n_interface, n_gas); no allocation, no wait."""
        if out.dtype != __import__("torch").float64 or out.numel() < 8 or not out.is_cuda:
            raise ValueError("out must be a float64 device tensor of 8 elements")
        self._check(self._lib.fslbm_mass_noalloc(self._h, C.cast(C.c_void_p(out.data_ptr()),
                                                                 C.POINTER(C.c_double))))

    def fields(self, pdf=True, check=True):
        n, q = self.n, self.q
        t = np.zeros(n, dtype=np.uint8)
        phi, rho, ux, uy, uz, m = (np.zeros(n) for _ in range(6))
        f = np.zeros(q * n) if pdf else None
        st = self._lib.fslbm_fields(self._h, _u8(t), _dp(phi), _dp(rho), _dp(ux), _dp(uy), _dp(uz),
                                    _dp(m), _dp(f))
        if check:
            self._check(st)
        out = dict(type=t, phi=phi, rho=rho, ux=ux, uy=uy, uz=uz, mass=m, status=st)
        if pdf:
            out["pdf"] = f.reshape(q, n)
        return out

    def types(self, check=True):
        """Cell types only (one copy of the flag bytes; waits for the stream)."""
        t = np.zeros(self.n, dtype=np.uint8)
        st = self._lib.fslbm_fields(self._h, _u8(t), None, None, None, None, None, None, None)
        if check:
            self._check(st)
        return t

    def interface_list(self):
        cnt = C.c_int64()
        self._check(self._lib.fslbm_interface_list(self._h, None, 0, C.byref(cnt)))
        out = np.zeros(max(cnt.value, 1), dtype=np.int32)
        self._check(self._lib.fslbm_interface_list(
            self._h, out.ctypes.data_as(C.POINTER(C.c_int32)), cnt.value, C.byref(cnt)))
        return out[:cnt.value]

    def bubbles(self, check=True):
        """Tracked bubbles (bubble model 2): labels (smallest cell index), gas
        volumes and volume pressures, ascending by label."""
        cnt = C.c_int64()
        st = self._lib.fslbm_bubbles(self._h, None, None, None, 0, C.byref(cnt))
        if check:
            self._check(st)
        k = max(cnt.value, 1)
        lab = np.zeros(k, dtype=np.int64)
        vol, pr = np.zeros(k), np.zeros(k)
        st = self._lib.fslbm_bubbles(self._h, lab.ctypes.data_as(C.POINTER(C.c_int64)), _dp(vol), _dp(pr),
                                     cnt.value, C.byref(cnt))
        if check:
            self._check(st)
        return lab[:cnt.value], vol[:cnt.value], pr[:cnt.value]

    def scalars(self):
        """(lost mass, p^V, p^V(0), V(0)) of the current state."""
        out = np.zeros(4)
        self._check(self._lib.fslbm_get_scalars(self._h, _dp(out)))
        return tuple(float(x) for x in out)

    def set_scalars(self, lost_mass, p_volume, p_volume0, volume0):
        """Restore the scalars of a saved state (after a resume from pdf and mass)."""
        v = np.array([lost_mass, p_volume, p_volume0, volume0], dtype=np.float64)
        self._check(self._lib.fslbm_set_scalars(self._h, _dp(v)))

    def set_graphs(self, enable):
        """Replay captured step graphs (default) or launch kernel by kernel."""
        self._check(self._lib.fslbm_set_graphs(self._h, int(bool(enable))))

    def set_compaction_tile(self, cells_per_thread):
        """Cells scanned per thread of a compaction tile (16 times a power of
        two, at least the library's choice); results are identical."""
        self._check(self._lib.fslbm_set_compaction_tile(self._h, int(cells_per_thread)))

    def set_timing(self, capacity):
        """Bracket the next `capacity` streaming-kernel launches (one per step) with HIP events."""
        self._check(self._lib.fslbm_set_timing(self._h, int(capacity)))

    def kernel_time(self):
        """(timed launches, summed duration in ms) of the streaming kernel."""
        n, ms = C.c_int64(), C.c_double()
        self._check(self._lib.fslbm_kernel_time(self._h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def synchronize(self):
        self._stream.synchronize()


class Server:
    """Batched serving of many independent runs on one GPU (fslbm_server_*).

    budget_bytes: device pool for the resident runs; max_slots: resident runs
    at most. All work goes to torch's current stream of `device` (or `stream`).
    """

    def __init__(self, budget_bytes, max_slots=64, device="cuda:0", stream=None):
        import torch

        self._lib = load_library()
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self._lib.fslbm_server_create(int(budget_bytes), int(max_slots),
                                           C.c_void_p(self._stream.cuda_stream), C.byref(h))
        if st != OK:
            raise FslbmError(st, "fslbm_server_create failed")
        self._h = h
        self._n = {}

    def submit(self, setup, nsteps):
        """Queue one run; returns its id."""
        p = setup.params
        arrays = [np.ascontiguousarray(setup.type, dtype=np.uint8)]
        arrays += [np.ascontiguousarray(a, dtype=np.float64) for a in
                   (setup.phi, setup.rho, setup.ux, setup.uy, setup.uz)]
        rid = C.c_uint64()
        st = self._lib.fslbm_server_submit(self._h, C.byref(make_params(p)), _u8(arrays[0]),
                                           *[_dp(a) for a in arrays[1:]], int(nsteps), C.byref(rid))
        if st != OK:
            raise FslbmError(st, "fslbm_server_submit rejected the run")
        self._n[rid.value] = p.n
        return rid.value

    def advance(self, ticks):
        """Run up to `ticks` batched steps (admitting and retiring runs)."""
        st = self._lib.fslbm_server_advance(self._h, int(ticks))
        if st != OK:
            raise FslbmError(st, "fslbm_server_advance failed")

    def poll(self, max_n=4096):
        """[(id, status)] of runs finished since the last poll."""
        ids = (C.c_uint64 * max_n)()
        sts = (C.c_int * max_n)()
        n = C.c_int()
        st = self._lib.fslbm_server_poll(self._h, ids, sts, max_n, C.byref(n))
        if st != OK:
            raise FslbmError(st, "fslbm_server_poll failed")
        return [(ids[i], sts[i]) for i in range(n.value)]

    def result(self, rid, phi=True):
        """(mass report dict, fill levels or None) of a finished run; frees it."""
        r = MassReport()
        out = np.zeros(self._n[rid]) if phi else None
        st = self._lib.fslbm_server_result(self._h, int(rid), C.byref(r), _dp(out))
        if st != OK:
            raise FslbmError(st, "no finished run %d" % rid)
        del self._n[rid]
        return r.as_dict(), out

    def stats(self):
        s = ServerStats()
        self._lib.fslbm_server_stats_get(self._h, C.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._lib.fslbm_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
