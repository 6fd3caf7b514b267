"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and validates parameters on the host (no GPU call is made)."""
import ctypes as C
import os
import re

import pytest

from paper_2207_13962_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fslbm.h")).read()
    return sorted(set(re.findall(r"\b(fslbm_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_2207_13962_amd import fslbm
    if not os.path.exists(fslbm.LIB_PATH):
        from paper_2207_13962_amd import build
        build.build()
    return fslbm


def test_exports_every_declared_symbol():
    fs = _lib()
    lib = C.CDLL(fs.LIB_PATH)
    names = _declared_symbols()
    assert "fslbm_create" in names and "fslbm_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(fs.EXPORTED) <= set(names)


def test_workspace_bytes_and_validation():
    fs = _lib()
    p = I.Params(256, 128, 64, q=19, storage=I.F32, collision=I.TRT, tau=0.503)
    n = fs.workspace_bytes(p)
    # two population grids of 19 x N floats dominate
    assert n > 2 * 19 * p.n * 4
    assert fs.workspace_bytes(p.with_(storage=I.F64)) > n
    assert fs.workspace_bytes(p.with_(storage=I.F16S)) < n
    # tracked bubbles: label, parent and target (int32), seven FP64 fields
    # and a flag byte per cell more (the gas-density field included)
    assert fs.workspace_bytes(p.with_(bubble_model=2)) - n >= 69 * p.n
    assert fs.workspace_bytes(p.with_(bubble_model=1)) == n
    bad = [p.with_(q=15), p.with_(tau=0.5), p.with_(variant=7), p.with_(nx=0),
           p.with_(storage=9), p.with_(boundary=(0, 1, 1, 1, 1, 1)), p.with_(bubble_model=3),
           p.with_(bubble_model=-1), p.with_(layout=2)]
    for b in bad:
        with pytest.raises(fs.FslbmError) as e:
            fs.workspace_bytes(b)
        assert e.value.status == fs.EINVAL


def test_inplace_layout_needs_one_grid_less():
    """The in-place layout drops the second population grid and adds two
    stash buffers of max(N/8, 2F, 1024) entries (F the largest face, at most
    N) of q populations and an int32 entry index per cell."""
    fs = _lib()
    for st, sb in ((I.F64, 8), (I.F32, 4), (I.F16S, 2)):
        for dims in ((256, 128, 64), (40, 40, 40), (48, 24, 12), (16, 16, 16)):
            p = I.Params(*dims, q=19, storage=st, collision=I.TRT, tau=0.503)
            two = fs.workspace_bytes(p)
            aa = fs.workspace_bytes(p.with_(layout=I.AA))
            n, q = p.n, p.q
            stride = (n + 255) // 256 * 256
            face = max(dims[0] * dims[1], dims[1] * dims[2], dims[0] * dims[2])
            cap = min(n, max(n // 8, 2 * face, 1024))
            # grids and stash are 256-byte-rounded; the staging buffer grows
            # to the slot bitmap (q * stride bits) on tiny domains
            diff = q * stride * sb - (2 * cap * q * sb + 255) // 256 * 256 - (4 * n + 255) // 256 * 256
            assert abs((two - aa) - diff) <= max(256, q * stride // 8), (st, dims, two - aa, diff)
    big = I.Params(256, 128, 64, q=19, storage=I.F32, collision=I.TRT, tau=0.503)
    assert fs.workspace_bytes(big.with_(layout=I.AA)) < 0.8 * fs.workspace_bytes(big)


def test_strerror_and_abi_version():
    fs = _lib()
    lib = fs.load_library()
    assert lib.fslbm_strerror(0) == b"ok"
    assert lib.fslbm_strerror(-4) == b"simulation unstable"
    cp = fs.make_params(I.Params(8, 8, 8))
    cp.abi_version = 99
    n = C.c_size_t()
    assert lib.fslbm_workspace_bytes(C.byref(cp), C.byref(n)) == fs.EINVAL
    assert b"abi" in lib.fslbm_last_error(None)


def test_create_rejects_bad_arguments_without_gpu():
    """fslbm_create validates on the host before touching the device."""
    fs = _lib()
    lib = fs.load_library()
    cp = fs.make_params(I.Params(8, 8, 8, tau=0.4))
    h = C.c_void_p()
    st = lib.fslbm_create(C.byref(cp), None, None, None, None, None, None, None, None, None, 0,
                          None, C.byref(h))
    assert st == fs.EINVAL and not h.value


def test_server_rejects_bad_arguments_without_gpu():
    """fslbm_server_create / _submit / _poll validate on the host first."""
    fs = _lib()
    lib = fs.load_library()
    h = C.c_void_p()
    assert lib.fslbm_server_create(0, 4, None, C.byref(h)) == fs.EINVAL and not h.value
    assert lib.fslbm_server_create(1 << 30, 0, None, C.byref(h)) == fs.EINVAL and not h.value
    assert lib.fslbm_server_create(1 << 30, 1 << 20, None, C.byref(h)) == fs.EINVAL
    rid = C.c_uint64()
    cp = fs.make_params(I.Params(8, 8, 8))
    assert lib.fslbm_server_submit(None, C.byref(cp), None, None, None, None, None, None, 10,
                                   C.byref(rid)) == fs.EINVAL
    n = C.c_int()
    assert lib.fslbm_server_poll(None, None, None, 0, C.byref(n)) == fs.EINVAL
    assert lib.fslbm_server_advance(None, 1) == fs.EINVAL
    lib.fslbm_server_destroy(None)
