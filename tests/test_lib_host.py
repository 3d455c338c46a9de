"""Host-only checks of the C-ABI library: it loads, exports every function declared in
include/pflb.h, and validates parameters without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1812_00118_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf(?:lb|sur)_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return _lib.load_library()


def test_exports_every_declared_symbol(L):
    names = _declared("pflb.h")
    assert "pflb_step" in names and "pflb_create" in names
    for n in names:
        assert hasattr(L, n), n


def _params(**kw):
    p = _lib.Params()
    p.lattice, p.nx, p.ny, p.nz = 19, 8, 8, 8
    p.bc[0], p.bc[1], p.bc[2] = 0, 0, 1
    p.rho_L, p.rho_H, p.nu_L, p.nu_H = 1.0, 1000.0, 0.1, 0.01
    p.M, p.W, p.sigma, p.eps, p.hoc = 0.1, 4.0, 1e-3, 1e-10, 1
    p.storage = 0
    for k, v in kw.items():
        if k == "scale":
            p.scale_log2[0], p.scale_log2[1] = v
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [dict(lattice=7), dict(nu_H=0.0), dict(nu_L=-1.0),
                                 dict(M=0.0), dict(W=-1.0), dict(rho_L=0.0),
                                 dict(nx=0), dict(lattice=9), dict(sigma=float("nan")),
                                 dict(storage=3), dict(storage=1, scale=(30, 0)),
                                 dict(hoc=2), dict(eps=0.0)])
def test_create_rejects_bad_params(L, bad):
    """tau <= 1/2 (nu <= 0), M/W <= 0, non-finite values, bad enums and D2Q9 with nz != 1
    return PFLB_ERR_PARAM and leave *out NULL."""
    p = _params(**bad)
    ctx = ctypes.c_void_p(1)
    rc = L.pflb_create(ctypes.byref(p), ctypes.byref(ctx))
    assert rc == -1
    assert not ctx.value
    assert L.pflb_required_bytes(ctypes.byref(p), 0) == 0


def test_required_bytes_and_unbound_errors(L):
    p = _params()
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        N = 8 * 8 * 8
        # a state buffer holds both sets: 19 float pairs per site, or a float pair plus
        # 19 half pairs per site in FP16S storage
        assert L.pflb_required_bytes(ctypes.byref(p), 0) >= 19 * N * 8
        p16 = _params(storage=1, scale=(16, 8))
        assert L.pflb_required_bytes(ctypes.byref(p16), 1) >= N * 8 + 19 * N * 4
        assert L.pflb_required_bytes(ctypes.byref(p16), 1) < 19 * N * 8
        assert L.pflb_required_bytes(ctypes.byref(p), 2) > 0
        assert L.pflb_required_bytes(ctypes.byref(p), 9) == 0
        # every state call before pflb_bind reports PFLB_ERR_UNBOUND without GPU work
        assert L.pflb_step(ctx, 1, None) == -3
        assert L.pflb_set_state(ctx, None, None, None) == -3
        assert b"bound" in L.pflb_last_error(ctx)
        # misaligned pointers are refused
        arr = (ctypes.c_void_p * 3)(*[4096 + 16] * 3)
        assert L.pflb_bind(ctx, arr, 3) == -2
        assert L.pflb_bind(ctx, arr, 2) == -1
    finally:
        L.pflb_destroy(ctx)
