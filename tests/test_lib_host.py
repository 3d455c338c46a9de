"""Host-only checks of the C-ABI library: it loads, exports every function declared in
include/pflb.h and include/pfsur.h, and validates parameters without touching a GPU."""
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


@pytest.mark.parametrize("header", ["pflb.h", "pfsur.h"])
def test_exports_every_declared_symbol(L, header):
    names = _declared(header)
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.exported_symbols(), n


def test_surrogate_parameter_count_matches_reference_network(L):
    from oracle import unet as U
    n = sum(co * 9 * ci + co for _, _, ci, co, _, _ in U.LAYERS) + U.OUT_CH * 32 + U.OUT_CH
    assert L.pfsur_num_params() == n


def _sur_cfg(**kw):
    c = _lib.SurCfg()
    c.H, c.W, c.max_batch = 256, 256, 4
    for k in range(4):
        c.in_scale[k] = 1.0
        c.out_scale[k] = 1.0
    c.lrr_scale = 1.0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_surrogate_workspace_planning(L):
    c = _sur_cfg()
    inf1 = L.pfsur_workspace_bytes(ctypes.byref(c), 1, 0)
    tr1 = L.pfsur_workspace_bytes(ctypes.byref(c), 1, 1)
    tr4 = L.pfsur_workspace_bytes(ctypes.byref(c), 4, 1)
    # inference holds at least the level-0 activations (32 + 64 + 32 + 32 BF16 channels)
    assert inf1 >= 256 * 256 * 160 * 2
    assert tr1 > 2 * inf1 and tr4 > 3.5 * tr1
    assert L.pfsur_workspace_bytes(ctypes.byref(c), 5, 1) == 0       # above max_batch
    assert L.pfsur_workspace_bytes(ctypes.byref(c), 0, 0) == 0
    for bad in (dict(H=20), dict(W=8), dict(max_batch=0), dict(max_batch=2000)):
        assert L.pfsur_workspace_bytes(ctypes.byref(_sur_cfg(**bad)), 1, 0) == 0, bad
    assert L.pfsur_guard_work_bytes(ctypes.byref(c), 1) > inf1
    assert L.pfsur_guard_work_bytes(ctypes.byref(c), 4) > 3 * L.pfsur_guard_work_bytes(ctypes.byref(c), 1)
    assert L.pfsur_guard_work_bytes(ctypes.byref(c), 5) == 0


def test_guard_accept_rule(L):
    """The fallback decision is a pure host function of two sums, the relative mass
    tolerance, the largest predicted speed and an optional phi error: forced from the
    host with synthetic values."""
    a = L.pfsur_guard_accept
    acc = lambda s_in, s_out, tol, chk, err, phi_tol, speed=0.02, u_max=0.1: a(
        s_in, s_out, tol, speed, u_max, chk, err, phi_tol)
    s = 4096.0
    assert acc(s, s * (1 + 0.9e-3), 1e-3, 0, 0.0, 0.0) == 1
    assert acc(s, s * (1 + 1e-2), 1e-3, 0, 0.0, 0.0) == 0           # injected +1e-2 sum(phi)
    assert acc(s, s * (1 - 1e-2), 1e-3, 0, 0.0, 0.0) == 0
    assert acc(s, float("nan"), 1e-3, 0, 0.0, 0.0) == 0
    assert acc(s, float("inf"), 1e-3, 0, 0.0, 0.0) == 0
    assert acc(s, s, 1e-3, 1, 0.02, 0.05) == 1
    assert acc(s, s, 1e-3, 1, 0.06, 0.05) == 0                      # checked window, phi off
    assert acc(s, s, 1e-3, 1, float("nan"), 0.05) == 0
    assert acc(s, s, 1e-3, 0, float("nan"), 0.05) == 1              # unchecked: error unused
    assert acc(s, s + 1e-9, 0.0, 0, 0.0, 0.0) == 0                  # zero tolerance
    assert acc(s, s, 1e-3, 0, 0.0, 0.0, speed=0.11) == 0            # unphysical speed
    assert acc(s, s, 1e-3, 0, 0.0, 0.0, speed=float("inf")) == 0
    assert acc(s, s, 1e-3, 0, 0.0, 0.0, speed=float("nan")) == 0
    assert acc(s, s, 1e-3, 0, 0.0, 0.0, speed=0.1) == 1             # at the bound


def test_conv_primitives_reject_bad_shapes(L):
    """Shape checks come before any device work: NULL pointers, channel counts that are
    not multiples of 8, odd sizes for the upsampling mode and unknown modes."""
    dummy = ctypes.c_void_p(4096)
    f = L.pfsur_conv_fwd
    assert f(None, 1, 16, 16, 8, 32, 0, dummy, None, 1, None, None, None) == -1
    assert f(dummy, 1, 16, 16, 12, 32, 0, dummy, None, 1, None, None, None) == -1
    assert f(dummy, 1, 15, 16, 8, 32, 1, dummy, None, 1, None, None, None) == -1
    assert f(dummy, 1, 16, 16, 8, 32, 3, dummy, None, 1, None, None, None) == -1
    assert f(dummy, 0, 16, 16, 8, 32, 0, dummy, None, 1, None, None, None) == -1
    assert f(ctypes.c_void_p(4098), 1, 16, 16, 8, 32, 0, dummy, None, 1, None, None, None) == -2
    g = L.pfsur_conv_wgrad
    assert g(dummy, dummy, 1, 16, 16, 8, 12, 0, dummy, None, dummy, None) == -1   # Cout % 8
    assert L.pfsur_conv_wgrad_work_bytes(1, 16, 16, 8, 32) >= 32 * 9 * 8 * 4


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
        elif k == "wall":                      # (face, component, velocity)
            p.wall_u[3 * v[0] + v[1]] = v[2]
        elif k == "wet":                       # (face, cos of the contact angle)
            p.wet_cos[v[0]] = v[1]
        elif k == "open":                      # (face, pressure) of an open face
            p.open[v[0]] = 1
            p.open_P[v[0]] = v[1]
        elif k == "open_flag":                 # (face, raw flag value)
            p.open[v[0]] = v[1]
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [dict(lattice=7), dict(nu_H=0.0), dict(nu_L=-1.0),
                                 dict(M=0.0), dict(W=-1.0), dict(rho_L=0.0),
                                 dict(nx=0), dict(lattice=9), dict(sigma=float("nan")),
                                 dict(storage=3), dict(storage=1, scale=(30, 0)),
                                 dict(hoc=2), dict(eps=0.0),
                                 dict(nx=4096, ny=4096, nz=256),
                                 dict(wall=(0, 1, 0.01)), dict(wall=(4, 2, 0.01)),
                                 dict(wall=(5, 0, float("nan"))),
                                 dict(lattice=9, nz=1, wall=(4, 0, 0.01)),
                                 dict(wet=(4, 1.5)), dict(wet=(5, float("nan"))),
                                 dict(wet=(0, 0.5)),
                                 dict(lattice=9, nz=1, bc=(1, 1, 0), wet=(4, 0.5)),
                                 # open faces: on a wall axis of at least 2 sites that
                                 # the lattice has, finite pressure, no contact angle on
                                 # the face, no moving wall anywhere, flag 0 or 1
                                 dict(open=(0, 0.0)),
                                 dict(bc=(0, 0, 0), open=(5, 0.0)),
                                 dict(open=(5, float("nan"))), dict(open=(4, float("inf"))),
                                 dict(open=(5, 0.0), wall=(4, 0, 0.01)),
                                 dict(open=(5, 0.0), wet=(5, 0.5)),
                                 dict(nz=1, open=(4, 0.0)),
                                 dict(open_flag=(5, 2)),
                                 dict(lattice=9, nz=1, bc=(1, 1, 0), open=(4, 0.0)),
                                 dict(lattice=9, nz=1, ny=1, bc=(1, 1, 0), open=(3, 0.0))])
def test_create_rejects_bad_params(L, bad):
    """tau <= 1/2 (nu <= 0), M/W <= 0, non-finite values, bad enums, D2Q9 with nz != 1,
    domains beyond 2^32 - 64 sites, wall velocities on periodic faces, normal to
    their face, non-finite or on faces D2Q9 does not have, and contact-angle cosines
    outside [-1, 1], non-finite, on periodic faces or on faces D2Q9 does not have return
    PFLB_ERR_PARAM and leave *out NULL."""
    p = _params(**bad)
    ctx = ctypes.c_void_p(1)
    rc = L.pflb_create(ctypes.byref(p), ctypes.byref(ctx))
    assert rc == -1
    assert not ctx.value
    assert L.pflb_required_bytes(ctypes.byref(p), 0) == 0


def test_create_accepts_tangential_wall_velocity(L):
    p = _params(wall=(5, 0, 0.01))            # z+ face moving along x
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    L.pflb_destroy(ctx)


@pytest.mark.parametrize("wet", [(4, 0.5), (5, -1.0), (5, 1.0)])
def test_create_accepts_contact_angles_on_wall_faces(L, wet):
    p = _params(wet=wet)                      # z faces are walls
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    L.pflb_destroy(ctx)


@pytest.mark.parametrize("kw", [dict(open=(5, 0.0)), dict(open=(4, -0.01), wet=(5, 0.3)),
                                dict(bc=(1, 0, 1), open=(0, 0.0)),
                                dict(bc=(1, 1, 1), nx=12, ny=5, nz=7, open=(3, 0.1)),
                                dict(lattice=9, nz=1, bc=(1, 1, 0), open=(3, 0.02)),
                                dict(lattice=9, nz=1, bc=(0, 1, 0), open=(2, 0.0)),
                                dict(lattice=9, nz=1, nx=20, ny=9, bc=(1, 0, 0), open=(1, 0.0))])
def test_create_accepts_open_faces(L, kw):
    """Open faces on wall axes; the state buffers grow by the boundary layers' pressures
    (one float per layer site, six layers of the largest face's size rounded up to 64
    sites)."""
    p = _params(**kw)
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    L.pflb_destroy(ctx)
    closed = _params(**{k: v for k, v in kw.items() if k != "open"})
    if p.lattice == 19:
        nx, ny, nz = p.nx, p.ny, p.nz
    else:
        nx, ny, nz = p.nx, 1, p.ny
    layer = max(ny * nz, nx * nz, nx * ny)
    side = 6 * 4 * ((layer + 63) // 64 * 64)
    base = L.pflb_required_bytes(ctypes.byref(closed), 0)
    assert L.pflb_required_bytes(ctypes.byref(p), 0) == (base + 255) // 256 * 256 + side
    assert L.pflb_required_bytes(ctypes.byref(p), 2) == L.pflb_required_bytes(ctypes.byref(closed), 2)


def test_inplace_storage_buffers(L):
    """In-place storage: one state buffer of the FP32 size, no second one (NULL binds),
    the phi field in the scratch buffer; open faces are refused."""
    p = _params(storage=2)
    fp32 = _params()
    N = 8 * 8 * 8
    assert L.pflb_required_bytes(ctypes.byref(p), 0) == L.pflb_required_bytes(ctypes.byref(fp32), 0)
    assert L.pflb_required_bytes(ctypes.byref(p), 1) == 0
    assert (L.pflb_required_bytes(ctypes.byref(p), 2) ==
            L.pflb_required_bytes(ctypes.byref(fp32), 2) + 4 * N)
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        arr = (ctypes.c_void_p * 3)(4096 * 256, None, 8192 * 256)
        assert L.pflb_bind(ctx, arr, 3) == 0
        arr = (ctypes.c_void_p * 3)(None, None, 8192 * 256)
        assert L.pflb_bind(ctx, arr, 3) == -1            # the state buffer is needed
    finally:
        L.pflb_destroy(ctx)
    for bad in (dict(storage=2, open=(5, 0.0)), dict(storage=3)):
        q = _params(**bad)
        c = ctypes.c_void_p(1)
        assert L.pflb_create(ctypes.byref(q), ctypes.byref(c)) == -1
        assert not c.value


def test_required_bytes_and_unbound_errors(L):
    p = _params()
    ctx = ctypes.c_void_p()
    assert L.pflb_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        N = 8 * 8 * 8
        # a state buffer holds both sets: 19 float pairs per site, or in FP16S storage a
        # float pair (the rest populations), a 16-byte moments word and 18 half pairs
        assert L.pflb_required_bytes(ctypes.byref(p), 0) >= 19 * N * 8
        p16 = _params(storage=1, scale=(16, 8))
        assert L.pflb_required_bytes(ctypes.byref(p16), 1) >= N * (8 + 16 + 18 * 4)
        assert L.pflb_required_bytes(ctypes.byref(p16), 1) < 19 * N * 8
        # a domain beyond 2^28 sites (64-bit slot addresses) is accepted
        big = _params(nx=2048, ny=1024, nz=256)
        assert L.pflb_required_bytes(ctypes.byref(big), 0) == 19 * 8 * 2048 * 1024 * 256
        assert L.pflb_required_bytes(ctypes.byref(p), 2) > 0
        assert L.pflb_required_bytes(ctypes.byref(p), 9) == 0
        # every state call before pflb_bind reports PFLB_ERR_UNBOUND without GPU work
        assert L.pflb_step(ctx, 1, None) == -3
        one = (ctypes.c_void_p * 1)(ctx.value)
        assert L.pflb_step_many(one, 1, 1, None) == -3
        assert L.pflb_step_many(one, 0, 1, None) == -1      # empty batch
        assert L.pflb_step_many(None, 1, 1, None) == -1
        assert L.pflb_set_state(ctx, None, None, None) == -3
        assert b"bound" in L.pflb_last_error(ctx)
        # misaligned pointers are refused
        arr = (ctypes.c_void_p * 3)(*[4096 + 16] * 3)
        assert L.pflb_bind(ctx, arr, 3) == -2
        assert L.pflb_bind(ctx, arr, 2) == -1
    finally:
        L.pflb_destroy(ctx)
