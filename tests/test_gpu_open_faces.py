"""Open (pressure) faces on the GPU against the FP64 oracle, through the C ABI.

The pressure condition of Section 4.4's dam-break top, in the reading both sides take:
the ghost layer beyond an open face copies the boundary layer (zero normal gradient of
phi and u) with the pressure taken linearly to the face's P_f, so a population entering
through the face is the one its boundary-layer source sent, plus 2 w_i (P_f - P)/T for
the hydrodynamic set.  Open faces are those of the z axis (D2Q9: the user's y axis).

Bars: one step as the other one-step cases (FP32: |d| <= 2e-6 max|ref| + 2e-5 |ref|;
FP16S: 2e-3 of max|ref|); runs: FP32 max|d phi| <= 1e-5 and relative momentum error
<= 1e-4; FP16S max|d phi| <= 5e-4 and relative momentum error <= 1e-3.
"""
import numpy as np
import pytest
import torch

import pfinputs
from oracle import pflbm as O

pytestmark = pytest.mark.gpu

W_, P_ = "wall", "periodic"
NAN = float("nan")
FACES = ("xm", "xp", "ym", "yp", "zm", "zp")


def _open(**faces):
    P = [NAN] * 6
    for k, v in faces.items():
        P[FACES.index(k)] = v
    return P


def _sim(cfg, storage="fp32"):
    from paper_1812_00118_amd import Sim
    return Sim(cfg, storage=storage)


def _cfg(q, shape, bc, **kw):
    d = dict(lattice=q, shape=shape, bc=bc, rho_L=1.0, rho_H=1000.0, nu_L=0.05, nu_H=0.01,
             M=0.1, W=4.0, sigma=1e-3, g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1, dtheta_C=0.0)
    d.update(kw)
    return d


def _prm(cfg):
    return O.Params.from_dict(pfinputs.model_params(cfg))


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _close(got, ref, rel_max=2e-6, rel=2e-5):
    tol = rel_max * np.abs(ref).max() + rel * np.abs(ref)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (np.abs(got - ref).max(), np.abs(ref).max(), int(bad.sum()))


def _jerr(Jg, Jr, rho_H):
    N = Jr[0].size
    return np.linalg.norm(Jg - Jr) / max(np.linalg.norm(Jr), rho_H * 1e-6 * np.sqrt(N))


# open z faces with closed x walls (sources crossing both bounce back) and periodic y
# (sources wrap), an open top over a closed box, the thinnest axis (2 planes, both faces
# open, every site on a face), a single column (only the straight population enters),
# and the D2Q9 mapping of the user's y faces
OPEN_CASES = [
    ("d3q19-open-z", 19, (17, 11, 6), (W_, P_, W_), _open(zm=0.02, zp=-0.01)),
    ("d3q19-open-top-box", 19, (13, 9, 7), (W_, W_, W_), _open(zp=0.0)),
    ("d3q19-open-thin", 19, (5, 4, 2), (P_, P_, W_), _open(zm=0.01, zp=-0.02)),
    ("d3q19-open-column", 19, (1, 1, 3), (W_, W_, W_), _open(zp=0.005)),
    ("d2q9-open-y", 9, (40, 21, 1), (W_, W_, P_), _open(ym=0.01, yp=-0.01)),
    ("d2q9-open-top-periodic-x", 9, (33, 5, 1), (P_, W_, P_), _open(yp=0.0)),
    # x and y faces; edges and corners where open faces meet each other and closed ones
    # (a population crossing several open faces takes the mean of their pressures)
    ("d3q19-open-x", 19, (9, 7, 6), (W_, P_, P_), _open(xm=0.02, xp=-0.01)),
    ("d3q19-open-edges", 19, (8, 7, 6), (W_, W_, W_), _open(xp=0.01, yp=-0.02, zp=0.0)),
    ("d3q19-open-all", 19, (5, 4, 3), (W_, W_, W_),
     _open(xm=0.01, xp=-0.01, ym=0.02, yp=0.0, zm=-0.01, zp=0.005)),
    ("d2q9-open-x", 9, (20, 9, 1), (W_, P_, P_), _open(xm=0.01, xp=-0.01)),
    ("d2q9-open-corner", 9, (12, 10, 1), (W_, W_, P_), _open(xp=0.01, yp=0.0)),
]


def _open_slots(q, shape, bc, op):
    """Number of (site, direction) pairs that enter through an open face."""
    from oracle.lattice import D2Q9, D3Q19
    lat = D3Q19 if q == 19 else D2Q9
    nx, ny, nz = shape
    count = 0
    for f, P in enumerate(op):
        if np.isnan(P):
            continue
        axis, side = f // 2, (-1 if f % 2 == 0 else 1)
        for c in lat.c:
            if c[axis] == -side:     # enters through face f
                count += (nx * ny * nz) // shape[axis]
    return count


@pytest.mark.parametrize("name,q,shape,bc,op", OPEN_CASES, ids=[c[0] for c in OPEN_CASES])
@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_one_step_open_faces(name, q, shape, bc, op, storage):
    """Every population after one step from a seeded random state, and sum(phi) after
    it (open faces let it change)."""
    cfg = _cfg(q, shape, bc, open_P=op,
               g=(2e-5, -1e-5, 3e-5) if q == 19 else (2e-5, -1e-5, 0))
    h0, g0 = pfinputs.random_state(q, shape, seed=sum(name.encode()) + 7)
    sim = _sim(cfg, storage=storage)
    sim.set_state(h0, g0)
    h0d, g0d = (_np(t) for t in sim.get_state())      # the encoded start (exact in FP32)
    m0, _ = sim.mass()
    sim.step(1)
    h1, g1 = (_np(t) for t in sim.get_state())
    m1, bad = sim.mass()
    prm = _prm(cfg)
    assert prm.open_faces
    hr, gr = O.step(prm, h0d, g0d)
    assert not bad
    # the same step with the faces closed
    hn, gn = O.step(_prm(dict(cfg, open_P=None)), h0d, g0d)
    dm_ref = O.mass(hr) - O.mass(h0d)
    if storage == "fp32":
        _close(h1, hr)
        _close(g1, gr)
        assert np.abs(gn - gr).max() > 100 * np.abs(g1 - gr).max()
        assert np.abs(hn - hr).max() > 100 * np.abs(h1 - hr).max()
        assert abs((m1 - m0) - dm_ref) <= 1e-6 * abs(m0)
    else:
        assert np.abs(h1 - hr).max() <= 2e-3 * np.abs(hr).max()
        assert np.abs(g1 - gr).max() <= 2e-3 * np.abs(gr).max()
        # each entering value is re-encoded once: its fp16 rounding, summed over them
        K = _open_slots(q, shape, bc, op)
        assert abs((m1 - m0) - dm_ref) <= 2e-3 * np.abs(hr).max() * K


def _channel(q, along="z"):
    """Water between no-slip walls, open faces at +-dP/2 along z (D2Q9: y) with the walls
    across x, or along x with the walls across z (D2Q9: y)."""
    dP = 0.6
    if along == "z":
        if q == 19:
            shape, bc, op = (9, 2, 16), (W_, P_, W_), _open(zm=dP / 2, zp=-dP / 2)
        else:
            shape, bc, op = (9, 16, 1), (W_, W_, P_), _open(ym=dP / 2, yp=-dP / 2)
    else:
        if q == 19:
            shape, bc, op = (16, 2, 9), (W_, P_, W_), _open(xm=dP / 2, xp=-dP / 2)
        else:
            shape, bc, op = (16, 9, 1), (W_, W_, P_), _open(xm=dP / 2, xp=-dP / 2)
    cfg = _cfg(q, shape, bc, open_P=op, nu_L=0.1, nu_H=0.1, g=(0.0, 0.0, 0.0))
    cfg["name"] = "channel"
    return cfg, dP


def _channel_fields(cfg):
    nx, ny, nz = cfg["shape"]
    phi = np.ones((nz, ny, nx), np.float32)
    return phi, np.zeros((3,) + phi.shape, np.float32), np.zeros_like(phi)


@pytest.mark.parametrize("q,along", [(9, "z"), (19, "z"), (9, "x"), (19, "x")])
def test_pressure_driven_channel_vs_oracle(q, along):
    """300 steps of the pressure-driven channel against the oracle's: the momentum at
    the FP32 bar.  phi leaves 1 only by ~1e-5 (what the zero-gradient ghost lets through
    the faces), where the interface normal grad(phi)/|grad(phi)| of Eq. 4's sharpening
    term is set by rounding: there phi is compared against the oracle's own divergence
    from a start perturbed by float32 half-ulp noise (4 times that floor, at least the
    plain 1e-5; the floor is the larger of the divergences a half-ulp start and a
    float32-rounded state give the oracle)."""
    cfg, _ = _channel(q, along)
    phi, u, P = _channel_fields(cfg)
    sim = _sim(cfg)
    sim.init_fields(phi, u, P)
    m0, _ = sim.mass()
    sim.step(300)
    r = {k: _np(v) for k, v in sim.read().items()}
    m1, bad = sim.mass()
    prm = _prm(cfg)
    h0, g0 = O.init(prm, phi.astype(np.float64), u.astype(np.float64), P.astype(np.float64))
    h, g = O.run(prm, h0, g0, 300)
    ro = O.read(prm, h, g)
    dm_ref = O.mass(h) - O.mass(h0)
    # the oracle's own divergence from two float32-sized disturbances: a start moved by
    # half-ulp noise, and its populations rounded to float32 after every step (what a
    # float32 state does to an otherwise exact step)
    rng = np.random.default_rng(99)
    hs = h0 * (1.0 + 2.0 ** -24 * rng.standard_normal(h0.shape))
    hp, gp = O.run(prm, hs, g0, 300)
    hf, gf = (a.astype(np.float32).astype(np.float64) for a in (h0, g0))
    for _ in range(300):
        hf, gf = O.step(prm, hf, gf)
        hf, gf = (a.astype(np.float32).astype(np.float64) for a in (hf, gf))
    floor = max(np.abs(O.read(prm, hp, gp)["phi"] - ro["phi"]).max(),
                np.abs(O.read(prm, hf, gf)["phi"] - ro["phi"]).max())
    dm_floor = max(abs((O.mass(hp) - O.mass(hs)) - dm_ref),
                   abs((O.mass(hf) - O.mass(h0)) - dm_ref))
    D = 3 if q == 19 else 2
    dphi = np.abs(r["phi"] - ro["phi"]).max()
    eJ = _jerr(r["J"], ro["J"][:D], cfg["rho_H"])
    print(f"\nchannel D{D} along {along}: max|dphi| {dphi:.2e} (oracle floor {floor:.2e}, max|phi - 1| "
          f"{np.abs(ro['phi'] - 1).max():.2e}), rel J err {eJ:.2e}, |J| "
          f"{np.abs(ro['J']).max():.3e}")
    assert not bad
    assert np.abs(ro["J"]).max() > 1.0         # the flow is under way
    assert dphi <= max(1e-5, 4.0 * floor)
    assert eJ <= 1e-4
    # the flux of phi through the faces carries the same conditioning
    print(f"mass change {m1 - m0:.4e} (oracle {dm_ref:.4e}, floor {dm_floor:.1e})")
    assert abs((m1 - m0) - dm_ref) <= max(1e-6 * m0, 4.0 * dm_floor)


@pytest.mark.parametrize("q,along", [(9, "z"), (19, "z"), (9, "x"), (19, "x")])
def test_pressure_driven_channel_is_poiseuille(q, along):
    """The GPU's channel at steady state (3000 steps): P linear between the faces (at
    -1/2 and n - 1/2 along the channel) and the plane Poiseuille profile across it,
    u = (dP/L)/(2 mu) s (H - s), s the distance from the wall, no cross flow."""
    cfg, dP = _channel(q, along)
    phi, u, P = _channel_fields(cfg)
    sim = _sim(cfg)
    sim.init_fields(phi, u, P)
    sim.step(3000)
    r = {k: _np(v) for k, v in sim.read().items()}
    rho, nu = cfg["rho_H"], cfg["nu_H"]
    D = 3 if q == 19 else 2
    # numpy axes of the fields (nz, ny, nx); the flow axis and the wall-normal axis
    flow_ax = {"z": (0 if q == 19 else 1), "x": 2}[along]
    wall_ax = 2 if along == "z" else (0 if q == 19 else 1)
    comp = {"z": (2 if q == 19 else 1), "x": 0}[along]   # J component along the flow
    Lc = r["P"].shape[flow_ax]
    H = r["P"].shape[wall_ax]
    pos = np.arange(Lc) + 0.5
    P_exact = dP / 2 - dP * pos / Lc
    Pm = np.moveaxis(r["P"], flow_ax, 0).reshape(Lc, -1)
    assert np.abs(Pm - P_exact[:, None]).max() <= 1e-3 * dP
    s = np.arange(H) + 0.5
    prof = (dP / Lc) / (2.0 * rho * nu) * s * (H - s)
    J = r["J"]
    ua = np.moveaxis(J[comp] / rho, wall_ax, 0).reshape(H, -1)
    assert np.abs(ua - prof[:, None]).max() <= 1e-2 * prof.max()
    cross = max(np.abs(J[k]).max() for k in range(D) if k != comp) / rho
    assert cross <= 1e-4 * prof.max()


def _drop_exit(q=9):
    """A water drop rising through air into an open top (P = 0), walls across x."""
    cfg = _cfg(9, (40, 30, 1), (W_, W_, P_), open_P=_open(yp=0.0), g=(0.0, 0.0, 0.0))
    cfg["name"] = "drop_exit"
    phi = pfinputs.drop_profile(cfg["shape"], (19.5, 22.0, 0.0), 6.0, cfg["W"])
    u = np.zeros((3,) + phi.shape)
    u[1] = 0.02 * phi
    return cfg, phi.astype(np.float32), u.astype(np.float32), np.zeros_like(phi, np.float32)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_drop_leaving_through_open_top(storage):
    """A drop crossing the open face within 300 steps (the interface meets the face):
    parity with the oracle at the storage's bar, and sum(phi) falling as the oracle's."""
    cfg, phi, u, P = _drop_exit()
    sim = _sim(cfg, storage=storage)
    sim.init_fields(phi, u, P)
    m0, _ = sim.mass()
    sim.step(300)
    r = {k: _np(v) for k, v in sim.read().items()}
    m1, bad = sim.mass()
    prm = _prm(cfg)
    h, g = O.init(prm, phi.astype(np.float64), u.astype(np.float64), P.astype(np.float64))
    mo0 = O.mass(h)
    h, g = O.run(prm, h, g, 300)
    ro = O.read(prm, h, g)
    dphi = np.abs(r["phi"] - ro["phi"]).max()
    eJ = _jerr(r["J"], ro["J"][:2], cfg["rho_H"])
    dm_ref = O.mass(h) - mo0
    print(f"\ndrop exit {storage}: max|dphi| {dphi:.2e}, rel J err {eJ:.2e}, "
          f"mass change {m1 - m0:.4e} (oracle {dm_ref:.4e})")
    assert not bad
    assert dm_ref < -1.0                     # water has left
    if storage == "fp32":
        assert dphi <= 1e-5
        assert eJ <= 1e-4
        assert abs((m1 - m0) - dm_ref) <= 1e-6 * m0
    else:
        assert dphi <= 5e-4
        assert eJ <= 1e-3
        assert abs((m1 - m0) - dm_ref) <= 1e-4 * m0


def _golden():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "make_oracle_runs.py")
    spec = importlib.util.spec_from_file_location("make_oracle_runs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_dam_break_reduced(storage):
    """The dam break (no-slip walls, open top at P = 0, rho_H/rho_L 1000, nu_water 4.9e-6)
    at 48x6x40 with a 16 x 20 column, 500 steps, against the oracle's stored run from the
    same start."""
    G = _golden()
    name = "dam_break_48x6x40"
    cfg, steps, d = G.load(name)
    assert str(d["source_sha1"]) == G.source_sha1(), "stale fixture: rerun make_oracle_runs.py"
    assert str(d["input_sha1"]) == G.input_sha1(cfg), "stale fixture: the seeded start changed"
    phi, u, P = pfinputs.fields(cfg)
    sim = _sim(cfg, storage=storage)
    sim.init_fields(phi, u, P)
    m0, _ = sim.mass()
    sim.step(steps)
    r = {k: _np(v) for k, v in sim.read().items()}
    m1, bad = sim.mass()
    dphi = np.abs(r["phi"] - d["phi"]).max()
    eJ = _jerr(r["J"], d["J"].astype(np.float64), cfg["rho_H"])
    dm_ref = float(d["mass1"]) - float(d["mass0"])
    print(f"\n{name} {storage} {steps} steps: max|dphi| {dphi:.2e}, rel J err {eJ:.2e}, "
          f"mass change {m1 - m0:.3e} (oracle {dm_ref:.3e})")
    assert not bad
    if storage == "fp32":
        assert dphi <= 1e-5
        assert eJ <= 1e-4
        assert abs((m1 - m0) - dm_ref) <= 1e-6 * m0
    else:
        assert dphi <= 5e-4
        assert eJ <= 1e-3
        assert abs((m1 - m0) - dm_ref) <= 1e-5 * m0


def test_open_faces_graph_batch_and_checkpoint(tmp_path):
    """An open context replayed from a captured graph, stepped in a pflb_step_many batch
    beside closed contexts, and saved and loaded, equals plain stepping bit for bit; a
    checkpoint is refused by a context whose open faces differ."""
    from paper_1812_00118_amd import Sim
    from paper_1812_00118_amd._lib import PflbError
    cfg, phi, u, P = _drop_exit()
    closed = dict(cfg, open_P=None)
    ref = _sim(cfg)
    ref.init_fields(phi, u, P)
    ref.step(40)
    want = [t.cpu().numpy() for t in ref.get_state()]
    a = _sim(cfg)
    a.init_fields(phi, u, P)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for n in (15, 15, 10):
            a.step_graph(n)
        st.synchronize()
    assert all(np.array_equal(x.cpu().numpy(), y) for x, y in zip(a.get_state(), want))
    b, c1, c2 = _sim(cfg), _sim(closed), _sim(closed)
    for s in (b, c1, c2):
        s.init_fields(phi, u, P)
    Sim.step_many([c1, b, c2], 40)
    assert all(np.array_equal(x.cpu().numpy(), y) for x, y in zip(b.get_state(), want))
    s = _sim(cfg)
    s.init_fields(phi, u, P)
    s.step(25)
    s.save(tmp_path / "open.bin")
    s2 = _sim(cfg)
    s2.load(tmp_path / "open.bin")
    s2.step(15)
    assert all(np.array_equal(x.cpu().numpy(), y) for x, y in zip(s2.get_state(), want))
    for other in (closed, dict(cfg, open_P=_open(yp=0.01))):
        s3 = _sim(other)
        with pytest.raises(PflbError):
            s3.load(tmp_path / "open.bin")
