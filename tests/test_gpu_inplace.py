"""In-place FP32 storage (one state buffer, two alternating layouts) against the FP64
oracle and against the two-buffer pull storage, through the C ABI.

The arithmetic per site is the pull step's (same gathers in index order, same phi sum,
same collision), so every population is compared with the oracle at the one-step bar
after 1, 2 and 3 steps (both layouts, both step kernels), and the 1000-step runs at the
plain bar (max|d phi| <= 1e-5, relative momentum error <= 1e-4).
"""
import numpy as np
import pytest
import torch

import pfinputs
from oracle import pflbm as O

pytestmark = pytest.mark.gpu

W_, P_ = "wall", "periodic"


def _sim(cfg, storage="fp32_inplace"):
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


CASES = [
    ("d2q9-periodic", 9, (67, 45, 1), (P_, P_, P_)),
    ("d2q9-walls", 9, (70, 33, 1), (W_, W_, P_)),
    ("d2q9-tiny", 9, (3, 2, 1), (P_, W_, P_)),
    ("d3q19-periodic", 19, (37, 21, 19), (P_, P_, P_)),
    ("d3q19-walls-z", 19, (70, 9, 13), (P_, P_, W_)),
    ("d3q19-walls-all", 19, (17, 11, 6), (W_, W_, W_)),
    ("d3q19-single-walls", 19, (1, 1, 1), (W_, W_, W_)),
    ("d3q19-single", 19, (1, 1, 1), (P_, P_, P_)),
]


@pytest.mark.parametrize("name,q,shape,bc", CASES, ids=[c[0] for c in CASES])
def test_steps_from_random_state(name, q, shape, bc):
    """Every population after 1, 2 and 3 steps (layout 0 -> 1 -> 0 -> 1) from a seeded
    random state against the oracle; sum(phi) conserved; the pull storage's state after
    the same steps is reported beside it."""
    cfg = _cfg(q, shape, bc, g=(2e-5, -1e-5, 3e-5) if q == 19 else (2e-5, -1e-5, 0))
    h0, g0 = pfinputs.random_state(q, shape, seed=sum(name.encode()) + 11)
    sim = _sim(cfg)
    ref = _sim(cfg, "fp32")
    sim.set_state(h0, g0)
    ref.set_state(h0, g0)
    hd, gd = (_np(t) for t in sim.get_state())
    assert np.array_equal(hd, h0) and np.array_equal(gd, g0)
    m0, _ = sim.mass()
    prm = _prm(cfg)
    hr, gr = h0.astype(np.float64), g0.astype(np.float64)
    for k in range(1, 4):
        sim.step(1)
        ref.step(1)
        hr, gr = O.step(prm, hr, gr)
        h1, g1 = (_np(t) for t in sim.get_state())
        hp, gp = (_np(t) for t in ref.get_state())
        print(f"\n{name} step {k}: in-place vs pull max|dh| {np.abs(h1 - hp).max():.1e} "
              f"max|dg| {np.abs(g1 - gp).max():.1e}")
        _close(h1, hr)
        _close(g1, gr)
        m1, bad = sim.mass()
        assert not bad
        assert abs(m1 - m0) <= 1e-7 * abs(m0)
        # the step count parity picks the layout; the read-out follows it
        r = sim.read()
        rp = ref.read()
        assert torch.allclose(r["phi"], rp["phi"], rtol=0, atol=1e-6)
        assert torch.allclose(r["P"], rp["P"], rtol=1e-4, atol=1e-6)


def test_contact_angles_one_step():
    """Wetting walls (the ghost rule applies to the phi field both kernels read)."""
    cfg = _cfg(19, (17, 11, 6), (W_, W_, W_), wet_cos=(0.3, -0.5, 0.8, -0.2, 0.6, -0.7),
               g=(1e-5, -2e-5, 0.0))
    h0, g0 = pfinputs.random_state(19, cfg["shape"], seed=77)
    sim = _sim(cfg)
    sim.set_state(h0, g0)
    hr, gr = h0.astype(np.float64), g0.astype(np.float64)
    for _ in range(2):
        sim.step(1)
        hr, gr = O.step(_prm(cfg), hr, gr)
    h1, g1 = (_np(t) for t in sim.get_state())
    _close(h1, hr)
    _close(g1, gr)


def _walls(**faces):
    w = np.zeros((6, 3))
    for k, v in faces.items():
        w[("xm", "xp", "ym", "yp", "zm", "zp").index(k)] = v
    return w


MOVING = [
    ("d3q19-moving-all", 19, (17, 11, 6), (W_, W_, W_),
     _walls(xm=(0, 0.01, -0.01), xp=(0, -0.02, 0.005), ym=(0.015, 0, 0.01),
            yp=(-0.005, 0, -0.01), zm=(0.01, 0.02, 0), zp=(-0.01, 0.005, 0))),
    ("d2q9-moving", 9, (70, 33, 1), (W_, W_, P_),
     _walls(xm=(0, 0.01, 0), xp=(0, -0.02, 0), ym=(0.015, 0, 0), yp=(-0.005, 0, 0))),
    ("d3q19-single-moving", 19, (1, 1, 1), (W_, W_, W_),
     _walls(xm=(0, 0.01, 0.02), xp=(0, -0.01, 0.01), ym=(0.02, 0, 0.01),
            yp=(0.01, 0, -0.02), zm=(0.01, -0.01, 0), zp=(0.02, 0.01, 0))),
]


@pytest.mark.parametrize("name,q,shape,bc,wall", MOVING, ids=[c[0] for c in MOVING])
def test_moving_walls_three_steps(name, q, shape, bc, wall):
    """Moving walls in place (momentum-corrected bounce-back at every wall face, edges and
    corners): every population after 1, 2 and 3 steps (both layouts) against the oracle,
    and sum(phi) changing as the oracle's."""
    cfg = _cfg(q, shape, bc, wall_u=wall,
               g=(2e-5, -1e-5, 3e-5) if q == 19 else (2e-5, -1e-5, 0))
    h0, g0 = pfinputs.random_state(q, shape, seed=sum(name.encode()) + 3)
    sim = _sim(cfg)
    sim.set_state(h0, g0)
    m0, _ = sim.mass()
    prm = _prm(cfg)
    hr, gr = h0.astype(np.float64), g0.astype(np.float64)
    for k in range(3):
        sim.step(1)
        hr, gr = O.step(prm, hr, gr)
        h1, g1 = (_np(t) for t in sim.get_state())
        _close(h1, hr)
        _close(g1, gr)
    m1, bad = sim.mass()
    assert not bad
    assert abs((m1 - m0) - (O.mass(hr) - O.mass(h0.astype(np.float64)))) <= 1e-7 * abs(m0)


def test_static_droplet_1000_steps():
    """The D2Q9 static droplet (64x64, rho 1000, R 16): 1000 steps at the plain bar."""
    cfg = pfinputs.static_droplet()
    phi, u, P = pfinputs.fields(cfg)
    sim = _sim(cfg)
    sim.init_fields(phi, u, P)
    m0, _ = sim.mass()
    sim.step(1000)
    r = {k: _np(v) for k, v in sim.read().items()}
    m1, bad = sim.mass()
    prm = _prm(cfg)
    h, g = O.init(prm, phi.astype(np.float64), u.astype(np.float64), P.astype(np.float64))
    h, g = O.run(prm, h, g, 1000)
    ro = O.read(prm, h, g)
    assert not bad
    assert np.abs(r["phi"] - ro["phi"]).max() <= 1e-5
    assert _jerr(r["J"], ro["J"][:2], cfg["rho_H"]) <= 1e-4
    assert abs(m1 - m0) / m0 <= 1e-7


def _golden():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "make_oracle_runs.py")
    spec = importlib.util.spec_from_file_location("make_oracle_runs", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["rising_bubble_24", "droplet_impact_36x28x30"])
def test_d3q19_reduced_1000_steps(name):
    """The reduced D3Q19 workloads, 1000 steps against the oracle's stored runs."""
    G = _golden()
    cfg, steps, d = G.load(name)
    assert str(d["source_sha1"]) == G.source_sha1(), "stale fixture: rerun make_oracle_runs.py"
    assert str(d["input_sha1"]) == G.input_sha1(cfg)
    phi, u, P = pfinputs.fields(cfg)
    sim = _sim(cfg)
    sim.init_fields(phi, u, P)
    m0, _ = sim.mass()
    sim.step(steps)
    r = {k: _np(v) for k, v in sim.read().items()}
    m1, bad = sim.mass()
    dphi = np.abs(r["phi"] - d["phi"]).max()
    eJ = _jerr(r["J"], d["J"].astype(np.float64), cfg["rho_H"])
    print(f"\n{name} in-place {steps} steps: max|dphi| {dphi:.2e}, rel J err {eJ:.2e}")
    assert not bad
    assert dphi <= 1e-5
    assert eJ <= 1e-4
    assert abs(m1 - m0) / m0 <= 1e-6


def test_graph_batch_checkpoint_and_buffers(tmp_path):
    """Graph replay (odd and even step counts, so both layouts start a capture), a
    pflb_step_many call (in-place contexts are stepped one by one) and a checkpoint saved
    in the odd layout all equal plain stepping bit for bit; the second state buffer needs
    no bytes; a pull-storage context refuses the checkpoint."""
    from paper_1812_00118_amd import Sim
    from paper_1812_00118_amd._lib import PflbError
    cfg = pfinputs.rayleigh_taylor(nx=64, ny=160)
    phi, u, P = pfinputs.fields(cfg)
    a, b = _sim(cfg), _sim(cfg)
    assert b.bufs[1].numel() == 0
    a.init_fields(phi, u, P)
    b.init_fields(phi, u, P)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for n in (7, 7, 4, 7):
            a.step_graph(n)
            b.step(n)
            ha, ga = a.get_state()
            hb, gb = b.get_state()
            st.synchronize()
            assert torch.equal(ha, hb) and torch.equal(ga, gb), n
    c, c2 = _sim(cfg), _sim(cfg)
    c.init_fields(phi, u, P)
    c2.init_fields(phi, u, P)
    Sim.step_many([c, c2], 25)
    for s in (c, c2):
        assert all(torch.equal(x, y) for x, y in zip(s.get_state(), b.get_state()))
    c.save(tmp_path / "ip.bin")               # 25 steps: the odd layout
    d = _sim(cfg)
    d.load(tmp_path / "ip.bin")
    assert d.steps == 25
    d.step(5)
    b.step(5)
    assert all(torch.equal(x, y) for x, y in zip(d.get_state(), b.get_state()))
    with pytest.raises(PflbError):
        _sim(cfg, "fp32").load(tmp_path / "ip.bin")


def test_maximum_domain_one_step_sampled():
    """Beyond 2^28 sites (64-bit addresses, 4.5e8 sites in one 68 GB buffer): one step
    from a hashed state filled on the GPU, checked at sampled sites against the oracle's
    site-by-site evaluation of the same hashed values; a second step conserves sum(phi)."""
    shape = (1500, 1000, 300)
    if torch.cuda.mem_get_info()[0] < 150 * 2 ** 30:
        pytest.skip("needs about 150 GiB of free device memory")
    cfg = _cfg(19, shape, (W_, W_, W_), g=(2e-5, -1e-5, 3e-5))
    st = pfinputs.HashedState(19, shape, seed=31)
    sim = _sim(cfg)
    h0, g0 = st.device(sim.device)
    sim.set_state(h0, g0)
    del h0, g0
    torch.cuda.empty_cache()
    m0, bad0 = sim.mass()
    sim.step(1)
    m1, bad1 = sim.mass()
    assert not bad0 and not bad1
    assert abs(m1 - m0) <= 1e-7 * abs(m0)
    h1, g1 = sim.get_state()
    sites = pfinputs.sample_sites(shape, 300, seed=5)
    x, y, z = (torch.as_tensor(v, device=h1.device) for v in sites.T)
    hg = _np(h1[:, z, y, x])
    gg = _np(g1[:, z, y, x])
    del h1, g1
    torch.cuda.empty_cache()
    sim.step(1)
    m2, bad2 = sim.mass()
    assert not bad2 and abs(m2 - m0) <= 1e-7 * abs(m0)
    del sim
    torch.cuda.empty_cache()
    hl, gl = st.lazy()
    hr, gr = O.step_sites(_prm(cfg), hl, gl, sites)
    _close(hg, hr)
    _close(gg, gr)
