"""The step's result does not depend on how the domain is cut into workgroup chunks.

A workgroup of the fused step collides a chunk of planes (rows, in 2-D) and gathers the
plane below and above it for the neighbours' phi (and, in FP16S, their moments words).
The number of planes per chunk (the PFLB_BZ override of the library's choice) changes
which sites are gathered as own and which as neighbours, and for two-dimensional FP32
domains cut into chunks of one or two rows it switches between the marching kernel and
the short-chunk kernel.  Neither may change a single bit of the state."""
import os

import numpy as np
import pytest
import torch

import pfinputs

pytestmark = pytest.mark.gpu

W_, P_ = "wall", "periodic"


def _state(cfg, storage, bz, steps=5):
    from paper_1812_00118_amd import Sim
    old = os.environ.get("PFLB_BZ")
    os.environ["PFLB_BZ"] = str(bz)
    try:
        sim = Sim(cfg, storage=storage)
    finally:
        if old is None:
            del os.environ["PFLB_BZ"]
        else:
            os.environ["PFLB_BZ"] = old
    sim.set_state(*pfinputs.random_state(cfg["lattice"], cfg["shape"], seed=7))
    sim.step(steps)
    h, g = sim.get_state()
    return torch.cat([h.flatten(), g.flatten()]).cpu().numpy()


def _cfg(q, shape, bc, **kw):
    d = dict(lattice=q, shape=shape, bc=bc, rho_L=1.0, rho_H=1000.0, nu_L=0.05, nu_H=0.01,
             M=0.1, W=4.0, sigma=1e-3, g=(2e-5, -1e-5, 0.0), eps=1e-10, hoc=1, dtheta_C=0.0)
    d.update(kw)
    return d


D2 = [("d2q9-periodic", (P_, P_, P_)), ("d2q9-walls-y", (P_, W_, P_)),
      ("d2q9-walls-x", (W_, P_, P_)), ("d2q9-walls-xy", (W_, W_, P_))]


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
@pytest.mark.parametrize("name,bc", D2, ids=[c[0] for c in D2])
def test_d2q9_chunking(name, bc, storage):
    """A 150 x 37 D2Q9 box (ragged in both axes) from a seeded random state, 5 steps with
    chunks of 1, 2, 3, 4 and 8 rows: bitwise the same state."""
    cfg = _cfg(9, (150, 37, 1), bc)
    ref = _state(cfg, storage, 1)
    for bz in (2, 3, 4, 8):
        got = _state(cfg, storage, bz)
        assert np.array_equal(got, ref), (bz, int((got != ref).sum()))


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_rayleigh_taylor_chunking(storage):
    """The 256 x 1024 Rayleigh-Taylor workload from its own start, 5 steps with chunks of
    1, 2, 3 and 6 rows: bitwise the same state."""
    cfg = pfinputs.rayleigh_taylor()
    from paper_1812_00118_amd import Sim
    out = []
    for bz in (1, 2, 3, 6):
        os.environ["PFLB_BZ"] = str(bz)
        try:
            sim = Sim(cfg, storage=storage)
        finally:
            del os.environ["PFLB_BZ"]
        sim.init_fields(*pfinputs.fields(cfg))
        sim.step(5)
        h, g = sim.get_state()
        out.append(torch.cat([h.flatten(), g.flatten()]).cpu().numpy())
    for bz, got in zip((2, 3, 6), out[1:]):
        assert np.array_equal(got, out[0]), (bz, int((got != out[0]).sum()))


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
@pytest.mark.parametrize("bc", [(P_, P_, W_), (W_, W_, W_)], ids=["walls-z", "walls-all"])
def test_d3q19_chunking(bc, storage):
    """A 70 x 9 x 37 D3Q19 box from a seeded random state, 5 steps with chunks of 5, 8, 13
    and 37 planes: bitwise the same state."""
    cfg = _cfg(19, (70, 9, 37), bc, g=(2e-5, -1e-5, 3e-5))
    ref = _state(cfg, storage, 5)
    for bz in (8, 13, 37):
        got = _state(cfg, storage, bz)
        assert np.array_equal(got, ref), (bz, int((got != ref).sum()))
