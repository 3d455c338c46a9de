"""Batched stepping (pflb_step_many) against each context's own pflb_step, through the C ABI.

The batched launch runs the same per-site code as the single-context step with each
context's own buffers and parameters, so every context must end bitwise equal to its own
run (and with the same step count), whatever its buffer parity, storage, physical
parameters or wall velocities.
"""
import numpy as np
import pytest
import torch

import pfinputs

pytestmark = pytest.mark.gpu

W_, P_ = "wall", "periodic"


def _cfg(q, shape, bc, **kw):
    d = dict(lattice=q, shape=shape, bc=bc, rho_L=1.0, rho_H=1000.0, nu_L=0.05, nu_H=0.01,
             M=0.1, W=4.0, sigma=1e-3, g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1, dtheta_C=0.0)
    d.update(kw)
    return d


def _sim(cfg, storage):
    from paper_1812_00118_amd import Sim
    return Sim(cfg, storage=storage)


# per-context physical parameters of one batch (same lattice, sizes and walls)
VARIANTS = [
    dict(),
    dict(rho_H=10.0, sigma=5e-3, hoc=0),
    dict(rho_H=100.0, nu_L=0.02, nu_H=0.004, M=0.05, W=5.0),
    dict(rho_H=3.0, g=(1e-5, -2e-5, 0.0), sigma=2e-3),
    dict(rho_H=500.0, dtheta_C=0.1),
]


def _pairs(q, shape, bc, storage, variants, pre_steps, extra=None):
    """Two identical contexts per variant (one for the batch, one stepped alone) from a
    seeded random state; pre_steps[k] steps are taken first so that the contexts hold
    their current state in different buffers."""
    batch, alone = [], []
    for k, v in enumerate(variants):
        kw = dict(v)
        if extra:
            kw.update(extra(k))
        if q == 9 and "g" in kw:
            kw["g"] = (kw["g"][0], kw["g"][1], 0.0)
        cfg = _cfg(q, shape, bc, **kw)
        h0, g0 = pfinputs.random_state(q, shape, seed=100 + k, h_noise=0.01, g_noise=0.01)
        a, b = _sim(cfg, storage), _sim(cfg, storage)
        for s in (a, b):
            s.set_state(h0, g0)
            if pre_steps[k]:
                s.step(pre_steps[k])
        batch.append(a)
        alone.append(b)
    return batch, alone


def _assert_same(batch, alone):
    for k, (a, b) in enumerate(zip(batch, alone)):
        ha, ga = a.get_state()
        hb, gb = b.get_state()
        assert torch.isfinite(hb).all() and torch.isfinite(gb).all(), k
        assert torch.equal(ha, hb) and torch.equal(ga, gb), (
            k, (ha - hb).abs().max().item(), (ga - gb).abs().max().item())
        assert a.steps == b.steps, (k, a.steps, b.steps)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_step_many_d2q9_mixed_parameters(storage):
    from paper_1812_00118_amd import Sim
    batch, alone = _pairs(9, (67, 45, 1), (P_, W_, P_), storage, VARIANTS, [0, 1, 0, 3, 2])
    Sim.step_many(batch, 7)
    for s in alone:
        s.step(7)
    _assert_same(batch, alone)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_step_many_d3q19_walls_one_moving(storage):
    """A context with a sliding top wall is stepped on its own (by its moving-wall kernel),
    the resting ones in one batched launch: all end as their own steps leave them."""
    from paper_1812_00118_amd import Sim

    def wall(k):
        w = np.zeros((6, 3))
        if k == 1:
            w[5] = (0.02, -0.01, 0.0)
        return dict(wall_u=w)

    batch, alone = _pairs(19, (37, 21, 19), (P_, P_, W_), storage, VARIANTS[:3], [1, 0, 0],
                          extra=wall)
    Sim.step_many(batch, 5)
    for s in alone:
        s.step(5)
    _assert_same(batch, alone)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_step_many_with_a_wetting_context(storage):
    """A context whose walls prescribe contact angles is stepped on its own (by the
    kernel variant that applies the wetting rule), the others batched: all end as their
    own steps leave them."""
    from paper_1812_00118_amd import Sim

    def wet(k):
        return dict(wet_cos=(0, 0, 0.5, -0.3, 0, 0)) if k == 2 else {}

    batch, alone = _pairs(9, (67, 45, 1), (P_, W_, P_), storage, VARIANTS, [0, 1, 0, 3, 2],
                          extra=wet)
    Sim.step_many(batch, 6)
    for s in alone:
        s.step(6)
    _assert_same(batch, alone)


def test_step_many_d3q19_periodic_full_tile():
    from paper_1812_00118_amd import Sim
    batch, alone = _pairs(19, (64, 8, 24), (P_, P_, P_), "fp32", VARIANTS[:2], [0, 1])
    Sim.step_many(batch, 4)
    for s in alone:
        s.step(4)
    _assert_same(batch, alone)


def test_step_many_seventeen_contexts():
    """17 contexts: two launches per step (16 + 1)."""
    from paper_1812_00118_amd import Sim
    variants = [VARIANTS[k % len(VARIANTS)] for k in range(17)]
    batch, alone = _pairs(9, (32, 32, 1), (P_, P_, P_), "fp32", variants,
                          [k % 2 for k in range(17)])
    Sim.step_many(batch, 4)
    for s in alone:
        s.step(4)
    _assert_same(batch, alone)


def test_step_many_zero_steps_and_rejections():
    from paper_1812_00118_amd import PflbError, Sim
    cfg = _cfg(9, (32, 32, 1), (P_, P_, P_))
    a, b = _sim(cfg, "fp32"), _sim(cfg, "fp32")
    h0, g0 = pfinputs.random_state(9, (32, 32, 1), seed=5)
    for s in (a, b):
        s.set_state(h0, g0)
    Sim.step_many([a, b], 0)
    assert a.steps == 0 and b.steps == 0
    with pytest.raises(PflbError):
        Sim.step_many([a, a], 1)          # the same context twice
    with pytest.raises(PflbError):
        Sim.step_many([a, _sim(_cfg(9, (32, 16, 1), (P_, P_, P_)), "fp32")], 1)   # sizes
    with pytest.raises(PflbError):
        Sim.step_many([a, _sim(cfg, "fp16s")], 1)                                   # storage
    with pytest.raises(PflbError):
        Sim.step_many([a, _sim(_cfg(9, (32, 32, 1), (P_, W_, P_)), "fp32")], 1)    # walls
    with pytest.raises(PflbError):
        Sim.step_many([a, b], -1)
    # nothing was stepped by the rejected calls
    assert a.steps == 0 and b.steps == 0
