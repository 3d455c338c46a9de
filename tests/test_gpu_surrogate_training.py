"""The trained surrogate against the method without it, on held-out seeds.

The network is trained on the GPU by the library's own kernels on (t, t + 16) pairs
that the solver generates for the seeded droplet family (D2Q9 256^2), then compared
on test seeds with what is available without it: persistence (the state at t as the
prediction of t + 16) and the untrained network.  The guarded hand-over keeps the
mass drift within its stated bound whatever the network predicts."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import pfinputs
    from paper_1812_00118_amd import surrogate as S, sur_train as T
    tr = T.Dataset(range(16), pfinputs.drops, t0=64, n_states=9)
    te = T.Dataset(range(2000, 2004), pfinputs.drops, t0=64, n_states=9)
    sur = S.Surrogate(256, 256, 8, T.normalisation(tr))
    sur.set_params(S.init_params(0))
    before = T.evaluate(sur, te)
    losses = T.train(sur, tr, 300, 8, 1e-3, seed=1)
    after = T.evaluate(sur, te)
    print(f"untrained {before}\ntrained {after}\nloss {losses[:3]} ... {losses[-3:]}")
    return sur, before, after, losses


def test_trained_network_beats_persistence_and_untrained(trained):
    _, before, after, losses = trained
    assert np.all(np.isfinite(losses))
    # the normalised residual has unit variance over the training pairs; persistence
    # scores mean(y^2) and the untrained net (small head) about the same
    assert after["mse"] < 0.5 * after["mse_persistence"], after
    assert after["mse"] < 0.5 * before["mse"], (before, after)
    assert after["phi_err"] < after["phi_err_persistence"], after


def test_guarded_advance_keeps_mass_within_bound(trained):
    import pfinputs
    from paper_1812_00118_amd import Sim
    sur = trained[0]
    cfg = pfinputs.drops(2001)
    sim = Sim(pfinputs.model_params(cfg))
    sim.init_fields(*pfinputs.fields(cfg))
    sim.step(64)
    m0, bad0 = sim.mass()
    windows = 6
    nf = sur.advance_guarded(sim, windows, mass_tol=1e-3,
                             phi_tol=0.05, check_every=2)
    m1, bad1 = sim.mass()
    print(f"fallbacks {nf} of {windows}, mass drift {(m1 - m0) / m0:.3e}")
    assert not bad0 and not bad1
    assert 0 <= nf <= windows and sim.steps == 64 + 16 * windows
    # each accepted window moves sum(phi) by at most 1e-3 relative; fallbacks conserve it
    assert abs(m1 - m0) <= windows * 1e-3 * abs(m0) + 1e-6 * abs(m0)
