"""The seeded input generators (CPU): the hashed state gives bitwise the same float32
values when built whole (as on the GPU, here through torch on the CPU) and when
evaluated at scattered sites on the host, and the oracle's site-by-site step reads it
through the lazy stand-ins exactly as it reads whole arrays."""
import numpy as np
import torch

import pfinputs
from oracle import pflbm as O


def test_hashed_state_whole_equals_sites():
    st = pfinputs.HashedState(19, (37, 5, 11), seed=8)
    h, g = st.device("cpu")
    n = 37 * 5 * 11
    lin = np.random.default_rng(1).permutation(n)[:500]
    hh, gh = st.host(lin)
    assert np.array_equal(h.reshape(19, -1).numpy()[:, lin], hh)
    assert np.array_equal(g.reshape(19, -1).numpy()[:, lin], gh)
    # indices near 2^28 (the largest domains) hash without overflow trouble
    big = np.array([2 ** 28 - 65, 2 ** 28 - 64 - 1000, 12345])
    hb, gb = st.host(big)
    hb2, gb2 = (np.stack([st._pop(torch.as_tensor(big), i, torch, _tc(st))[k].numpy()
                          for i in range(19)]) for k in (0, 1))
    assert np.array_equal(hb, hb2) and np.array_equal(gb, gb2)
    # values: h_i = a_i (phi + 0.02 noise) with phi in [0, 1), g_i = a_i O(0.07)
    a = np.array(pfinputs._MAG[19])[:, None]
    assert np.all(h.reshape(19, -1).numpy() >= -0.021 * a)
    assert np.all(h.reshape(19, -1).numpy() <= 1.021 * a)
    assert np.all(np.abs(g.reshape(19, -1).numpy()) <= 0.071 * a)


def _tc(st):
    f = lambda v: torch.tensor(np.float32(v))  # noqa: E731
    return {"1": f(1.0), "2": f(2.0), "0.02": f(0.02), "0.05": f(0.05),
            "a": [f(v) for v in st.a]}


def test_step_sites_on_lazy_hashed_state():
    shape = (9, 7, 6)
    cfg = dict(lattice=19, shape=shape, bc=("wall", "periodic", "wall"), rho_L=1.0,
               rho_H=1000.0, nu_L=0.05, nu_H=0.01, M=0.1, W=4.0, sigma=1e-3,
               g=(2e-5, -1e-5, 3e-5), eps=1e-10, hoc=1, dtheta_C=0.0)
    prm = O.Params.from_dict(pfinputs.model_params(cfg))
    st = pfinputs.HashedState(19, shape, seed=29)
    h, g = (t.numpy().astype(np.float64) for t in st.device("cpu"))
    sites = pfinputs.sample_sites(shape, 30, seed=3)
    hs, gs = O.step_sites(prm, h, g, sites)
    hl, gl = st.lazy()
    hz, gz = O.step_sites(prm, hl, gl, sites)
    assert np.array_equal(hs, hz) and np.array_equal(gs, gz)
    h1, g1 = O.step(prm, h, g)
    x, y, z = sites.T
    assert np.allclose(hz, h1[:, z, y, x], atol=1e-15, rtol=1e-13)
    assert np.allclose(gz, g1[:, z, y, x], atol=1e-13, rtol=1e-12)
