"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Closed forms, exact invariants and special cases that a plausible mistake in the
oracle (a dropped term, a wrong sign or index, a transposed operand) would break.
"""
import numpy as np
import pytest

from oracle import pflbm as O
from oracle.lattice import D2Q9, D3Q19, T

LATS = [D2Q9, D3Q19]


def _prm(q, shape, bc=None, **kw):
    base = dict(rho_L=1.0, rho_H=1000.0, nu_L=0.05, nu_H=0.02, M=0.1, W=4.0,
                sigma=1e-3)
    base.update(kw)
    if bc is None:
        bc = (O.PERIODIC,) * 3
    return O.Params(q, shape, bc, **base)


# --------------------------------------------------------------------------- lattice

@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_lattice_isotropy(lat):
    """sum w = 1, sum w c = 0, sum w c c = T I, sum w c_a^4 = 3 T^2, sum w c_a^2 c_b^2 = T^2
    (T = 1/3), odd moments vanish, and opp(i) is the opposite velocity."""
    c, w = lat.c.astype(float), lat.w
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-15
    D = lat.D
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(second[:D, :D], T * np.eye(D), atol=1e-15)
    third = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(third).max() < 1e-15
    for a in range(D):
        assert abs((w * c[:, a] ** 4).sum() - 3 * T * T) < 1e-15
        for b in range(D):
            if a != b:
                assert abs((w * c[:, a] ** 2 * c[:, b] ** 2).sum() - T * T) < 1e-15
    assert np.array_equal(c[lat.opp], -c)
    assert lat.opp[0] == 0


# ---------------------------------------------------------------- central differences

@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_cd_exact_on_polynomials(lat):
    """On polynomials of degree <= 4 the central differences of Section 2 are exactly
    grad_CD = grad + (T/2) grad(lap) and lap_CD = lap + (T/4) lap(lap) (Taylor series:
    odd terms cancel, 4th-order isotropy fixes the remainder).  Derivatives by sympy."""
    import sympy as sp
    X, Y, Z = sp.symbols("x y z")
    if lat.D == 2:
        poly = (sp.Rational(3, 10) * X ** 3 - sp.Rational(1, 5) * X * Y ** 2
                + sp.Rational(1, 20) * X ** 2 * Y ** 2 + sp.Rational(7, 10) * Y + Y ** 4 / 7)
        axes = (X, Y)
    else:
        poly = (sp.Rational(3, 10) * X ** 3 - sp.Rational(1, 5) * X * Y * Z
                + sp.Rational(1, 20) * X ** 2 * Z ** 2 + Y ** 4 / 10 + sp.Rational(7, 10) * Z
                + X * Y ** 2 * Z / 3)
        axes = (X, Y, Z)
    lap = sum(sp.diff(poly, a, 2) for a in axes)
    lap2 = sum(sp.diff(lap, a, 2) for a in axes)
    Tq = sp.Rational(1, 3)
    want_g = [sp.diff(poly, a) + Tq / 2 * sp.diff(lap, a) for a in axes]
    want_l = lap + Tq / 4 * lap2
    n = 12
    shape = (n, n, n if lat.D == 3 else 1)
    z, y, x = np.meshgrid(np.arange(shape[2], dtype=float), np.arange(n, dtype=float),
                          np.arange(n, dtype=float), indexing="ij")
    ev = lambda e: sp.lambdify((X, Y, Z), e, "numpy")(x, y, z) + 0 * x
    prm = _prm(lat.Q, shape)
    nb = O.phi_stencil(ev(poly), lat, prm.bc)
    G = O.grad_cd(lat, nb)
    L = O.lap_cd(lat, nb)
    inner = (slice(1, -1) if lat.D == 3 else slice(None), slice(1, -1), slice(1, -1))
    for a in range(lat.D):
        assert np.allclose(G[a][inner], ev(want_g[a])[inner], rtol=1e-12, atol=1e-9)
    assert np.allclose(L[inner], ev(want_l)[inner], rtol=1e-12, atol=1e-9)
    # and the plain derivative is NOT recovered (the correction terms are real)
    assert not np.allclose(L[inner], ev(lap)[inner], rtol=1e-6)


# --------------------------------------------------------------- equilibrium moments

def _rand_site(lat, rng, S=64):
    u = 0.05 * rng.standard_normal((3, S))
    if lat.D == 2:
        u[2] = 0
    phi = rng.uniform(-0.05, 1.05, S)
    grad = 0.2 * rng.standard_normal((3, S))
    if lat.D == 2:
        grad[2] = 0
    lap = 0.1 * rng.standard_normal(S)
    return u, phi, grad, lap


def _mom(lat, f, order):
    c = lat.c.astype(float)
    if order == 0:
        return f.sum(0)
    if order == 1:
        return np.einsum("ia,i...->a...", c, f)
    return np.einsum("ia,ib,i...->ab...", c, c, f)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_gamma_and_heq_moments(lat):
    """sum Gamma = 1, sum c Gamma = u, sum c c Gamma = T I + u u;
    sum h^eq = phi, sum c h^eq = phi u + T theta n."""
    rng = np.random.default_rng(1)
    u, phi, grad, lap = _rand_site(lat, rng)
    prm = _prm(lat.Q, (4, 4, 4 if lat.D == 3 else 1))
    Gam = O.gamma(lat, u)
    D = lat.D
    assert np.allclose(_mom(lat, Gam, 0), 1.0, atol=1e-14)
    assert np.allclose(_mom(lat, Gam, 1)[:D], u[:D], atol=1e-15)
    want2 = T * np.eye(3)[:, :, None] + u[:, None] * u[None, :]
    assert np.allclose(_mom(lat, Gam, 2)[:D, :D], want2[:D, :D], atol=1e-15)
    theta = O.theta_of(prm, phi, grad, lap)
    n = O.normal_of(prm, grad)
    heq = O.h_eq(lat, phi, Gam, theta, n)
    assert np.allclose(heq.sum(0), phi, atol=1e-15)
    assert np.allclose(_mom(lat, heq, 1)[:D], (phi * u + T * theta * n)[:D], atol=1e-15)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("hoc", [0, 1])
def test_forcing_and_geq_moments(lat, hoc):
    """sum K = rho_dif u.grad(phi); sum c K = mu grad(phi) + F;
    sum g^eq = P/T - rho_dif u.grad/2; sum c g^eq = (rho + lap(rho)/4) u - (mu grad + F)/2
    (lap(rho) term only with the high-order correction)."""
    rng = np.random.default_rng(2 + hoc)
    u, phi, grad, lap = _rand_site(lat, rng)
    prm = _prm(lat.Q, (4, 4, 4 if lat.D == 3 else 1), hoc=hoc, g=(1e-3, -2e-3, 3e-3))
    D = lat.D
    rho = prm.rho_L + phi * prm.rho_dif
    mu = O.mu_chm(prm, phi, lap)
    F = prm.g[:, None] * rho
    if D == 2:
        F[2] = 0
    P = 0.01 * rng.standard_normal(phi.shape)
    Gam = O.gamma(lat, u)
    K = O.forcing_K(lat, prm, Gam, u, grad, mu, F)
    ug = (u * grad).sum(0)
    assert np.allclose(K.sum(0), prm.rho_dif * ug, rtol=1e-12, atol=1e-12)
    assert np.allclose(_mom(lat, K, 1)[:D], (mu * grad + F)[:D], rtol=1e-12, atol=1e-12)
    geq = O.g_eq(lat, prm, rho, P, Gam, K, u, lap)
    assert np.allclose(geq.sum(0), P / T - prm.rho_dif * ug / 2, rtol=1e-12, atol=1e-10)
    rho_p = rho + (prm.rho_dif * lap / 4 if hoc else 0.0)
    want = rho_p * u - (mu * grad + F) / 2
    assert np.allclose(_mom(lat, geq, 1)[:D], want[:D], rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_hermite_filter(lat):
    """Phi_i : Pi has zero 0th and 1st moments and 2nd moment Pi (for the D-dim block);
    for a non-equilibrium that is itself pure 2nd-order Hermite content the filter
    returns it unchanged."""
    rng = np.random.default_rng(3)
    D = lat.D
    neq = rng.standard_normal((lat.Q, 16))
    proj, Pi = O.hermite_filter(lat, neq)
    assert np.allclose(proj.sum(0), 0, atol=1e-13)
    assert np.allclose(_mom(lat, proj, 1), 0, atol=1e-13)
    assert np.allclose(_mom(lat, proj, 2)[:D, :D], Pi[:D, :D], atol=1e-13)
    # pure Hermite content: w_i/(2T^2)(c c - T I):A for a symmetric A
    A = rng.standard_normal((3, 3, 16))
    A = A + A.transpose(1, 0, 2)
    if D == 2:
        A[2, :] = 0
        A[:, 2] = 0
    c = lat.c.astype(float)
    H = np.stack([lat.w[i] / (2 * T * T) * (np.einsum("a,b,ab...->...", c[i], c[i], A)
                                           - T * np.einsum("aa...->...", A))
                  for i in range(lat.Q)])
    proj2, _ = O.hermite_filter(lat, H)
    assert np.allclose(proj2, H, atol=1e-13)


# ------------------------------------------------------------------ collision level

@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_filtered_equals_bgk_at_tau_one(lat):
    """With tau_mix = 1 (nu = T/2 in both phases) the filtered update of Eq. 10 equals
    the BGK-with-force update of Eq. 5, g* = g^eq + K, whatever the non-equilibrium."""
    shape = (6, 5, 4 if lat.D == 3 else 1)
    prm = _prm(lat.Q, shape, nu_L=T / 2, nu_H=T / 2, g=(1e-4, 2e-4, -1e-4))
    h, g = _random(lat, shape, 11)
    phi = h.sum(0)
    nb = O.phi_stencil(phi, lat, prm.bc)
    hstar, gstar, m = O.collide(lat, prm, h, g, nb)
    Gam = O.gamma(lat, m["u"])
    K = O.forcing_K(lat, prm, Gam, m["u"], m["grad"], m["mu"], m["F"])
    geq = O.g_eq(lat, prm, m["rho"], m["P"], Gam, K, m["u"], m["lap"])
    assert np.allclose(gstar, geq + K, atol=1e-12)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_collision_conserves(lat):
    """Per site: sum h* = sum h (phi conserved); sum c g* = sum c g + mu grad + F
    (momentum changes only by the force); the h first moment relaxes towards phi u +
    T theta n at rate 1/tau_phi."""
    shape = (6, 5, 4 if lat.D == 3 else 1)
    prm = _prm(lat.Q, shape, g=(1e-4, 2e-4, -1e-4))
    h, g = _random(lat, shape, 12)
    nb = O.phi_stencil(h.sum(0), lat, prm.bc)
    hstar, gstar, m = O.collide(lat, prm, h, g, nb)
    D = lat.D
    assert np.allclose(hstar.sum(0), h.sum(0), atol=1e-14)
    dJ = _mom(lat, gstar, 1) - _mom(lat, g, 1)
    assert np.allclose(dJ[:D], (m["mu"] * m["grad"] + m["F"])[:D], atol=1e-11)
    j_h = _mom(lat, h, 1)
    target = m["phi"] * m["u"] + T * m["theta"] * m["n"]
    want = j_h - (j_h - target) / prm.tau_phi
    assert np.allclose(_mom(lat, hstar, 1)[:D], want[:D], atol=1e-14)


def _random(lat, shape, seed):
    import pfinputs
    h, g = pfinputs.random_state(lat.Q, shape, seed)
    return h.astype(np.float64), g.astype(np.float64)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_density_scale_invariance(lat):
    """(rho_L, rho_H, sigma, P, g-set) -> lambda (...) with lambda = 2^-7 leaves phi and u
    unchanged and scales P and J by lambda, exactly (power-of-two scaling commutes with
    rounding), over 20 steps with walls and gravity."""
    shape = (8, 6, 5 if lat.D == 3 else 1)
    bc = (O.PERIODIC, O.WALL, O.WALL if lat.D == 3 else O.PERIODIC)
    lam = 2.0 ** -7
    kw = dict(g=(1e-4, -2e-4, 1e-4))
    p1 = _prm(lat.Q, shape, bc, **kw)
    p2 = _prm(lat.Q, shape, bc, rho_L=lam, rho_H=1000.0 * lam, sigma=1e-3 * lam, **kw)
    h, g = _random(lat, shape, 21)
    h1, g1 = O.run(p1, h, g, 20)
    h2, g2 = O.run(p2, h, g * lam, 20)
    r1, r2 = O.read(p1, h1, g1), O.read(p2, h2, g2)
    assert np.array_equal(h1, h2)
    assert np.array_equal(r1["u"], r2["u"])
    assert np.array_equal(r1["P"] * lam, r2["P"])
    assert np.array_equal(r1["J"] * lam, r2["J"])


# ------------------------------------------------------------- streaming / boundaries

@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
@pytest.mark.parametrize("walls", [False, True])
def test_mass_conservation(lat, walls):
    """sum_x phi is conserved to rounding over many steps (periodic and walled)."""
    shape = (10, 9, 7 if lat.D == 3 else 1)
    bc = (O.PERIODIC, O.WALL if walls else O.PERIODIC,
          O.WALL if (walls and lat.D == 3) else O.PERIODIC)
    prm = _prm(lat.Q, shape, bc, g=(0, -1e-5, 0))
    h, g = _random(lat, shape, 31)
    m0 = O.mass(h)
    h1, g1 = O.run(prm, h, g, 100)
    assert abs(O.mass(h1) - m0) / abs(m0) < 1e-12


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_stream_is_a_permutation(lat):
    """Streaming with periodic and wall axes moves every population value exactly once."""
    shape = (5, 4, 3 if lat.D == 3 else 1)
    prm = _prm(lat.Q, shape, (O.WALL, O.PERIODIC, O.WALL if lat.D == 3 else O.PERIODIC))
    f = np.arange(lat.Q * np.prod(shape), dtype=float).reshape((lat.Q,) + shape[::-1])
    out = O.stream(lat, prm, f)
    assert np.array_equal(np.sort(out.ravel()), np.sort(f.ravel()))
    # a population pulled across a wall came from the same site, opposite direction
    i = 1  # +x
    assert np.array_equal(out[i][:, :, 0], f[lat.opp[i]][:, :, 0])
    assert np.array_equal(out[i][:, :, 1:], f[i][:, :, :-1])


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_init_recovers_fields(lat):
    """The equilibrium start returns u0 and P0 when read back (J = (rho + lap rho/4) u0)."""
    import pfinputs
    shape = (12, 10, 8 if lat.D == 3 else 1)
    prm = _prm(lat.Q, shape, (O.PERIODIC, O.WALL, O.PERIODIC), g=(0, -1e-5, 0))
    phi = pfinputs.smooth_random_field(shape, 5)
    u0 = 0.01 * np.stack([pfinputs.smooth_random_field(shape, s, lo=-1, hi=1)
                          for s in (6, 7, 8)])
    if lat.D == 2:
        u0[2] = 0
    P0 = 1e-3 * pfinputs.smooth_random_field(shape, 9)
    h, g = O.init(prm, phi, u0, P0)
    r = O.read(prm, h, g)
    assert np.allclose(r["phi"], phi, atol=1e-14)
    assert np.allclose(r["u"], u0, atol=1e-14)
    assert np.allclose(r["P"], P0, atol=1e-13)


@pytest.mark.parametrize("wet", [False, True], ids=["mirror", "contact-angles"])
@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_step_sites_matches_step(lat, wet):
    """The sampled-site evaluation agrees with the whole-array step (also with contact
    angles on the wall faces, whose ghost rule the two apply separately)."""
    import pfinputs
    shape = (7, 6, 5 if lat.D == 3 else 1)
    bc = (O.PERIODIC, O.WALL, O.WALL if lat.D == 3 else O.PERIODIC)
    kw = dict(wet_cos=(0, 0, 0.7, -0.4) + ((0.3, -0.9) if lat.D == 3 else (0, 0))) if wet else {}
    prm = _prm(lat.Q, shape, bc, g=(1e-4, -1e-4, 2e-4), **kw)
    h, g = _random(lat, shape, 41)
    h1, g1 = O.step(prm, h, g)
    sites = pfinputs.sample_sites(shape, 20, 3)
    hs, gs = O.step_sites(prm, h, g, sites)
    x, y, z = sites.T
    assert np.allclose(hs, h1[:, z, y, x], atol=1e-15, rtol=1e-13)
    assert np.allclose(gs, g1[:, z, y, x], atol=1e-13, rtol=1e-12)


def _collide_brute_force(q, c_list, prm, h, g, phi_nb):
    """One site's collision in 50-digit arithmetic, from the definitions, with the filter
    applied as the explicit Q x Q matrix of Section 2's footnote,
    A_il = w_i/(2T^2) [(c_i.c_l)^2 - T |c_l|^2], acting on g - g^eq (not through Pi).
    Weights from the speed classes: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36."""
    import mpmath as mp
    mp.mp.dps = 50
    f = mp.mpf
    Tm = f(1) / 3
    wc = {9: (f(4) / 9, f(1) / 9, f(1) / 36), 19: (f(1) / 3, f(1) / 18, f(1) / 36)}[q]
    cs = [tuple(int(v) for v in c) for c in c_list]
    w = [wc[sum(v * v for v in c)] for c in cs]
    opp = [cs.index(tuple(-v for v in c)) for c in cs]
    h = [f(float(v)) for v in h]
    g = [f(float(v)) for v in g]
    pn = [f(float(v)) for v in phi_nb]
    dot = lambda a, b: sum(x * y for x, y in zip(a, b))
    rho_L, rho_H = f(prm.rho_L), f(prm.rho_H)
    rdif = rho_H - rho_L
    tau_L = f(prm.nu_L) / Tm + f(1) / 2
    tau_H = f(prm.nu_H) / Tm + f(1) / 2
    M, W, sig, eps, C = f(prm.M), f(prm.W), f(prm.sigma), f(prm.eps), f(prm.dtheta_C)
    beta = f(1) if prm.hoc else f(0)
    gvec = [f(float(v)) for v in prm.g]
    phi = pn[0]
    grad = [sum(w[i] * cs[i][a] * (pn[i] - pn[opp[i]]) for i in range(q)) / (2 * Tm)
            for a in range(3)]
    lap = (2 / Tm) * sum(w[i] * (pn[i] - phi) for i in range(q))
    rho = rho_L + phi * rdif
    om = 1 / tau_L + phi * (1 / tau_H - 1 / tau_L)
    mu = (48 * sig / W) * phi * (phi - 1) * (phi - f(1) / 2) - (3 * sig * W / 2) * lap
    gn = mp.sqrt(dot(grad, grad))
    n = [x / (gn + eps) for x in grad]
    theta = (M / Tm) * (1 - 4 * (phi - f(1) / 2) ** 2) / W
    if C != 0 and abs(phi - f(1) / 2) > f(35) / 100 and (phi - f(1) / 2) * lap > 0:
        theta -= C * (M / Tm) * gn
    F = [rho * x for x in gvec]
    J = [sum(cs[i][a] * g[i] for i in range(q)) + (mu * grad[a] + F[a]) / 2 for a in range(3)]
    u = [x / (rho + beta * rdif * lap / 4) for x in J]
    P = Tm * sum(g) + (Tm * rdif / 2) * dot(u, grad)
    uu = dot(u, u)
    Gam = [w[i] * (1 + dot(cs[i], u) / Tm + dot(cs[i], u) ** 2 / (2 * Tm ** 2) - uu / (2 * Tm))
           for i in range(q)]
    heq = [phi * Gam[i] + theta * w[i] * dot(cs[i], n) for i in range(q)]
    om_phi = 1 / (M / Tm + f(1) / 2)
    hs = [h[i] - om_phi * (h[i] - heq[i]) for i in range(q)]
    K = []
    for i in range(q):
        cmu = [cs[i][a] - u[a] for a in range(3)]
        K.append(((Gam[i] - w[i]) * rdif + Gam[i] * mu / Tm) * dot(cmu, grad)
                 + Gam[i] * dot(cmu, F) / Tm)
    geq = [rho * Gam[i] + w[i] * (P / Tm - rho) - K[i] / 2
           + beta * w[i] * dot(cs[i], u) * rdif * lap / (4 * Tm) for i in range(q)]
    A = [[w[i] / (2 * Tm ** 2) * (dot(cs[i], cs[l]) ** 2 - Tm * dot(cs[l], cs[l]))
          for l in range(q)] for i in range(q)]
    neq = [g[l] - geq[l] for l in range(q)]
    gs = [geq[i] + K[i] + (1 - om) * sum(A[i][l] * neq[l] for l in range(q))
          for i in range(q)]
    return np.array([float(v) for v in hs]), np.array([float(v) for v in gs])


BRUTE_CASES = [  # (lattice, hoc, dtheta_C, phi at the site, neighbour spread)
    (9, 1, 0.0, 0.62, 0.2), (9, 0, 0.0, 0.37, 0.2), (19, 1, 0.0, 0.55, 0.2),
    (19, 1, 10.0, 0.93, 0.03),   # a dense dip: the Eq. 14 branch is taken
]


@pytest.mark.parametrize("q,hoc,C,phi0,spread", BRUTE_CASES)
def test_single_site_collision_brute_force(q, hoc, C, phi0, spread):
    """The oracle's FP64 collision of one site against the same step evaluated in 50-digit
    arithmetic with the filter as the explicit Q x Q matrix: agreement to FP64 rounding."""
    lat = D2Q9 if q == 9 else D3Q19
    rng = np.random.default_rng(q * 100 + int(10 * C) + hoc)
    gz = 3e-4 if q == 19 else 0.0
    prm = _prm(q, (1, 1, 1), rho_H=1000.0, nu_L=0.05, nu_H=0.01, M=0.1, W=4.0, sigma=1e-3,
               g=(1e-4, -2e-4, gz), eps=1e-10, hoc=hoc, dtheta_C=C)
    w = np.array([{0: 4 / 9, 1: 1 / 9, 2: 1 / 36}[int(c @ c)] if q == 9 else
                  {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(c @ c)] for c in lat.c])
    h = w * (phi0 + 0.05 * rng.standard_normal(q))
    g = w * (0.3 + 2.0 * rng.standard_normal(q))
    phi_nb = phi0 + spread * rng.uniform(0.1, 1.0, q) * (1.0 if C else rng.choice([-1, 1], q))
    phi_nb[0] = phi0
    hs, gs, m = O.collide(lat, prm, h[:, None], g[:, None], phi_nb[:, None])
    hb, gb = _collide_brute_force(q, lat.c, prm, h, g, phi_nb)
    if C:
        assert m["theta"][0] < (prm.M / T) * (1 - 4 * (phi0 - 0.5) ** 2) / prm.W   # taken
    assert np.abs(hs[:, 0] - hb).max() <= 1e-13 * np.abs(hb).max()
    assert np.abs(gs[:, 0] - gb).max() <= 1e-12 * np.abs(gb).max()
