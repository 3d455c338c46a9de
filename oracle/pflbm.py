"""FP64 reference of one time step of the phase-field lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function cites the
passage of the paper it follows.  Arrays of a field have shape (nz, ny, nx)
(D2Q9: nz = 1); a distribution set has shape (Q, nz, ny, nx).  The state at step n is
the pre-collision, post-streaming pair (h, g) on every site.

Readings of points the paper leaves open (each is also listed in the design notes):

* rho_L = rho_air, rho_H = rho_water, rho_dif = rho_H - rho_L > 0, phi = 1 is the
  heavy phase (Eq. 9 returns tau_water at phi = 1).
* tau = nu / T + 1/2 for both phases (the same relation as tau_phi = M/T + 1/2, Eq. 1).
* Filtered collision (Eqs. 10-12): G^eq_i = g^eq_i + K_i is the tau-independent part
  of the BGK update Eq. 5, and the non-equilibrium that is projected is g - g^eq, so
  Pi = sum_l c_l c_l (g_l - g^eq_l).  At tau_mix = 1 this equals the BGK update.
* High-order correction (Eq. 13): delta f^eq_i = w_i (c_i.u) lap(rho) / (4T) is added to
  g^eq with lap(rho) = rho_dif lap(phi); the "modified definition of velocity" is
  u = J / (rho + lap(rho)/4), the only choice for which the equilibrium carries the
  same first moment as g (momentum-conserving collision).
  With hoc = 0 both modifications are off (the model of Section 2 alone).
* The momentum reported is J = sum_i c_i g_i + (mu grad(phi) + F_ex)/2 (Section 2).
* External force F_ex = rho(phi) g (gravity as a body force on the local density).
* Dense-bubble correction (Eq. 14): the paper leaves C and F open.  Used here:
  F = -1 where |phi - 1/2| > 0.35 and (phi - 1/2) lap(phi) > 0, else 0; C is a
  parameter (default 0: correction off; 10 removes a seeded dense bubble and leaves a
  decent one, as Section 3 describes).  PARITY UNPINNED beyond C = 0, mass conservation
  and that behaviour.
* Boundaries: periodic axes wrap; wall axes use halfway bounce-back for both sets,
  and the ghost value of phi outside a wall equals the adjacent fluid site's value
  (zero normal gradient).
* Moving walls (not in the paper; the standard momentum correction of halfway
  bounce-back for a wall moving with velocity u_w, Ladd 1994): a population leaving x in
  direction i into a wall face returns as opp(i) at x reduced by 2 w_i (c_i . u_w)/T
  times phi(x) (set h) or rho(x) (set g), the site's pre-collision values.  u_w is the
  velocity of the face crossed; a population that crosses two or three wall faces at an
  edge or corner takes the mean of their velocities.  Face velocities are tangential.
* Open faces (the paper's "pressure condition" of the dam-break case names no
  mechanism; used here: the sites beyond an open face are copies of the boundary-layer
  sites they face, zero normal gradient of phi and u, with the pressure extrapolated
  linearly to the face's P_f): a population i entering x through the face comes from
  s' = x - c_i with its out-of-range coordinate put back into the layer, as f*_i(s'),
  plus 2 w_i (P_f - P(s'))/T for g.  A population that crosses a closed wall face as
  well is bounced back (with the mean velocity of the closed faces it crosses); one that
  crosses several open faces takes the mean of their P_f.
* Wetting (not in the paper, which has no contact angles; the usual geometric condition
  of diffuse-interface models): a wall face f may prescribe a contact angle theta_f,
  measured through the heavy phase, by n_w . grad(phi) = -(4/W) cos(theta_f) phi (1 - phi)
  with n_w the unit normal into the fluid; 4 phi (1 - phi)/W is |grad(phi)| of the
  equilibrium profile.  Taken across the half-way wall between the boundary site and
  its ghost one site out, the ghost value becomes phi_m + k phi_m (1 - phi_m) with phi_m
  the adjacent fluid site's value (the mirror above) and k the sum of
  (4/W) cos(theta_f) over the wall faces the ghost lies beyond (edges and corners add
  the faces they cross).  cos(theta_f) = 0 (90 degrees) is the zero-gradient rule.
* No clipping of phi anywhere; n = grad(phi)/(|grad(phi)| + eps) exactly as printed.
"""
import numpy as np

from .lattice import T, lattice as _lattice

PERIODIC = "periodic"
WALL = "wall"
# wall faces in the order of Params.wall_u: (axis, side)
FACES = ((0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1))


class Params:
    """Model parameters (Section 2; Section 4 lists the values per case).

    lattice: 9 or 19.  shape: (nx, ny, nz), nz = 1 for D2Q9.  bc: one entry per axis
    (x, y, z), PERIODIC or WALL (both faces of an axis alike).
    """

    def __init__(self, lattice, shape, bc, rho_L, rho_H, nu_L, nu_H, M, W, sigma,
                 g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1, dtheta_C=0.0, wall_u=None,
                 open_P=None, wet_cos=None):
        self.lat = _lattice(lattice)
        nx, ny, nz = shape
        if self.lat.D == 2 and nz != 1:
            raise ValueError("D2Q9 needs nz = 1")
        self.shape = (int(nx), int(ny), int(nz))
        self.bc = tuple(bc)
        if self.lat.D == 2:
            self.bc = (self.bc[0], self.bc[1], PERIODIC)
        self.rho_L = float(rho_L)
        self.rho_H = float(rho_H)
        self.nu_L = float(nu_L)
        self.nu_H = float(nu_H)
        self.M = float(M)
        self.W = float(W)
        self.sigma = float(sigma)
        self.g = np.asarray(g, dtype=np.float64).reshape(3)
        self.eps = float(eps)
        self.hoc = int(hoc)
        self.dtheta_C = float(dtheta_C)
        # velocity of each wall face, rows x-, x+, y-, y+, z-, z+ (see FACES)
        self.wall_u = (np.zeros((6, 3)) if wall_u is None
                       else np.asarray(wall_u, dtype=np.float64).reshape(6, 3))
        for f, (a, _) in enumerate(FACES):
            if self.wall_u[f, a] != 0.0:
                raise ValueError("a wall moves tangentially: normal velocity must be 0")
            if self.bc[a] != WALL and np.any(self.wall_u[f] != 0.0):
                raise ValueError("velocity given for a face of a periodic axis")
        # open faces: pressure P given per face (None or NaN: a closed wall)
        self.open_P = (np.full(6, np.nan) if open_P is None
                       else np.asarray(open_P, dtype=np.float64).reshape(6).copy())
        for f, (a, _) in enumerate(FACES):
            if np.isnan(self.open_P[f]):
                continue
            if self.bc[a] != WALL:
                raise ValueError("an open face must be on a wall axis")
            if np.any(self.wall_u[f] != 0.0):
                raise ValueError("an open face has no wall velocity")
            if not np.isfinite(self.open_P[f]):
                raise ValueError("open-face pressure must be finite")

        # wetting: cos(contact angle) per wall face (0: 90 degrees, the mirror ghost)
        self.wet_cos = (np.zeros(6) if wet_cos is None
                        else np.asarray(wet_cos, dtype=np.float64).reshape(6).copy())
        for f, (a, _) in enumerate(FACES):
            if not np.isfinite(self.wet_cos[f]) or abs(self.wet_cos[f]) > 1.0:
                raise ValueError("wet_cos must be finite and in [-1, 1]")
            if self.wet_cos[f] != 0.0 and self.bc[a] != WALL:
                raise ValueError("a contact angle given for a face of a periodic axis")
            if self.wet_cos[f] != 0.0 and not np.isnan(self.open_P[f]):
                raise ValueError("a contact angle given for an open face")

    @property
    def wet_k(self):
        """(4/W) cos(theta_f) per face: the ghost's phi_m (1 - phi_m) coefficient."""
        return 4.0 * self.wet_cos / self.W

    @property
    def open_faces(self):
        return [f for f in range(6) if not np.isnan(self.open_P[f])]

    # Eq. 1: relaxation time of h is M/T + 0.5
    @property
    def tau_phi(self):
        return self.M / T + 0.5

    # Eq. 9 and its text: tau of each phase from its kinematic viscosity, nu = T (tau - 1/2)
    @property
    def tau_L(self):
        return self.nu_L / T + 0.5

    @property
    def tau_H(self):
        return self.nu_H / T + 0.5

    # text after Eq. 7: rho_dif, difference of the two characteristic densities
    @property
    def rho_dif(self):
        return self.rho_H - self.rho_L

    @classmethod
    def from_dict(cls, d):
        keys = ("lattice", "shape", "bc", "rho_L", "rho_H", "nu_L", "nu_H", "M", "W",
                "sigma", "g", "eps", "hoc", "dtheta_C", "wall_u", "open_P", "wet_cos")
        return cls(**{k: d[k] for k in keys if k in d})


# ---------------------------------------------------------------------------
# neighbour access with the boundary rules
# ---------------------------------------------------------------------------

def _ghost_pad(field, bc):
    """Pad a (nz, ny, nx) field by one site per side: wrap on periodic axes, copy the
    adjacent fluid site on wall axes."""
    out = field
    # numpy axes: 0 = z, 1 = y, 2 = x ; bc is ordered (x, y, z)
    for ax_np, ax_bc in ((0, 2), (1, 1), (2, 0)):
        pad = [(0, 0)] * 3
        pad[ax_np] = (1, 1)
        out = np.pad(out, pad, mode="wrap" if bc[ax_bc] == PERIODIC else "edge")
    return out


def _wet_pad(p, wet_k):
    """Apply the wetting ghost rule to a ghost-padded phi field: each ghost beyond wall
    faces f gets phi_m + (sum_f k_f) phi_m (1 - phi_m), phi_m its mirrored value."""
    if wet_k is None or not np.any(wet_k != 0.0):
        return p
    k = np.zeros_like(p)
    # face f = (axis, side); numpy axis of bc axis a is 2 - a
    for f, (a, side) in enumerate(FACES):
        if wet_k[f] != 0.0:
            sl = [slice(None)] * 3
            sl[2 - a] = 0 if side < 0 else -1
            k[tuple(sl)] += wet_k[f]
    return p + k * p * (1.0 - p)


def neighbour(field, c, bc, wet_k=None):
    """field(x + c) for every site x, with the ghost rules at walls."""
    p = _wet_pad(_ghost_pad(field, bc), wet_k)
    nz, ny, nx = field.shape
    cx, cy, cz = (int(v) for v in c)
    return p[1 + cz:1 + cz + nz, 1 + cy:1 + cy + ny, 1 + cx:1 + cx + nx]


def phi_stencil(phi, lat, bc, wet_k=None):
    """phi at x + c_k for k = 0..Q-1 (index 0 is phi itself); wet_k: the wetting
    coefficients per wall face (None: the mirror ghost)."""
    return np.stack([neighbour(phi, lat.c[k], bc, wet_k) for k in range(lat.Q)])


# ---------------------------------------------------------------------------
# Section 2, central differences (the unnumbered display after the momentum text)
# ---------------------------------------------------------------------------

def grad_cd(lat, phi_nb):
    """grad(phi) = sum_i {phi(x + c_i) - phi(x - c_i)} c_i w_i / (2T), summed over all i.

    phi(x - c_i) is phi(x + c_opp(i))."""
    grad = np.zeros((3,) + phi_nb.shape[1:])
    for i in range(lat.Q):
        diff = phi_nb[i] - phi_nb[lat.opp[i]]
        for a in range(3):
            grad[a] += diff * lat.c[i, a] * lat.w[i]
    return grad / (2.0 * T)


def lap_cd(lat, phi_nb):
    """lap(phi) = 2 sum_i {phi(x + c_i) - phi(x)} w_i / T."""
    acc = np.zeros(phi_nb.shape[1:])
    for i in range(lat.Q):
        acc += (phi_nb[i] - phi_nb[0]) * lat.w[i]
    return 2.0 * acc / T


# ---------------------------------------------------------------------------
# Section 2, equilibria and forcing
# ---------------------------------------------------------------------------

def gamma(lat, u):
    """Eq. 3: Gamma_i = w_i {1 + c_i.u/T + (c_i.u)^2/(2T^2) - u^2/(2T)}.  u: (3, ...)."""
    u2 = (u * u).sum(0)
    out = []
    for i in range(lat.Q):
        cu = sum(lat.c[i, a] * u[a] for a in range(3))
        out.append(lat.w[i] * (1.0 + cu / T + cu * cu / (2.0 * T * T) - u2 / (2.0 * T)))
    return np.stack(out)


def theta_of(prm, phi, grad, lap):
    """Eq. 4: theta = (M/T)(1 - 4(phi - 1/2)^2)/W, plus the Eq. 14 correction
    delta theta = C (M/T) F(phi, lap) |grad phi| (F as read in the module docstring)."""
    theta = (prm.M / T) * (1.0 - 4.0 * (phi - 0.5) ** 2) / prm.W
    if prm.dtheta_C != 0.0:
        gnorm = np.sqrt((grad * grad).sum(0))
        F = np.where((np.abs(phi - 0.5) > 0.35) & ((phi - 0.5) * lap > 0.0), -1.0, 0.0)
        theta = theta + prm.dtheta_C * (prm.M / T) * F * gnorm
    return theta


def normal_of(prm, grad):
    """Text after Eq. 4: n = grad(phi) / (|grad(phi)| + eps)."""
    gnorm = np.sqrt((grad * grad).sum(0))
    return grad / (gnorm + prm.eps)


def mu_chm(prm, phi, lap):
    """Eq. 8: mu = (48 sigma / W) phi (phi - 1)(phi - 1/2) - (3 sigma W / 2) lap(phi)."""
    return (48.0 * prm.sigma / prm.W) * phi * (phi - 1.0) * (phi - 0.5) \
        - 1.5 * prm.sigma * prm.W * lap


def h_eq(lat, phi, Gam, theta, n):
    """Eq. 2: h^eq_i = phi Gamma_i + theta w_i (c_i . n)."""
    out = []
    for i in range(lat.Q):
        cn = sum(lat.c[i, a] * n[a] for a in range(3))
        out.append(phi * Gam[i] + theta * lat.w[i] * cn)
    return np.stack(out)


def forcing_K(lat, prm, Gam, u, grad, mu, F):
    """Eq. 7: K_i = {(Gamma_i - w_i) rho_dif + Gamma_i mu / T} (c_i - u).grad(phi)
                  + Gamma_i (c_i - u).F_ex / T."""
    out = []
    for i in range(lat.Q):
        cmu_grad = sum((lat.c[i, a] - u[a]) * grad[a] for a in range(3))
        cmu_F = sum((lat.c[i, a] - u[a]) * F[a] for a in range(3))
        out.append(((Gam[i] - lat.w[i]) * prm.rho_dif + Gam[i] * mu / T) * cmu_grad
                   + Gam[i] * cmu_F / T)
    return np.stack(out)


def g_eq(lat, prm, rho, P, Gam, K, u, lap):
    """Eq. 6: g^eq_i = rho Gamma_i + w_i (P/T - rho) - K_i/2, plus (hoc on) the Eq. 13
    correction delta f^eq_i = w_i (c_i.u) lap(rho) / (4T), lap(rho) = rho_dif lap(phi)."""
    out = []
    for i in range(lat.Q):
        val = rho * Gam[i] + lat.w[i] * (P / T - rho) - K[i] / 2.0
        if prm.hoc:
            cu = sum(lat.c[i, a] * u[a] for a in range(3))
            val = val + lat.w[i] * cu * (prm.rho_dif * lap) / (4.0 * T)
        out.append(val)
    return np.stack(out)


def hermite_filter(lat, neq):
    """Eqs. 11-12: Pi = sum_l c_l c_l neq_l and Phi_i : Pi with
    Phi_i = w_i/(2T^2) (c_i c_i - T I).  Returns (Phi_i : Pi for all i, Pi)."""
    Pi = np.zeros((3, 3) + neq.shape[1:])
    for l in range(lat.Q):
        for a in range(3):
            for b in range(3):
                if lat.c[l, a] * lat.c[l, b] != 0:
                    Pi[a, b] += lat.c[l, a] * lat.c[l, b] * neq[l]
    trace = Pi[0, 0] + Pi[1, 1] + Pi[2, 2]
    out = []
    for i in range(lat.Q):
        cc_Pi = sum(lat.c[i, a] * lat.c[i, b] * Pi[a, b]
                    for a in range(3) for b in range(3))
        out.append(lat.w[i] / (2.0 * T * T) * (cc_Pi - T * trace))
    return np.stack(out), Pi


# ---------------------------------------------------------------------------
# macroscopic quantities and the collision of a set of sites
# ---------------------------------------------------------------------------

def macros(lat, prm, h, g, phi_nb):
    """Quantities of the pre-collision state at a set of sites.

    phi (text after Eq. 4), grad/lap (central differences), rho = rho_L + phi rho_dif,
    1/tau_mix (Eq. 9), mu (Eq. 8), n and theta (Eq. 4, Eq. 14), F_ex = rho g,
    J = sum c_i g_i + (mu grad + F)/2 (end of Section 2), u = J/(rho + lap(rho)/4)
    (Eq. 13's modified velocity; u = J/rho with hoc off), P = T sum g_i +
    (T rho_dif/2) u.grad (end of Section 2)."""
    phi = phi_nb[0]
    grad = grad_cd(lat, phi_nb)
    lap = lap_cd(lat, phi_nb)
    rho = prm.rho_L + phi * prm.rho_dif
    inv_tau = 1.0 / prm.tau_L + phi * (1.0 / prm.tau_H - 1.0 / prm.tau_L)
    mu = mu_chm(prm, phi, lap)
    n = normal_of(prm, grad)
    theta = theta_of(prm, phi, grad, lap)
    F = prm.g.reshape((3,) + (1,) * phi.ndim) * rho
    J = np.zeros((3,) + phi.shape)
    for i in range(lat.Q):
        for a in range(3):
            if lat.c[i, a] != 0:
                J[a] += lat.c[i, a] * g[i]
    J = J + (mu * grad + F) / 2.0
    rho_p = rho + (prm.rho_dif * lap / 4.0 if prm.hoc else 0.0)
    u = J / rho_p
    P = T * g.sum(0) + (T * prm.rho_dif / 2.0) * (u * grad).sum(0)
    return dict(phi=phi, grad=grad, lap=lap, rho=rho, inv_tau=inv_tau, mu=mu, n=n,
                theta=theta, F=F, J=J, u=u, P=P)


def collide(lat, prm, h, g, phi_nb):
    """Post-collision populations (h*, g*) at a set of sites.

    h: BGK of Eq. 1 with the equilibrium of Eqs. 2-4.
    g: filtered collision of Eq. 10, g* = G^eq + (1 - 1/tau_mix) Phi : Pi with
       G^eq = g^eq + K and Pi built from g - g^eq (Eqs. 5-7, 11-13)."""
    m = macros(lat, prm, h, g, phi_nb)
    Gam = gamma(lat, m["u"])
    heq = h_eq(lat, m["phi"], Gam, m["theta"], m["n"])
    hstar = h - (h - heq) / prm.tau_phi
    K = forcing_K(lat, prm, Gam, m["u"], m["grad"], m["mu"], m["F"])
    geq = g_eq(lat, prm, m["rho"], m["P"], Gam, K, m["u"], m["lap"])
    proj, _ = hermite_filter(lat, g - geq)
    gstar = geq + K + (1.0 - m["inv_tau"]) * proj
    return hstar, gstar, m


# ---------------------------------------------------------------------------
# streaming with boundaries (Eqs. 1, 5, 10: populations move from x to x + c_i)
# ---------------------------------------------------------------------------

def _source_solid(c, shape, bc):
    """Mask of sites x whose upstream site x - c lies outside a wall face."""
    nx, ny, nz = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), dtype=bool)
    for coord, n, cc, b in ((xx, nx, c[0], bc[0]), (yy, ny, c[1], bc[1]),
                            (zz, nz, c[2], bc[2])):
        if b == WALL:
            src = coord - cc
            solid |= (src < 0) | (src >= n)
    return solid


def _crossed(prm, k, xyz):
    """(N, 6) mask of the faces (FACES order) a population leaving the sites xyz (N, 3
    integer (x, y, z)) in direction k crosses."""
    c = prm.lat.c[k]
    out = np.zeros((len(xyz), 6), dtype=bool)
    for f, (a, side) in enumerate(FACES):
        if prm.bc[a] != WALL or c[a] != side:
            continue
        dest = xyz[:, a] + c[a]
        out[:, f] = (dest < 0) | (dest >= prm.shape[a])
    return out


def wall_cu(prm, k, xyz):
    """c_k . u_w for populations leaving the sites xyz (N, 3 integer (x, y, z)) in
    direction k: u_w is the velocity of the closed wall face the population crosses, the
    mean of the crossed closed faces' velocities at an edge or corner, 0 where it crosses
    none."""
    c = prm.lat.c[k]
    closed = _crossed(prm, k, xyz)
    closed[:, prm.open_faces] = False
    s = (closed * (prm.wall_u @ c)[None, :]).sum(1)
    n = closed.sum(1)
    return np.where(n > 0, s / np.maximum(n, 1), 0.0)


def open_return(prm, i, xyz, m, which, fstar):
    """Populations i arriving at the sites xyz from beyond open faces: (mask of those
    whose source x - c_i crosses open faces only, their values).  The site beyond an
    open face is a copy of the site of the boundary layer it faces (zero normal gradient
    of phi and u) with the pressure extrapolated linearly to P_f at the face: the source
    x - c_i, its out-of-range coordinates put back into the layer, is the site s' that
    population i comes from, with value f*_i(s') and, for g, plus 2 w_i (P_f - P(s'))/T
    (the filtered collision depends on P only through w_i P/T).  m: the sites'
    macroscopic quantities (P), flattened; fstar: post-collision populations, flattened
    per direction."""
    lat = prm.lat
    k = lat.opp[i]
    cr = _crossed(prm, k, xyz)
    is_open = np.zeros(6, dtype=bool)
    is_open[prm.open_faces] = True
    only_open = cr.any(1) & ~(cr & ~is_open[None, :]).any(1)
    nx, ny, nz = prm.shape
    src = xyz - lat.c[i][None, :]
    for a, n in enumerate((nx, ny, nz)):
        if prm.bc[a] == WALL:
            src[:, a] = np.clip(src[:, a], 0, n - 1)
        else:
            src[:, a] %= n
    lin = (src[:, 2] * ny + src[:, 1]) * nx + src[:, 0]
    val = fstar[i][lin]
    if which == "g":
        Pf = np.where(is_open, np.nan_to_num(prm.open_P), 0.0)
        P = (cr * Pf[None, :]).sum(1) / np.maximum(cr.sum(1), 1)
        val = val + 2.0 * lat.w[i] * (P - m["P"][lin]) / T
    return only_open, val


def _all_sites(shape):
    nx, ny, nz = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def stream(lat, prm, fstar, m=None, which="h"):
    """f_i(x, n+1) = f*_i(x - c_i, n); where x - c_i is outside a wall the population
    comes back from x itself: f_i(x, n+1) = f*_opp(i)(x, n) (halfway bounce-back), less
    2 w (c_opp(i) . u_w)/T times phi(x) (which = "h") or rho(x) ("g") for a moving wall,
    or by anti-bounce-back through an open face (open_return).  m: the pre-collision
    macroscopic quantities of the step (needed for moving walls and open faces)."""
    out = np.empty_like(fstar)
    moving = m is not None and np.any(prm.wall_u != 0.0)
    opens = m is not None and len(prm.open_faces) > 0
    xyz = _all_sites(prm.shape) if (moving or opens) else None
    if opens:
        mf = {"P": m["P"].ravel()}
    for i in range(lat.Q):
        c = lat.c[i]
        pulled = np.roll(fstar[i], shift=(int(c[2]), int(c[1]), int(c[0])), axis=(0, 1, 2))
        j = lat.opp[i]
        back = fstar[j]
        if moving:
            cu = wall_cu(prm, j, xyz).reshape(back.shape)
            scale = m["phi"] if which == "h" else m["rho"]
            back = back - (2.0 / T) * lat.w[j] * cu * scale
        if opens:
            only_open, val = open_return(prm, i, xyz, mf, which,
                                         fstar.reshape(lat.Q, -1))
            back = np.where(only_open.reshape(back.shape), val.reshape(back.shape), back)
        out[i] = np.where(_source_solid(c, prm.shape, prm.bc), back, pulled)
    return out


# ---------------------------------------------------------------------------
# whole-domain operations
# ---------------------------------------------------------------------------

def step(prm, h, g):
    """One time step of both sets: (h, g) at step n -> (h, g) at step n + 1."""
    lat = prm.lat
    phi = h.sum(0)
    phi_nb = phi_stencil(phi, lat, prm.bc, prm.wet_k)
    hstar, gstar, m = collide(lat, prm, h, g, phi_nb)
    return stream(lat, prm, hstar, m, "h"), stream(lat, prm, gstar, m, "g")


def run(prm, h, g, nsteps):
    for _ in range(nsteps):
        h, g = step(prm, h, g)
    return h, g


def read(prm, h, g):
    """phi, P, J (= rho u as printed) and u of the state at step n."""
    lat = prm.lat
    phi = h.sum(0)
    m = macros(lat, prm, h, g, phi_stencil(phi, lat, prm.bc, prm.wet_k))
    return dict(phi=m["phi"], P=m["P"], J=m["J"], u=m["u"])


def mass(h):
    """sum_x phi(x), phi = sum_i h_i."""
    return float(h.sum())


def init(prm, phi0, u0, P0=None):
    """Equilibrium start from (phi0, u0, P0): h = h^eq, g = g^eq evaluated with u = u0
    and P = P0 (the paper does not state its initialisation).  Reading the state back
    with read() returns u0 and P0."""
    lat = prm.lat
    phi0 = np.asarray(phi0, dtype=np.float64)
    u0 = np.asarray(u0, dtype=np.float64)
    P0 = np.zeros_like(phi0) if P0 is None else np.asarray(P0, dtype=np.float64)
    phi_nb = phi_stencil(phi0, lat, prm.bc, prm.wet_k)
    grad = grad_cd(lat, phi_nb)
    lap = lap_cd(lat, phi_nb)
    rho = prm.rho_L + phi0 * prm.rho_dif
    mu = mu_chm(prm, phi0, lap)
    n = normal_of(prm, grad)
    theta = theta_of(prm, phi0, grad, lap)
    F = prm.g.reshape(3, 1, 1, 1) * rho
    Gam = gamma(lat, u0)
    h = h_eq(lat, phi0, Gam, theta, n)
    K = forcing_K(lat, prm, Gam, u0, grad, mu, F)
    g = g_eq(lat, prm, rho, P0, Gam, K, u0, lap)
    return h, g


# ---------------------------------------------------------------------------
# one step evaluated only at sampled output sites (for full-size domains)
# ---------------------------------------------------------------------------

def _map_axis(v, n, b):
    """Site index of coordinate v on an axis: wrap (periodic) or mirror-to-edge (wall)."""
    if b == PERIODIC:
        return v % n
    return np.clip(v, 0, n - 1)


def step_sites(prm, h, g, sites):
    """(h, g) at step n + 1 at the given sites, from the full state at step n.

    sites: integer array (S, 3) of (x, y, z).  Computes the same step as step(), but
    only the collisions of the upstream sites the outputs need."""
    lat = prm.lat
    nx, ny, nz = prm.shape
    sites = np.asarray(sites, dtype=np.int64).reshape(-1, 3)
    S = len(sites)
    # upstream site and population for every (output site, direction)
    src = np.empty((S, lat.Q, 3), dtype=np.int64)
    pop = np.empty((S, lat.Q), dtype=np.int64)
    for i in range(lat.Q):
        up = sites - lat.c[i][None, :]
        solid = np.zeros(S, dtype=bool)
        for a, (n, b) in enumerate(zip((nx, ny, nz), prm.bc)):
            if b == WALL:
                solid |= (up[:, a] < 0) | (up[:, a] >= n)
            else:
                up[:, a] %= n
        src[:, i] = np.where(solid[:, None], sites, up)
        pop[:, i] = np.where(solid, lat.opp[i], i)
    ups = src.reshape(-1, 3)
    # pre-collision populations and phi stencil of each upstream site
    hf = h.reshape(lat.Q, -1)
    gf = g.reshape(lat.Q, -1)

    def lin(x, y, z):
        return (z * ny + y) * nx + x

    idx = lin(ups[:, 0], ups[:, 1], ups[:, 2])
    hu = hf[:, idx].astype(np.float64)
    gu = gf[:, idx].astype(np.float64)
    phi_nb = np.empty((lat.Q, len(ups)))
    wk = prm.wet_k
    for k in range(lat.Q):
        raw = ups + lat.c[k][None, :]
        x = _map_axis(raw[:, 0], nx, prm.bc[0])
        y = _map_axis(raw[:, 1], ny, prm.bc[1])
        z = _map_axis(raw[:, 2], nz, prm.bc[2])
        pm = hf[:, lin(x, y, z)].astype(np.float64).sum(0)
        # wetting ghost rule for the neighbours beyond wall faces
        kk = np.zeros(len(ups))
        for f, (a, side) in enumerate(FACES):
            if wk[f] != 0.0:
                n_a = prm.shape[a]
                kk += np.where(raw[:, a] < 0 if side < 0 else raw[:, a] >= n_a, wk[f], 0.0)
        phi_nb[k] = pm + kk * pm * (1.0 - pm) if np.any(wk != 0.0) else pm
    hstar, gstar, m = collide(lat, prm, hu, gu, phi_nb)
    hstar = hstar.reshape(lat.Q, S, lat.Q)
    gstar = gstar.reshape(lat.Q, S, lat.Q)
    rows = np.arange(S)
    h_out = np.empty((lat.Q, S))
    g_out = np.empty((lat.Q, S))
    moving = np.any(prm.wall_u != 0.0)
    if prm.open_faces:
        raise NotImplementedError("sampled-site steps with open faces")
    for i in range(lat.Q):
        h_out[i] = hstar[pop[:, i], rows, i]
        g_out[i] = gstar[pop[:, i], rows, i]
        if moving:
            # bounced entries (pop = opp(i)) come from the output site itself
            j = lat.opp[i]
            bounced = pop[:, i] == j if i != 0 else np.zeros(S, dtype=bool)
            cu = np.where(bounced, wall_cu(prm, j, sites), 0.0)
            k = (2.0 / T) * lat.w[j] * cu
            h_out[i] -= k * m["phi"].reshape(S, lat.Q)[:, i]
            g_out[i] -= k * m["rho"].reshape(S, lat.Q)[:, i]
    return h_out, g_out
