"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload definitions (parameter sets, grid sizes, boundary kinds)
and field generators (phase profiles, velocity fields, random distribution states).
It contains none of the lattice Boltzmann method's arithmetic: it only produces the
numbers both the CPU reference and the GPU library are fed.  Every array it returns
is float32 (rounded once from float64), so both sides start from identical values.

Workloads (lattice units, rho_L = 1):
  static_droplet   D2Q9 64x64 periodic, R=16, W=4, rho_H=1000, M=0.1, sigma=1e-3,
                   nu_H=nu_L=0.01 (the paper's static-droplet case, Section 4.1, with
                   the density ratio of 1000 used throughout).
  rayleigh_taylor  D2Q9 256x1024, x periodic, y walls, Atwood 0.5 (rho_H=3), g=1e-5,
                   W=5, Re=UL/nu_H=3000 with U=sqrt(gL), mu_H=mu_L, Pe=UL/M=1000,
                   Ca=rho_H U nu_H/sigma=0.26, interface y0 = 511.5 + 0.1 L cos(2 pi x/L)
                   (Section 4.3's rho_ratio = 3 case, rescaled to L = 256).
  rising_bubble    D3Q19 128^3, x,y periodic, z walls, rho_H=1000, mu_H/mu_L=100,
                   nu_H=0.01, R=16, W=4, M=0.1, g=1e-5, Eotvos g drho (2R)^2/sigma = 10.
  droplet_impact   D3Q19 256x256x128, x,y periodic, z walls, rho_H=1000, R=32, film
                   depth 16, impact velocity 0.05, Re=UD/nu_H=500, We=rho_H U^2 D/sigma
                   =8000, mu_H/mu_L=100, W=4, M=0.1, g=0.
  drops            D2Q9 256x256 periodic, the surrogate's training and test family:
                   per seed 2-8 droplets, R ~ U[8, 32], rho_H ~ logU[10, 1000], centres
                   uniform on the torus at least W apart (edge to edge), each drop moving
                   with a random velocity |u| <= 0.02; nu_H = nu_L = 0.01, M = 0.1, W = 4,
                   sigma = 1e-2.  Seeds: train 0-255, validation 1000-1031, test 2000-2031.
  sessile_drop     D2Q9 96x40, x periodic, y walls, a half disc R = 12 on the bottom
                   wall, which prescribes a contact angle (rho_H = 10, nu = 0.1, M = 0.1,
                   W = 4, sigma = 0.05): the wetting check (not a case of the paper);
                   D3Q19 variant nx x nx x nz with a half ball on the z- wall.
  dam_break        D3Q19 537x50x198 (Section 4.4's 537x198x50 with its height along z),
                   no-slip walls, open top at P = 0, water column H = 100 by L = 200 (2 H;
                   the text gives no length) against the x- wall, rho_H = 1000, g = 4e-6,
                   W = 4, M = 0.02, nu_air = 8.3e-3, nu_water = 4.9e-6, sigma = 5.2e-3;
                   hydrostatic start, P = 0 in the top layer.
  dense_bubble     D2Q9 80x40 periodic water (phi = 1) holding a dense bubble (a shallow
                   Gaussian dip, phi 0.93 at its centre, standard deviation 3 sites) and
                   a decent bubble (phi = 0 inside, R = 10) 40 sites apart; rho_H = 1000,
                   nu_H = nu_L = 0.1, W = 3, M = 0.17 (Section 3's dense-bubble values of W
                   and M), sigma = 1e-3, u = 0, P = 0; dtheta_C as given.
"""
import math

import numpy as np

PERIODIC = "periodic"
WALL = "wall"


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


# ---------------------------------------------------------------------------
# parameter sets
# ---------------------------------------------------------------------------

def static_droplet(n=64, R=16.0, W=4.0, rho_H=1000.0, sigma=1e-3, nu=0.01, M=0.1):
    return dict(name="static_droplet", lattice=9, shape=(n, n, 1),
                bc=(PERIODIC, PERIODIC, PERIODIC), rho_L=1.0, rho_H=rho_H, nu_L=nu,
                nu_H=nu, M=M, W=W, sigma=sigma, g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1,
                dtheta_C=0.0, R=R, steps=1000)


def dense_bubble(nx=80, ny=40, C=10.0, depth=0.07, spread=3.0, R=10.0):
    return dict(name="dense_bubble", lattice=9, shape=(nx, ny, 1),
                bc=(PERIODIC, PERIODIC, PERIODIC), rho_L=1.0, rho_H=1000.0, nu_L=0.1,
                nu_H=0.1, M=0.17, W=3.0, sigma=1e-3, g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1,
                dtheta_C=C, depth=depth, spread=spread, R=R,
                dense_at=(nx / 4.0, (ny - 1) / 2.0), decent_at=(3.0 * nx / 4.0, (ny - 1) / 2.0))


def sessile_drop(theta_deg, nx=96, ny=40, R=12.0, lattice=9, nz=32):
    """Cap on the bottom wall whose bottom wall prescribes the contact angle theta_deg;
    it starts as a half disc (90 degrees).  D2Q9: nx x ny, x periodic, y walls; D3Q19:
    nx x nx x nz, x and y periodic, z walls (a hemisphere)."""
    c = math.cos(math.radians(theta_deg))
    if lattice == 9:
        shape, bc, wet = (nx, ny, 1), (PERIODIC, WALL, PERIODIC), (0.0, 0.0, c, 0.0, 0.0, 0.0)
    else:
        shape, bc, wet = (nx, nx, nz), (PERIODIC, PERIODIC, WALL), (0.0, 0.0, 0.0, 0.0, c, 0.0)
    return dict(name="sessile_drop", lattice=lattice, shape=shape, bc=bc, rho_L=1.0,
                rho_H=10.0, nu_L=0.1, nu_H=0.1, M=0.1, W=4.0, sigma=0.05, g=(0.0, 0.0, 0.0),
                eps=1e-10, hoc=1, dtheta_C=0.0, wet_cos=wet, theta_deg=theta_deg, R=R)


def rayleigh_taylor(nx=256, ny=1024):
    g = 1e-5
    U = math.sqrt(g * nx)
    rho_H = 3.0
    nu_H = U * nx / 3000.0
    nu_L = nu_H * rho_H          # mu_H = mu_L
    M = U * nx / 1000.0
    sigma = rho_H * U * nu_H / 0.26
    return dict(name="rayleigh_taylor", lattice=9, shape=(nx, ny, 1),
                bc=(PERIODIC, WALL, PERIODIC), rho_L=1.0, rho_H=rho_H, nu_L=nu_L,
                nu_H=nu_H, M=M, W=5.0, sigma=sigma, g=(0.0, -g, 0.0), eps=1e-10,
                hoc=1, dtheta_C=0.0, amp=0.1 * nx, steps=20000)


def rising_bubble(n=128, R=16.0):
    rho_H, rho_L, g = 1000.0, 1.0, 1e-5
    sigma = g * (rho_H - rho_L) * (2 * R) ** 2 / 10.0
    return dict(name="rising_bubble", lattice=19, shape=(n, n, n),
                bc=(PERIODIC, PERIODIC, WALL), rho_L=rho_L, rho_H=rho_H, nu_L=0.1,
                nu_H=0.01, M=0.1, W=4.0, sigma=sigma, g=(0.0, 0.0, -g), eps=1e-10,
                hoc=1, dtheta_C=0.0, R=R, steps=10000)


def droplet_impact(nx=256, ny=256, nz=128, R=32.0, film=16.0, U=0.05):
    rho_H = 1000.0
    D = 2 * R
    nu_H = U * D / 500.0
    sigma = rho_H * U * U * D / 8000.0
    return dict(name="droplet_impact", lattice=19, shape=(nx, ny, nz),
                bc=(PERIODIC, PERIODIC, WALL), rho_L=1.0, rho_H=rho_H, nu_L=10.0 * nu_H,
                nu_H=nu_H, M=0.1, W=4.0, sigma=sigma, g=(0.0, 0.0, 0.0), eps=1e-10,
                hoc=1, dtheta_C=0.0, R=R, film=film, U=U, steps=5000)


def dam_break(nx=537, ny=50, nz=198, H=100.0, L=200.0, g=4e-6):
    """Section 4.4's dam break with the height along z: the paper's 537 x 198 x 50 box
    (length, height, span) as nx x nz x ny here, since only z faces may be open.  No-slip
    walls, an open top at P = 0, a water column of height H and length L (L is not in
    the text; 2 H here) against the x- wall."""
    nan = float("nan")
    return dict(name="dam_break", lattice=19, shape=(nx, ny, nz),
                bc=(WALL, WALL, WALL), rho_L=1.0, rho_H=1000.0, nu_L=8.3e-3,
                nu_H=4.9e-6, M=0.02, W=4.0, sigma=5.2e-3, g=(0.0, 0.0, -g), eps=1e-10,
                hoc=1, dtheta_C=0.0, open_P=[nan, nan, nan, nan, nan, 0.0], H=H, L=L,
                steps=20000)


def drops(seed, n=256):
    """Parameters and droplet layout of one seed of the surrogate family (see above);
    numpy's PCG64 generator seeded with `seed` draws every random number."""
    rng = np.random.default_rng(int(seed))
    rho_H = float(10.0 ** rng.uniform(1.0, 3.0))
    W = 4.0
    n_drop = int(rng.integers(2, 9))
    placed = []
    tries = 0
    while len(placed) < n_drop and tries < 2000:
        tries += 1
        R = float(rng.uniform(8.0, 32.0))
        c = rng.uniform(0.0, n, size=2)
        ok = True
        for (c2, R2, _) in placed:
            d = np.abs(c - c2)
            d = np.minimum(d, n - d)
            if math.hypot(d[0], d[1]) < R + R2 + W:
                ok = False
                break
        if ok:
            ang = rng.uniform(0.0, 2.0 * math.pi)
            speed = rng.uniform(0.0, 0.02)
            placed.append((c, R, (speed * math.cos(ang), speed * math.sin(ang))))
    return dict(name="drops", lattice=9, shape=(n, n, 1),
                bc=(PERIODIC, PERIODIC, PERIODIC), rho_L=1.0, rho_H=rho_H, nu_L=0.01,
                nu_H=0.01, M=0.1, W=W, sigma=1e-2, g=(0.0, 0.0, 0.0), eps=1e-10, hoc=1,
                dtheta_C=0.0, seed=int(seed),
                drops=[(float(c[0]), float(c[1]), R, v[0], v[1]) for c, R, v in placed])


def model_params(cfg):
    """The subset of a workload dict both sides take as model parameters."""
    keys = ("lattice", "shape", "bc", "rho_L", "rho_H", "nu_L", "nu_H", "M", "W",
            "sigma", "g", "eps", "hoc", "dtheta_C")
    d = {k: cfg[k] for k in keys}
    if cfg.get("wall_u") is not None:       # wall face velocities, rows x-, x+, y-, y+, z-, z+
        d["wall_u"] = np.asarray(cfg["wall_u"], dtype=np.float64).reshape(6, 3)
    if cfg.get("open_P") is not None:       # open-face pressures, same order (NaN: closed)
        d["open_P"] = np.asarray(cfg["open_P"], dtype=np.float64).reshape(6)
    if cfg.get("wet_cos") is not None:      # cos(contact angle) per wall face, same order
        d["wet_cos"] = np.asarray(cfg["wet_cos"], dtype=np.float64).reshape(6)
    return d


# ---------------------------------------------------------------------------
# field generators; arrays have shape (nz, ny, nx), vectors (3, nz, ny, nx)
# ---------------------------------------------------------------------------

def _grid(shape):
    nx, ny, nz = shape
    return np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")


def drop_profile(shape, centre, R, W, inside=1.0):
    """1/2 - 1/2 tanh(2 (r - R)/W) (value `inside` at the centre, 1 - inside far away)."""
    z, y, x = _grid(shape)
    cx, cy, cz = centre
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + ((z - cz) ** 2 if shape[2] > 1 else 0.0))
    p = 0.5 - 0.5 * np.tanh(2.0 * (r - R) / W)
    return p if inside == 1.0 else 1.0 - p


def centre_of(shape):
    nx, ny, nz = shape
    return ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0 if nz > 1 else 0.0)


def hydrostatic_pressure(cfg, phi):
    """Pressure in hydrostatic balance with gravity, dP/ds = rho(phi) g along the gravity
    axis (trapezoidal sum from the first site, rho = rho_L + phi (rho_H - rho_L)), shifted
    to zero mean.  A start with P = 0 under gravity launches a pressure shock from the
    walls that nucleates spurious dense bubbles."""
    g = np.asarray(cfg["g"], dtype=np.float64)
    axis = int(np.argmax(np.abs(g)))
    if g[axis] == 0.0:
        return np.zeros_like(phi)
    rho = cfg["rho_L"] + phi * (cfg["rho_H"] - cfg["rho_L"])
    np_axis = {0: 2, 1: 1, 2: 0}[axis]            # field arrays are (z, y, x)
    f = rho * g[axis]
    P = np.cumsum(f, axis=np_axis) - 0.5 * f - 0.5 * np.take(f, [0], axis=np_axis)
    return P - P.mean()


def fields_static_droplet(cfg):
    phi = drop_profile(cfg["shape"], centre_of(cfg["shape"]), cfg["R"], cfg["W"])
    u = np.zeros((3,) + phi.shape)
    return _f32(phi), _f32(u), _f32(np.zeros_like(phi))


def fields_rayleigh_taylor(cfg):
    nx, ny, nz = cfg["shape"]
    z, y, x = _grid(cfg["shape"])
    y0 = (ny - 1) / 2.0 + cfg["amp"] * np.cos(2.0 * np.pi * x / nx)
    phi = 0.5 + 0.5 * np.tanh(2.0 * (y - y0) / cfg["W"])      # heavy fluid on top
    u = np.zeros((3,) + phi.shape)
    return _f32(phi), _f32(u), _f32(hydrostatic_pressure(cfg, phi))


def fields_rising_bubble(cfg):
    nx, ny, nz = cfg["shape"]
    centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, nz / 4.0)
    phi = drop_profile(cfg["shape"], centre, cfg["R"], cfg["W"], inside=0.0)
    u = np.zeros((3,) + phi.shape)
    return _f32(phi), _f32(u), _f32(hydrostatic_pressure(cfg, phi))


def fields_droplet_impact(cfg):
    nx, ny, nz = cfg["shape"]
    z, y, x = _grid(cfg["shape"])
    film = 0.5 - 0.5 * np.tanh(2.0 * (z - (cfg["film"] - 0.5)) / cfg["W"])
    zc = cfg["film"] + cfg["W"] + cfg["R"]
    drop = drop_profile(cfg["shape"], ((nx - 1) / 2.0, (ny - 1) / 2.0, zc), cfg["R"],
                        cfg["W"])
    phi = np.maximum(film, drop)
    u = np.zeros((3,) + phi.shape)
    u[2] = -cfg["U"] * drop
    return _f32(phi), _f32(u), _f32(np.zeros_like(phi))


def fields_drops(cfg):
    """phi = the largest of the periodic drop profiles; u = each drop's velocity
    weighted by its profile; P = 0."""
    nx, ny, _ = cfg["shape"]
    z, y, x = _grid(cfg["shape"])
    phi = np.zeros((1, ny, nx))
    u = np.zeros((3, 1, ny, nx))
    for cx, cy, R, vx, vy in cfg["drops"]:
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy)
        dy = np.minimum(dy, ny - dy)
        p = 0.5 - 0.5 * np.tanh(2.0 * (np.sqrt(dx * dx + dy * dy) - R) / cfg["W"])
        phi = np.maximum(phi, p)
        u[0] += p * vx
        u[1] += p * vy
    return _f32(phi), _f32(u), _f32(np.zeros_like(phi))


def fields_dense_bubble(cfg):
    """phi = min(1 - depth exp(-r1^2 / (2 spread^2)), tanh bubble of radius R at r2)."""
    z, y, x = _grid(cfg["shape"])
    (ax, ay), (bx, by) = cfg["dense_at"], cfg["decent_at"]
    r1 = np.sqrt((x - ax) ** 2 + (y - ay) ** 2)
    r2 = np.sqrt((x - bx) ** 2 + (y - by) ** 2)
    dense = 1.0 - cfg["depth"] * np.exp(-r1 ** 2 / (2.0 * cfg["spread"] ** 2))
    decent = 0.5 + 0.5 * np.tanh(2.0 * (r2 - cfg["R"]) / cfg["W"])
    phi = np.minimum(dense, decent)
    u = np.zeros((3,) + phi.shape)
    return _f32(phi), _f32(u), _f32(np.zeros_like(phi))


def fields_sessile_drop(cfg):
    """Half disc (D2Q9) or half ball (D3Q19) of radius R centred on the wall line
    y = -1/2 (resp. plane z = -1/2), phi = 1 inside."""
    z, y, x = _grid(cfg["shape"])
    nx, ny = cfg["shape"][0], cfg["shape"][1]
    if cfg["lattice"] == 9:
        r = np.sqrt((x - (nx - 1) / 2.0) ** 2 + (y + 0.5) ** 2)
    else:
        r = np.sqrt((x - (nx - 1) / 2.0) ** 2 + (y - (ny - 1) / 2.0) ** 2 + (z + 0.5) ** 2)
    phi = 0.5 - 0.5 * np.tanh(2.0 * (r - cfg["R"]) / cfg["W"])
    u = np.zeros((3,) + phi.shape)
    return _f32(phi), _f32(u), _f32(np.zeros_like(phi))


def fields_dam_break(cfg):
    """phi: the water column x < L, z < H (faces at L - 1/2 and H - 1/2) through the
    tanh profile of its signed distance (Euclidean round the top corner); u = 0; P in
    hydrostatic balance, 0 in the top layer."""
    z, y, x = _grid(cfg["shape"])
    dx = x - (cfg["L"] - 0.5)
    dz = z - (cfg["H"] - 0.5)
    out = np.sqrt(np.maximum(dx, 0.0) ** 2 + np.maximum(dz, 0.0) ** 2)
    d = np.where((dx > 0) | (dz > 0), out, np.maximum(dx, dz))
    phi = 0.5 - 0.5 * np.tanh(2.0 * d / cfg["W"])
    u = np.zeros((3,) + phi.shape)
    P = hydrostatic_pressure(cfg, phi)
    P = P - P[-1:, :, :]
    return _f32(phi), _f32(u), _f32(P)


FIELDS = {"static_droplet": fields_static_droplet,
          "sessile_drop": fields_sessile_drop,
          "dense_bubble": fields_dense_bubble,
          "drops": fields_drops,
          "rayleigh_taylor": fields_rayleigh_taylor,
          "rising_bubble": fields_rising_bubble,
          "droplet_impact": fields_droplet_impact,
          "dam_break": fields_dam_break}


def fields(cfg):
    return FIELDS[cfg["name"]](cfg)


# ---------------------------------------------------------------------------
# seeded random states (pre-collision distributions) for one-step checks
# ---------------------------------------------------------------------------

_MAG = {9: [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
        19: [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12}


def smooth_random_field(shape, seed, modes=4, lo=0.0, hi=1.0):
    """Sum of a few random long-wave Fourier modes mapped into [lo, hi]."""
    rng = np.random.default_rng(seed)
    z, y, x = _grid(shape)
    nx, ny, nz = shape
    acc = np.zeros_like(x)
    for _ in range(modes):
        kx, ky = rng.integers(0, 3, size=2)
        kz = rng.integers(0, 3) if nz > 1 else 0
        ph = rng.uniform(0, 2 * np.pi)
        acc += np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / max(nz, 1)) + ph)
    acc = (acc - acc.min()) / max(acc.max() - acc.min(), 1e-12)
    return lo + (hi - lo) * acc


def random_state(q, shape, seed, phi=None, h_noise=0.02, g_scale=0.05, g_noise=0.02):
    """Pre-collision populations (h, g), shape (Q, nz, ny, nx), float32.

    h_i = a_i (phi + h_noise * N(0,1)), g_i = a_i (g_scale * s(x) + g_noise * N(0,1)),
    with a_i the usual lattice-weight magnitudes, phi a smooth random field in [0, 1]
    unless given, and s a smooth random field in [-1, 1]."""
    rng = np.random.default_rng(seed + 7919)
    a = np.asarray(_MAG[q]).reshape(q, 1, 1, 1)
    if phi is None:
        phi = smooth_random_field(shape, seed)
    phi = np.asarray(phi, dtype=np.float64)
    s = smooth_random_field(shape, seed + 1, lo=-1.0, hi=1.0)
    nz, ny, nx = phi.shape
    h = a * (phi[None] + h_noise * rng.standard_normal((q, nz, ny, nx)))
    g = a * (g_scale * s[None] + g_noise * rng.standard_normal((q, nz, ny, nx)))
    return _f32(h), _f32(g)


def sample_sites(shape, count, seed, include_faces=True):
    """Integer (S, 3) array of (x, y, z) sites: random ones plus (optionally) the
    corners and face centres of the box, where the boundary rules act."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    pts = [np.stack([rng.integers(0, nx, count), rng.integers(0, ny, count),
                     rng.integers(0, nz, count)], axis=1)]
    if include_faces:
        xs, ys, zs = (0, nx // 2, nx - 1), (0, ny // 2, ny - 1), (0, nz // 2, nz - 1)
        pts.append(np.array([(x, y, z) for x in xs for y in ys for z in zs]))
    return np.unique(np.concatenate(pts), axis=0)


# ---------------------------------------------------------------------------
# hashed states for domains too large to build on the host
# ---------------------------------------------------------------------------

_M32 = 0xFFFFFFFF


def _mix32(x):
    """32-bit integer hash (xor-shift-multiply finaliser) of non-negative int64 values
    below 2^32, on numpy or torch int64 arrays alike (products wrap modulo 2^64, whose
    low 32 bits are the 32-bit product)."""
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & _M32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & _M32
    return x ^ (x >> 16)


class HashedState:
    """Pre-collision populations defined site by site from an integer hash, so that a
    domain of hundreds of millions of sites can be filled on the GPU while the host
    evaluates only the sites it needs, with bitwise the same float32 values:

        u_k(s)  = (mix32((s * 0x9E3779B1 + k * 0x85EBCA77 + seed * 0xC2B2AE3D) mod 2^32) >> 8) 2^-24
        h_i(s)  = a_i (phi(s) + 0.02 (2 u_i(s) - 1)),          phi(s) = u_256(s)
        g_i(s)  = a_i (0.05 (2 u_257(s) - 1) + 0.02 (2 u_{128+i}(s) - 1))

    with s the linear site index (z ny + y) nx + x and a_i the lattice-weight
    magnitudes; every float operation is a single float32 operation in this order."""

    def __init__(self, q, shape, seed):
        self.q = int(q)
        self.shape = tuple(int(v) for v in shape)
        self.seed = int(seed)
        self.a = [np.float32(v) for v in _MAG[self.q]]

    def _u(self, lin, k, xp):
        key = (lin * 0x9E3779B1 + (k * 0x85EBCA77 + self.seed * 0xC2B2AE3D)) & _M32
        m = _mix32(key) >> 8
        if xp is np:
            return m.astype(np.float32) * np.float32(2.0 ** -24)
        return m.to(xp.float32) * (2.0 ** -24)

    def _pop(self, lin, i, xp, c):
        """(h_i, g_i) at the linear indices lin; c holds the float32 constants."""
        one, two, hn, gs = c["1"], c["2"], c["0.02"], c["0.05"]
        phi = self._u(lin, 256, xp)
        s = self._u(lin, 257, xp) * two - one
        h = (phi + (self._u(lin, i, xp) * two - one) * hn) * c["a"][i]
        g = (s * gs + (self._u(lin, 128 + i, xp) * two - one) * hn) * c["a"][i]
        return h, g

    def host(self, lin):
        """(h, g) float32 numpy arrays (Q, len(lin)) at the given linear indices."""
        lin = np.asarray(lin, dtype=np.int64).reshape(-1)
        c = {"1": np.float32(1.0), "2": np.float32(2.0), "0.02": np.float32(0.02),
             "0.05": np.float32(0.05), "a": self.a}
        h = np.empty((self.q, lin.size), dtype=np.float32)
        g = np.empty_like(h)
        for i in range(self.q):
            h[i], g[i] = self._pop(lin, i, np, c)
        return h, g

    def device(self, device):
        """(h, g) float32 torch tensors (Q, nz, ny, nx) built on `device`."""
        import torch
        nx, ny, nz = self.shape
        n = nx * ny * nz
        f = lambda v: torch.tensor(np.float32(v), device=device)  # noqa: E731
        c = {"1": f(1.0), "2": f(2.0), "0.02": f(0.02), "0.05": f(0.05),
             "a": [f(v) for v in self.a]}
        h = torch.empty((self.q, n), dtype=torch.float32, device=device)
        g = torch.empty_like(h)
        lin = torch.arange(n, dtype=torch.int64, device=device)
        for i in range(self.q):
            h[i], g[i] = self._pop(lin, i, torch, c)
        return h.view(self.q, nz, ny, nx), g.view(self.q, nz, ny, nx)

    def lazy(self):
        """Host stand-ins for the full (Q, N) arrays: objects whose `[:, idx]` returns
        the values at those linear indices (what a site-by-site evaluation reads)."""
        st = self

        class _Set:
            def __init__(self, which):
                self.which = which

            def reshape(self, *shape):
                return self

            def __getitem__(self, key):
                rows, idx = key
                assert rows == slice(None)
                return st.host(idx)[self.which]

        return _Set(0), _Set(1)
