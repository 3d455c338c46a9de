"""Python handle of one lattice Boltzmann context of libpflb (device memory via torch)."""
import ctypes
import math

import numpy as np
import torch

from ._lib import (BC_PERIODIC, BC_WALL, ERR_NONFINITE, NBUF, Params, PflbError,
                   STORE_FP16S, STORE_FP32, STORE_FP32_INPLACE, lib)

_BC = {"periodic": BC_PERIODIC, "wall": BC_WALL, BC_PERIODIC: BC_PERIODIC, BC_WALL: BC_WALL}


def default_scales(rho_H):
    """Power-of-two scale exponents of the fp16 deviations of h and g: h deviations are
    O(w_i) <= 1, g deviations grow with rho_H |u| (kept below 2^15 / scale)."""
    sg = 15 - int(math.ceil(math.log2(max(rho_H, 1.0) * 0.05))) - 2
    return 16, max(-14, min(24, sg))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Sim:
    """cfg: dict with lattice (9/19), shape (nx, ny, nz), bc (per axis 'periodic'/'wall'),
    rho_L, rho_H, nu_L, nu_H, M, W, sigma, g (3), eps, hoc, dtheta_C; optionally wall_u
    (6 faces x 3) and wet_cos (cos of the contact angle per face), faces x-, x+, y-, y+,
    z-, z+.
    Fields use shape (nz, ny, nx) (nz = 1 for D2Q9), vectors (D, nz, ny, nx),
    distributions (Q, nz, ny, nx)."""

    def __init__(self, cfg, storage="fp32", scale_log2=None, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libpflb needs a HIP GPU; none is visible")
        self.L = lib()
        self.device = torch.device(device or "cuda")
        p = Params()
        p.lattice = int(cfg["lattice"])
        p.nx, p.ny, p.nz = (int(v) for v in cfg["shape"])
        for a in range(3):
            p.bc[a] = _BC[cfg["bc"][a]]
        for k in ("rho_L", "rho_H", "nu_L", "nu_H", "M", "W", "sigma"):
            setattr(p, k, float(cfg[k]))
        for a in range(3):
            p.g[a] = float(cfg.get("g", (0, 0, 0))[a])
        p.eps = float(cfg.get("eps", 1e-10))
        p.hoc = int(cfg.get("hoc", 1))
        p.dtheta_C = float(cfg.get("dtheta_C", 0.0))
        p.storage = {"fp32": STORE_FP32, "fp16s": STORE_FP16S,
                     "fp32_inplace": STORE_FP32_INPLACE}[storage]
        sl = scale_log2 if scale_log2 is not None else default_scales(p.rho_H)
        p.scale_log2[0], p.scale_log2[1] = int(sl[0]), int(sl[1])
        wu = cfg.get("wall_u")
        if wu is not None:
            wu = [float(v) for row in wu for v in row]
            if len(wu) != 18:
                raise ValueError("wall_u: 6 faces x 3 components")
            for k in range(18):
                p.wall_u[k] = wu[k]
        wc = cfg.get("wet_cos")
        if wc is not None:
            wc = [float(v) for v in np.asarray(wc).reshape(-1)]
            if len(wc) != 6:
                raise ValueError("wet_cos: one value per face")
            for k in range(6):
                p.wet_cos[k] = wc[k]
        op = cfg.get("open_P")
        if op is not None:
            # faces with a finite pressure are open (NaN: a closed wall), rows as wall_u
            op = [float(v) for v in np.asarray(op, dtype=np.float64).reshape(-1)]
            if len(op) != 6:
                raise ValueError("open_P: one value per face")
            for k in range(6):
                if not math.isnan(op[k]):
                    p.open[k] = 1
                    p.open_P[k] = op[k]
        self.params = p
        self.Q = p.lattice
        self.D = 3 if p.lattice == 19 else 2
        self.shape = (p.nz, p.ny, p.nx)
        self.N = p.nx * p.ny * p.nz
        ctx = ctypes.c_void_p()
        rc = self.L.pflb_create(ctypes.byref(p), ctypes.byref(ctx))
        if rc != 0:
            raise PflbError(rc, "invalid parameters")
        self.ctx = ctx
        with torch.cuda.device(self.device):
            self.bufs = [torch.empty(int(self.L.pflb_required_bytes(ctypes.byref(p), k)),
                                     dtype=torch.uint8, device=self.device)
                         for k in range(NBUF)]
        arr = (ctypes.c_void_p * NBUF)(*[b.data_ptr() for b in self.bufs])
        self._check(self.L.pflb_bind(self.ctx, arr, NBUF))
        self._work = None

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc):
        if rc != 0:
            raise PflbError(rc, self.L.pflb_last_error(self.ctx).decode())

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, shape):
        t = torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a)
        t = t.to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.L.pflb_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ------------------------------------------------------------------ state
    def equilibrium(self, phi, u, P=None):
        phi_t = self._dev(phi, self.shape)
        u_t = self._dev(np.asarray(u)[:self.D] if not torch.is_tensor(u) else u[:self.D],
                        (self.D,) + self.shape)
        P_t = self._dev(P, self.shape) if P is not None else None
        h = torch.empty((self.Q,) + self.shape, device=self.device)
        g = torch.empty_like(h)
        self._check(self.L.pflb_equilibrium(self.ctx, _ptr(phi_t), _ptr(u_t), _ptr(P_t),
                                            _ptr(h), _ptr(g), self._stream()))
        return h, g

    def init_fields(self, phi, u, P=None):
        phi_t = self._dev(phi, self.shape)
        u_t = self._dev(np.asarray(u)[:self.D] if not torch.is_tensor(u) else u[:self.D],
                        (self.D,) + self.shape)
        P_t = self._dev(P, self.shape) if P is not None else None
        if self._work is None and self.params.storage != STORE_FP32_INPLACE:
            # in-place storage takes the equilibria straight into its state
            self._work = torch.empty(2 * self.Q * self.N, device=self.device)
        self._check(self.L.pflb_init_fields(self.ctx, _ptr(phi_t), _ptr(u_t), _ptr(P_t),
                                            _ptr(self._work), self._stream()))

    def init_fields_noalloc(self, phi, u, P=None):
        """init_fields through pflb_init_fields_noalloc: the library stages the
        equilibria in its fixed device array (no work buffer; domains up to
        pflb_noalloc_scratch_bytes() / (8 Q) sites)."""
        phi_t = self._dev(phi, self.shape)
        u_t = self._dev(np.asarray(u)[:self.D] if not torch.is_tensor(u) else u[:self.D],
                        (self.D,) + self.shape)
        P_t = self._dev(P, self.shape) if P is not None else None
        self._check(self.L.pflb_init_fields_noalloc(self.ctx, _ptr(phi_t), _ptr(u_t),
                                                    _ptr(P_t), self._stream()))

    def reconstruct(self, phi, J, P=None, advance=0):
        """Replace the state by the equilibria of (phi, P, J); the step counter grows by
        `advance`."""
        phi_t = self._dev(phi, self.shape)
        J_t = self._dev(J, (self.D,) + self.shape)
        P_t = self._dev(P, self.shape) if P is not None else None
        work = torch.empty((2 * self.Q + self.D) * self.N, device=self.device)
        self._check(self.L.pflb_reconstruct(self.ctx, _ptr(phi_t), _ptr(P_t), _ptr(J_t),
                                            _ptr(work), int(advance), self._stream()))
        torch.cuda.current_stream(self.device).synchronize()

    def release_work(self):
        self._work = None

    def set_state(self, h, g):
        h_t = self._dev(h, (self.Q,) + self.shape)
        g_t = self._dev(g, (self.Q,) + self.shape)
        self._check(self.L.pflb_set_state(self.ctx, _ptr(h_t), _ptr(g_t), self._stream()))

    def get_state(self):
        h = torch.empty((self.Q,) + self.shape, device=self.device)
        g = torch.empty_like(h)
        self._check(self.L.pflb_get_state(self.ctx, _ptr(h), _ptr(g), self._stream()))
        return h, g

    def step(self, n=1):
        self._check(self.L.pflb_step(self.ctx, int(n), self._stream()))

    def step_graph(self, n=1):
        """step(n) replayed from a captured HIP graph (pflb_step_graph); needs torch's
        current stream to be a created stream, not the null stream."""
        self._check(self.L.pflb_step_graph(self.ctx, int(n), self._stream()))

    @staticmethod
    def step_many(sims, n=1):
        """Advance several Sims by n steps each (pflb_step_many): one launch per step for
        every 16 of them.  They must share lattice, storage, sizes and walls; the result
        is what each one's own step(n) gives."""
        sims = list(sims)
        if not sims:
            return
        ctxs = (ctypes.c_void_p * len(sims))(*[s.ctx.value for s in sims])
        s0 = sims[0]
        s0._check(s0.L.pflb_step_many(ctxs, len(sims), int(n), s0._stream()))

    @property
    def steps(self):
        return int(self.L.pflb_step_count(self.ctx))

    def read(self, fields=("phi", "P", "J", "u")):
        phi = torch.empty(self.shape, device=self.device)
        P = torch.empty(self.shape, device=self.device) if "P" in fields else None
        J = torch.empty((self.D,) + self.shape, device=self.device) if "J" in fields else None
        u = torch.empty((self.D,) + self.shape, device=self.device) if "u" in fields else None
        self._check(self.L.pflb_read(self.ctx, _ptr(phi), _ptr(P), _ptr(J), _ptr(u),
                                     self._stream()))
        out = {"phi": phi, "P": P, "J": J, "u": u}
        return {k: v for k, v in out.items() if v is not None}

    def mass(self):
        """(sum of phi in float64, nonfinite flag) -- synchronous."""
        s = ctypes.c_double()
        f = ctypes.c_int()
        rc = self.L.pflb_mass(self.ctx, ctypes.byref(s), ctypes.byref(f), self._stream())
        if rc not in (0, ERR_NONFINITE):
            self._check(rc)
        return s.value, bool(f.value)

    def save(self, path):
        self._check(self.L.pflb_save(self.ctx, str(path).encode(), self._stream()))

    def load(self, path):
        self._check(self.L.pflb_load(self.ctx, str(path).encode(), self._stream()))
