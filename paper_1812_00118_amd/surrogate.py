"""Python handle of the convolutional surrogate in libpflb (include/pfsur.h).

Argument marshalling only: the network's forward and backward passes, the loss, Adam,
the packing of solver fields and the guarded hand-over run in the library's kernels;
PyTorch provides device memory and the current stream.  Layouts are NHWC: the network
input x is BF16 (batch, H, W, 8), outputs and targets are FP32 (batch, H, W, 4).
"""
import ctypes
import math

import numpy as np
import torch

from ._lib import PflbError, SurCfg, lib

IN_CH, OUT_CH, STEPS = 8, 4, 16

# (name, Cin, Cout) of the 3x3 layers in parameter order (include/pfsur.h), then the head
LAYERS = [("e0a", 8, 32), ("e0b", 32, 32), ("e1a", 32, 64), ("e1b", 64, 64),
          ("e2a", 64, 128), ("e2b", 128, 128), ("b3a", 128, 256), ("b3b", 256, 256),
          ("u2", 256, 128), ("d2a", 256, 128), ("d2b", 128, 128), ("u1", 128, 64),
          ("d1a", 128, 64), ("d1b", 64, 64), ("u0", 64, 32), ("d0a", 64, 32), ("d0b", 32, 32)]
HEAD = (32, OUT_CH)


def init_params(seed, head_scale=0.1):
    """He-normal 3x3 weights, zero biases, a small head (the first predictions stay
    near persistence); flat float32 array in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, cin, cout in LAYERS:
        parts.append(rng.standard_normal(cout * 9 * cin) * math.sqrt(2.0 / (9 * cin)))
        parts.append(np.zeros(cout))
    parts.append(rng.standard_normal(HEAD[0] * HEAD[1]) * head_scale / math.sqrt(HEAD[0]))
    parts.append(np.zeros(HEAD[1]))
    return np.concatenate(parts).astype(np.float32)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Surrogate:
    """H, W: grid; norm: dict with in_shift[4], in_scale[4], out_scale[4], lrr_scale
    (channels phi, P, J_x, J_y)."""

    def __init__(self, H, W, max_batch, norm, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libpflb needs a HIP GPU; none is visible")
        self.L = lib()
        self.device = torch.device(device or "cuda")
        c = SurCfg()
        c.H, c.W, c.max_batch = int(H), int(W), int(max_batch)
        for k in range(4):
            c.in_shift[k] = float(norm["in_shift"][k])
            c.in_scale[k] = float(norm["in_scale"][k])
            c.out_scale[k] = float(norm["out_scale"][k])
        c.lrr_scale = float(norm["lrr_scale"])
        self.cfg = c
        self.H, self.W, self.max_batch = c.H, c.W, c.max_batch
        self.norm = {k: (list(v) if not np.isscalar(v) else float(v)) for k, v in norm.items()}
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.L.pfsur_create(ctypes.byref(c), ctypes.byref(ctx))
        if rc != 0:
            raise PflbError(rc, "pfsur_create failed")
        self.ctx = ctx
        self.nparams = int(self.L.pfsur_num_params())
        self._ws = {}

    def _check(self, rc):
        if rc != 0:
            raise PflbError(rc, self.L.pfsur_last_error(self.ctx).decode())

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                torch.cuda.synchronize(self.device)
                self.L.pfsur_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def workspace(self, batch, training):
        key = (int(batch), bool(training))
        if key not in self._ws:
            n = int(self.L.pfsur_workspace_bytes(ctypes.byref(self.cfg), key[0], int(key[1])))
            if n == 0:
                raise PflbError(-1, f"no workspace for batch {batch}")
            self._ws[key] = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        t = self._ws[key]
        off = (-t.data_ptr()) % 256
        return ctypes.c_void_p(t.data_ptr() + off)

    def layer_io(self, batch, training, layer):
        """Where 3x3 layer `layer` reads and writes its activations in the workspace of
        (batch, training): a dict of the pfsur_layer_io fields (offsets in bytes from the
        workspace's start, None for the network input and for no pooled copy)."""
        from ._lib import LayerIO
        io = LayerIO()
        rc = self.L.pfsur_layer_io_of(ctypes.byref(self.cfg), int(batch), int(training),
                                      int(layer), ctypes.byref(io))
        if rc != 0:
            raise PflbError(rc, "pfsur_layer_io_of")
        none = (1 << (8 * ctypes.sizeof(ctypes.c_size_t))) - 1
        d = {f: getattr(io, f) for f, _ in LayerIO._fields_}
        for k in ("in_off", "pool_off"):
            if d[k] == none:
                d[k] = None
        return d

    def workspace_tensor(self, batch, training):
        """The workspace of (batch, training) as a uint8 tensor starting at the address
        the library is given."""
        ptr = self.workspace(batch, training).value
        t = self._ws[(int(batch), bool(training))]
        off = ptr - t.data_ptr()
        n = int(self.L.pfsur_workspace_bytes(ctypes.byref(self.cfg), int(batch), int(training)))
        return t[off:off + n]

    def release_workspaces(self):
        self._ws = {}

    # ------------------------------------------------------------------ parameters
    def set_params(self, flat):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        if a.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {a.size}")
        self._check(self.L.pfsur_set_params(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        a = np.empty(self.nparams, dtype=np.float32)
        self._check(self.L.pfsur_get_params(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def save(self, path):
        self._check(self.L.pfsur_save(self.ctx, str(path).encode()))

    def load(self, path):
        self._check(self.L.pfsur_load(self.ctx, str(path).encode()))

    # ------------------------------------------------------------------ data
    def _f32(self, t, shape):
        t = torch.as_tensor(t).to(device=self.device, dtype=torch.float32).contiguous()
        return t.reshape(shape)

    @staticmethod
    def _rho(rho, B):
        """(rho_L, rho_H) per sample -> host double array [B][2]."""
        r = np.asarray(rho, dtype=np.float64).reshape(-1, 2)
        if len(r) != B:
            raise ValueError(f"expected {B} (rho_L, rho_H) pairs, got {len(r)}")
        return (ctypes.c_double * (2 * B))(*r.ravel().tolist())

    def pack(self, phi, P, J, rho):
        """phi, P (B, H, W); J (B, 2, H, W); rho: B pairs (rho_L, rho_H).  The network
        input carries the velocity J / rho(phi) (include/pfsur.h)."""
        B = len(np.asarray(rho, dtype=np.float64).reshape(-1, 2))
        phi = self._f32(phi, (B, self.H, self.W))
        P = self._f32(P, (B, self.H, self.W))
        J = self._f32(J, (B, 2, self.H, self.W))
        x = torch.empty((B, self.H, self.W, IN_CH), dtype=torch.bfloat16, device=self.device)
        self._check(self.L.pfsur_pack(self.ctx, _ptr(phi), _ptr(P), _ptr(J), self._rho(rho, B),
                                      B, _ptr(x), _stream(self.device)))
        return x

    def pack_target(self, f0, f1, rho):
        """f0, f1: (phi, P, J) of the same batch 16 steps apart; rho: B pairs (rho_L,
        rho_H) -> y FP32 (B, H, W, 4), the normalised residual of (phi, P, u_x, u_y)."""
        B = f0[0].shape[0]
        a = [self._f32(f0[0], (B, self.H, self.W)), self._f32(f0[1], (B, self.H, self.W)),
             self._f32(f0[2], (B, 2, self.H, self.W)), self._f32(f1[0], (B, self.H, self.W)),
             self._f32(f1[1], (B, self.H, self.W)), self._f32(f1[2], (B, 2, self.H, self.W))]
        y = torch.empty((B, self.H, self.W, OUT_CH), dtype=torch.float32, device=self.device)
        self._check(self.L.pfsur_pack_target(self.ctx, *[_ptr(t) for t in a], self._rho(rho, B),
                                             B, _ptr(y), _stream(self.device)))
        return y

    def forward(self, x):
        B = x.shape[0]
        out = torch.empty((B, self.H, self.W, OUT_CH), dtype=torch.float32, device=self.device)
        self._check(self.L.pfsur_forward(self.ctx, _ptr(x), _ptr(out), B,
                                         self.workspace(B, False), _stream(self.device)))
        return out

    def apply(self, out, phi, P, J, rho):
        """In place: phi, P and the velocity J / rho(phi) advance by out * out_scale, J is
        rebuilt from the new phi (phi, P, J: contiguous float32 device tensors (B, H, W),
        (B, H, W), (B, 2, H, W); rho: B pairs (rho_L, rho_H))."""
        B = out.shape[0]
        for t in (phi, P, J):
            assert t.is_contiguous() and t.dtype == torch.float32
        self._check(self.L.pfsur_apply(self.ctx, _ptr(out), _ptr(phi), _ptr(P), _ptr(J),
                                       self._rho(rho, B), B, _stream(self.device)))

    def train_step(self, x, y, lr):
        B = x.shape[0]
        loss = ctypes.c_float()
        self._check(self.L.pfsur_train_step(self.ctx, _ptr(x), _ptr(y), B, float(lr),
                                            ctypes.byref(loss), self.workspace(B, True),
                                            _stream(self.device)))
        return float(loss.value)

    def gradients(self, x, y):
        B = x.shape[0]
        g = np.empty(self.nparams, dtype=np.float32)
        loss = ctypes.c_float()
        self._check(self.L.pfsur_gradients(self.ctx, _ptr(x), _ptr(y), B,
                                           g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss),
                                           self.workspace(B, True), _stream(self.device)))
        return g, float(loss.value)

    # ------------------------------------------------------------------ hand-over
    def advance_guarded(self, sims, windows, mass_tol=1e-3, phi_tol=0.05, check_every=0,
                        u_max=0.1, trace=False):
        """Advance D2Q9 periodic Sims (one, or a list of at most max_batch) by windows x 16
        steps with one batched forward pass per window; returns the number of (window,
        sim) pairs that fell back to the plain steps.  A prediction is rejected when it
        changes sum(phi) from its value at the start of the call by more than mass_tol
        (relative), when its largest speed exceeds u_max, or (on every check_every-th
        window) when it is more than phi_tol from the plain steps.  With trace=True returns
        (n_fallback, records), records a float64 array [windows][len(sims)][6] of
        (sum phi at the start, sum phi_in, sum phi_out, max speed, max|phi_out - phi_LB|
        (NaN unchecked), accepted) per decision."""
        if not isinstance(sims, (list, tuple)):
            sims = [sims]
        n = len(sims)
        nb = int(self.L.pfsur_guard_work_bytes(ctypes.byref(self.cfg), n))
        if nb == 0:
            raise PflbError(-1, f"no guard workspace for {n} contexts")
        work = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        wp = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        ctxs = (ctypes.c_void_p * n)(*[s.ctx.value for s in sims])
        nf = ctypes.c_int()
        rec = np.zeros((max(int(windows), 0), n, 6), dtype=np.float64) if trace else None
        self._check(self.L.pflb_advance_guarded_trace(
            ctxs, n, self.ctx, int(windows), float(mass_tol), float(phi_tol), float(u_max),
            int(check_every), ctypes.byref(nf),
            rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if trace else None, wp,
            _stream(self.device)))
        return (int(nf.value), rec) if trace else int(nf.value)


# ---------------------------------------------------------------------- building blocks

def conv_fwd(x, w, b=None, mode=0, act=True):
    """One 3x3 layer: x BF16 NHWC, w BF16 (Cout, 3, 3, Cin), b FP32 (Cout,) or None.
    Returns (y_pre FP32, y_act BF16) of shape (B, H, W, Cout)."""
    L = lib()
    B, Hin, Win, Cin = x.shape
    H, W = {0: (Hin, Win), 1: (2 * Hin, 2 * Win), 2: (Hin // 2, Win // 2)}[mode]
    Cout = w.shape[0]
    y_pre = torch.empty((B, H, W, Cout), dtype=torch.float32, device=x.device)
    y_act = torch.empty((B, H, W, Cout), dtype=torch.bfloat16, device=x.device)
    rc = L.pfsur_conv_fwd(_ptr(x.contiguous()), B, H, W, Cin, Cout, mode, _ptr(w.contiguous()),
                          _ptr(b), int(bool(act)), _ptr(y_pre), _ptr(y_act), _stream(x.device))
    if rc != 0:
        raise PflbError(rc, "pfsur_conv_fwd")
    return y_pre, y_act


def conv_wgrad(x, dy, mode=0):
    """Weight and bias gradients of one 3x3 layer from its input x (BF16 NHWC) and the
    gradient dy (BF16, (B, H, W, Cout)).  Returns (dw (Cout, 3, 3, Cin), db (Cout,))."""
    L = lib()
    B, H, W, Cout = dy.shape
    Cin = x.shape[3]
    n = int(L.pfsur_conv_wgrad_work_bytes(B, H, W, Cin, Cout))
    work = torch.empty(max(n, 4) // 4 + 64, dtype=torch.float32, device=x.device)
    dw = torch.empty((Cout, 3, 3, Cin), dtype=torch.float32, device=x.device)
    db = torch.empty((Cout,), dtype=torch.float32, device=x.device)
    rc = L.pfsur_conv_wgrad(_ptr(x.contiguous()), _ptr(dy.contiguous()), B, H, W, Cin, Cout, mode,
                            _ptr(dw), _ptr(db), _ptr(work), _stream(x.device))
    if rc != 0:
        raise PflbError(rc, "pfsur_conv_wgrad")
    return dw, db
