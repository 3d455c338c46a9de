"""Data generation, training and evaluation of the 16-step surrogate.

The solver (Sim, FP32 storage) generates trajectories of the seeded multi-droplet
family; states every 16 steps form (t, t + 16) pairs.  The library packs inputs and
targets, runs forward/backward/Adam, and applies predictions; this module only
schedules those calls and keeps the dataset in device memory.
"""
import math
import time

import numpy as np
import torch

from .sim import Sim
from .surrogate import STEPS, Surrogate


def trajectory(cfg, fields, t0, n_states, stride=STEPS):
    """Run the solver from `fields` and return the states at t0, t0 + stride, ...:
    phi, P (K, H, W) and J (K, 2, H, W) float32 device tensors."""
    sim = Sim(cfg)
    phi0, u0, P0 = fields
    sim.init_fields(phi0, u0, P0)
    sim.release_work()
    sim.step(t0)
    phis, Ps, Js = [], [], []
    for k in range(n_states):
        if k:
            sim.step(stride)
        f = sim.read(("phi", "P", "J"))
        phis.append(f["phi"].reshape(f["phi"].shape[-2:]))
        Ps.append(f["P"].reshape(f["P"].shape[-2:]))
        Js.append(f["J"].reshape((2,) + f["J"].shape[-2:]))
    mass, bad = sim.mass()
    if bad:
        raise FloatingPointError(f"trajectory of seed {cfg.get('seed')} became non-finite")
    return torch.stack(phis), torch.stack(Ps), torch.stack(Js)


class Dataset:
    """States of several trajectories, and the (t, t + 16) pairs inside each."""

    def __init__(self, seeds, make_cfg, t0=64, n_states=9, log=None):
        import pfinputs as I
        phi, P, J, rho, pairs = [], [], [], [], []
        base = 0
        t = time.time()
        for s in seeds:
            cfg = make_cfg(s)
            f = I.fields(cfg)
            a, b, c = trajectory(I.model_params(cfg), f, t0, n_states)
            phi.append(a)
            P.append(b)
            J.append(c)
            rho += [(cfg["rho_L"], cfg["rho_H"])] * n_states
            pairs += [(base + k, base + k + 1) for k in range(n_states - 1)]
            base += n_states
        self.phi = torch.cat(phi)
        self.P = torch.cat(P)
        self.J = torch.cat(J)
        self.rho = np.asarray(rho, dtype=np.float64)           # (rho_L, rho_H) per state
        self.lrr = np.log10(self.rho[:, 1] / self.rho[:, 0])
        self.pairs = np.asarray(pairs, dtype=np.int64)
        self.seconds = time.time() - t
        if log:
            log(f"dataset: {len(seeds)} trajectories, {len(self.pairs)} pairs, "
                f"{self.seconds:.1f} s")

    def __len__(self):
        return len(self.pairs)

    def fields(self, idx):
        i = torch.as_tensor(idx, device=self.phi.device)
        return (self.phi.index_select(0, i).contiguous(), self.P.index_select(0, i).contiguous(),
                self.J.index_select(0, i).contiguous())


def velocity(ds):
    """u = J / rho(phi) per state, rho(phi) = rho_L + clamp(phi, 0, 1) (rho_H - rho_L):
    the quantity the network sees and predicts in place of J."""
    r = torch.as_tensor(ds.rho, dtype=torch.float32, device=ds.phi.device)
    rho = r[:, 0, None, None] + ds.phi.clamp(0.0, 1.0) * (r[:, 1] - r[:, 0])[:, None, None]
    return ds.J / rho[:, None]


def normalisation(ds):
    """Per-channel standardisation of the inputs (phi, P, u_x, u_y) and of their 16-step
    residuals."""
    u = velocity(ds)
    f0 = [ds.phi, ds.P, u[:, 0], u[:, 1]]
    a = torch.as_tensor(ds.pairs[:, 0], device=ds.phi.device)
    b = torch.as_tensor(ds.pairs[:, 1], device=ds.phi.device)
    shift, scale, out = [], [], []
    for f in f0:
        shift.append(float(f.mean()))
        scale.append(1.0 / max(float(f.std()), 1e-12))
        out.append(max(float((f.index_select(0, b) - f.index_select(0, a)).std()), 1e-12))
    lmin, lmax = float(ds.lrr.min()), float(ds.lrr.max())
    return dict(in_shift=shift, in_scale=scale, out_scale=out,
                lrr_scale=1.0 / max(lmax, 1.0))


def batch(sur, ds, idx):
    p = ds.pairs[idx]
    f0 = ds.fields(p[:, 0])
    f1 = ds.fields(p[:, 1])
    rho = ds.rho[p[:, 0]]
    x = sur.pack(*f0, rho)
    y = sur.pack_target(f0, f1, rho)
    return x, y


def train(sur, ds, steps, batch_size, lr, seed=0, log=None, log_every=50):
    rng = np.random.default_rng(seed)
    losses = []
    t = time.time()
    for k in range(steps):
        idx = rng.choice(len(ds), size=batch_size, replace=len(ds) < batch_size)
        x, y = batch(sur, ds, idx)
        # cosine decay of the learning rate
        lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / max(steps, 1)))
        losses.append(sur.train_step(x, y, lr_k))
        if log and (k % log_every == 0 or k == steps - 1):
            log(f"step {k:5d}  loss {losses[-1]:.4e}  {time.time() - t:.1f} s")
    return np.asarray(losses)


def evaluate(sur, ds, batch_size=8):
    """Normalised MSE of the network and of persistence (zero residual), and the max
    phi error of one window for both, over all pairs of ds."""
    se_net = se_pers = 0.0
    n = 0
    err_net = err_pers = 0.0
    for s in range(0, len(ds), batch_size):
        idx = np.arange(s, min(len(ds), s + batch_size))
        p = ds.pairs[idx]
        f0 = ds.fields(p[:, 0])
        f1 = ds.fields(p[:, 1])
        rho = ds.rho[p[:, 0]]
        x = sur.pack(*f0, rho)
        y = sur.pack_target(f0, f1, rho)
        out = sur.forward(x)
        se_net += float(((out - y) ** 2).sum())
        se_pers += float((y ** 2).sum())
        n += y.numel()
        phi, P, J = (t.clone() for t in f0)
        sur.apply(out, phi, P, J, rho)
        err_net = max(err_net, float((phi - f1[0]).abs().max()))
        err_pers = max(err_pers, float((f0[0] - f1[0]).abs().max()))
    return dict(mse=se_net / n, mse_persistence=se_pers / n, phi_err=err_net,
                phi_err_persistence=err_pers)
