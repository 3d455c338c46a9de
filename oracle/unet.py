"""FP64 reference of the convolutional surrogate (forward, backward, loss, optimiser).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The surrogate is not part of
the paper: it is the learned 16-step advance that sits beside the lattice Boltzmann
solver.  Everything here is written from the textbook definitions, in float64 numpy,
over whole arrays.

Tensors are NHWC: (B, H, W, C).  A 3x3 convolution with circular padding is
    out[b, y, x, o] = bias[o] + sum_{ky, kx, c} in[b, (y + ky - 1) % H, (x + kx - 1) % W, c]
                                                * w[o, ky, kx, c]
with weights w of shape (Cout, 3, 3, Cin).  "up" convolutions read their input through
a 2x nearest upsampling, in_up[y, x] = in[y // 2, x // 2].

Network (4 levels, 32 / 64 / 128 / 256 channels, SiLU after every 3x3 convolution):
  e0a = conv(x, 8->32)     e0b = conv(e0a, 32->32)            (256^2)
  e1a = conv(pool(e0b))    e1b = conv(e1a, 64->64)             (128^2)
  e2a = conv(pool(e1b))    e2b = conv(e2a, 128->128)           (64^2)
  b3a = conv(pool(e2b))    b3b = conv(b3a, 256->256)           (32^2)
  u2 = upconv(b3b, 256->128); d2a = conv([e2b, u2], 256->128); d2b = conv(d2a)
  u1 = upconv(d2b, 128->64);  d1a = conv([e1b, u1], 128->64);  d1b = conv(d1a)
  u0 = upconv(d1b, 64->32);   d0a = conv([e0b, u0], 64->32);   d0b = conv(d0a)
  out = head(d0b, 32->4)  (1x1, no activation)
"""
import numpy as np

# (name, input(s), Cin, Cout, level, kind) -- kind: conv | up (input upsampled 2x)
LAYERS = [
    ("e0a", ("x",), 8, 32, 0, "conv"),
    ("e0b", ("e0a",), 32, 32, 0, "conv"),
    ("e1a", ("pool:e0b",), 32, 64, 1, "conv"),
    ("e1b", ("e1a",), 64, 64, 1, "conv"),
    ("e2a", ("pool:e1b",), 64, 128, 2, "conv"),
    ("e2b", ("e2a",), 128, 128, 2, "conv"),
    ("b3a", ("pool:e2b",), 128, 256, 3, "conv"),
    ("b3b", ("b3a",), 256, 256, 3, "conv"),
    ("u2", ("b3b",), 256, 128, 2, "up"),
    ("d2a", ("e2b", "u2"), 256, 128, 2, "conv"),
    ("d2b", ("d2a",), 128, 128, 2, "conv"),
    ("u1", ("d2b",), 128, 64, 1, "up"),
    ("d1a", ("e1b", "u1"), 128, 64, 1, "conv"),
    ("d1b", ("d1a",), 64, 64, 1, "conv"),
    ("u0", ("d1b",), 64, 32, 0, "up"),
    ("d0a", ("e0b", "u0"), 64, 32, 0, "conv"),
    ("d0b", ("d0a",), 32, 32, 0, "conv"),
]
HEAD = ("head", 32, 4)
IN_CH = 8
OUT_CH = 4


# --------------------------------------------------------------------------- primitives

def conv3x3(x, w, b):
    """Circular-padded 3x3 convolution (definition in the module docstring)."""
    B, H, W, C = x.shape
    out = np.zeros((B, H, W, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))    # xs[y,x] = x[y+ky-1, x+kx-1]
            out += xs @ w[:, ky, kx, :].T
    return out


def conv3x3_backward(x, w, dout):
    """Gradients of conv3x3 with respect to input, weights and bias."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dout, xs)
            g = dout @ w[:, ky, kx, :]                               # d xs
            dx += np.roll(g, shift=(ky - 1, kx - 1), axis=(1, 2))
    db = dout.sum(axis=(0, 1, 2))
    return dx, dw, db


def upsample2(x):
    """Nearest 2x upsampling: out[y, x] = in[y // 2, x // 2]."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(d):
    B, H, W, C = d.shape
    return d.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def avgpool2(x):
    """2x2 average pooling with stride 2."""
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(d):
    return upsample2(d) / 4.0


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mse(pred, target):
    """Mean squared error over all elements and its gradient."""
    d = pred - target
    return float((d * d).mean()), 2.0 * d / d.size


def adam(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns the new (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------- network

def init_weights(seed, scale=1.0):
    """He-style random weights for every layer (seeded; the same numbers are given to
    the GPU library).  Returns {name: (w, b)}."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, _, cin, cout, _, _ in LAYERS:
        out[name] = (scale * rng.standard_normal((cout, 3, 3, cin)) * np.sqrt(2.0 / (9 * cin)),
                     0.01 * rng.standard_normal(cout))
    out["head"] = (scale * rng.standard_normal((OUT_CH, 1, 1, 32)) * np.sqrt(1.0 / 32),
                   np.zeros(OUT_CH))
    return out


def _gather(acts, src):
    if src.startswith("pool:"):
        return avgpool2(acts[src[5:]])
    return acts[src]


def forward(params, x):
    """x: (B, 256, 256, 8).  Returns (out, cache)."""
    acts = {"x": x}
    z = {}
    inputs = {}
    for name, srcs, cin, cout, lvl, kind in LAYERS:
        xin = np.concatenate([_gather(acts, s) for s in srcs], axis=3)
        if kind == "up":
            xin = upsample2(xin)
        w, b = params[name]
        inputs[name] = xin
        z[name] = conv3x3(xin, w, b)
        acts[name] = silu(z[name])
    wh, bh = params["head"]
    out = acts["d0b"] @ wh[:, 0, 0, :].T + bh
    return out, dict(acts=acts, z=z, inputs=inputs)


def backward(params, cache, dout):
    """Gradients of all parameters given d(loss)/d(out).  Returns {name: (dw, db)}."""
    acts, z, inputs = cache["acts"], cache["z"], cache["inputs"]
    grads = {}
    wh, _ = params["head"]
    grads["head"] = (np.einsum("bhwo,bhwc->oc", dout, acts["d0b"])[:, None, None, :],
                     dout.sum(axis=(0, 1, 2)))
    dacts = {name: np.zeros_like(a) for name, a in acts.items()}
    dacts["d0b"] += dout @ wh[:, 0, 0, :]
    for name, srcs, cin, cout, lvl, kind in reversed(LAYERS):
        dz = dacts[name] * silu_grad(z[name])
        w, _ = params[name]
        dxin, dw, db = conv3x3_backward(inputs[name], w, dz)
        grads[name] = (dw, db)
        if kind == "up":
            dxin = upsample2_backward(dxin)
        c0 = 0
        for s in srcs:
            src = s[5:] if s.startswith("pool:") else s
            a = _gather(acts, s)
            part = dxin[..., c0:c0 + a.shape[3]]
            c0 += a.shape[3]
            dacts[src] += avgpool2_backward(part) if s.startswith("pool:") else part
    return grads
