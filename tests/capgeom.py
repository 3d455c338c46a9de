"""Contact angle of a two-dimensional cap resting on the y- wall, from its phi field.

A circular cap of radius R meeting the wall at angle t (through the cap) has area
A = R^2 (t - sin t cos t) and height H = R (1 - cos t), so A / H^2 = f(t) with
f(t) = (t - sin t cos t) / (1 - cos t)^2, which falls monotonically from infinity (t -> 0)
to pi/4 (t = pi).  A is sum(phi); H is the height of the phi = 1/2 level on the middle
columns above the wall line y = -1/2.
"""
import math

import numpy as np


def cap_angle(phi):
    """Angle in degrees of the cap in phi (shape (1, ny, nx), the cap centred in x)."""
    phi = np.asarray(phi, dtype=np.float64)
    nx = phi.shape[2]
    A = phi.sum()
    col = phi[0, :, nx // 2 - 1:nx // 2 + 1].mean(1)
    j = int(np.where(col < 0.5)[0][0])
    H = (j - 1) + (col[j - 1] - 0.5) / (col[j - 1] - col[j]) + 0.5
    r = A / H ** 2

    def f(t):
        return (t - math.sin(t) * math.cos(t)) / (1.0 - math.cos(t)) ** 2

    lo, hi = 1e-6, math.pi - 1e-6
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > r else (lo, mid)
    return math.degrees(0.5 * (lo + hi))


def cap_angle_3d(phi):
    """Angle in degrees of a three-dimensional cap on the z- wall (phi of shape
    (nz, ny, nx), the cap centred in x and y): a spherical cap of radius R and angle t
    has volume V = pi R^3 (2 - 3 cos t + cos^3 t) / 3 and height H = R (1 - cos t), so
    V / H^3 = pi (2 - 3 cos t + cos^3 t) / (3 (1 - cos t)^3), which falls monotonically
    from infinity to pi/6."""
    phi = np.asarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    V = phi.sum()
    col = phi[:, ny // 2 - 1:ny // 2 + 1, nx // 2 - 1:nx // 2 + 1].mean((1, 2))
    j = int(np.where(col < 0.5)[0][0])
    H = (j - 1) + (col[j - 1] - 0.5) / (col[j - 1] - col[j]) + 0.5
    r = V / H ** 3

    def f(t):
        c = math.cos(t)
        return math.pi * (2.0 - 3.0 * c + c ** 3) / (3.0 * (1.0 - c) ** 3)

    lo, hi = 1e-6, math.pi - 1e-6
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > r else (lo, mid)
    return math.degrees(0.5 * (lo + hi))
