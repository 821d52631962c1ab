"""Exact circular and spherical transforms of disks and balls (pins).

These follow from elementary geometry, not from the paper; they pin the
oracle's circle transform (Sec. 2, measure rho dphi), its half-circle transform
(measure l dtheta) and their composition (the surface integral of Sec. 2).
"""
from __future__ import annotations

import numpy as np


def circle_in_disk(l, d, a):
    """Length of the circle of radius l whose centre is at distance d from the
    centre of a disk of radius a, inside that disk."""
    l, d, a = np.broadcast_arrays(np.asarray(l, float), np.asarray(d, float),
                                  np.asarray(a, float))
    out = np.zeros(l.shape)
    full = l <= a - d
    out[full] = 2.0 * np.pi * l[full]
    part = (np.abs(d - a) < l) & (l < d + a) & ~full
    c = (l[part] ** 2 + d[part] ** 2 - a[part] ** 2) / (2.0 * l[part] * d[part])
    out[part] = 2.0 * l[part] * np.arccos(np.clip(c, -1.0, 1.0))
    return out


def sphere_in_ball(l, d, a):
    """Area of the sphere of radius l whose centre is at distance d from the
    centre of a ball of radius a, inside that ball (spherical cap area):
    4 pi l^2 when the sphere lies inside, pi l / d (a^2 - (d - l)^2) when the
    two surfaces cross, 0 otherwise."""
    l, d, a = np.broadcast_arrays(np.asarray(l, float), np.asarray(d, float),
                                  np.asarray(a, float))
    out = np.zeros(l.shape)
    full = l <= a - d
    out[full] = 4.0 * np.pi * l[full] ** 2
    part = (np.abs(d - a) < l) & (l < d + a) & ~full
    out[part] = np.pi * l[part] / d[part] * (a[part] ** 2 - (d[part] - l[part]) ** 2)
    return out


def srt_of_balls(ap, balls: np.ndarray) -> np.ndarray:
    """Exact SRT (surface integral, Sec. 2) of a sum of uniform balls, sampled
    at every sensor (a, h) and radius l: Y[a][h][l]."""
    ca = np.stack([ap.radius * np.cos(ap.angles), ap.radius * np.sin(ap.angles)], -1)
    Y = np.zeros(ap.data_shape)
    for cx, cy, cz, r, amp in balls:
        dxy2 = (ca[:, 0] - cx) ** 2 + (ca[:, 1] - cy) ** 2  # [a]
        d = np.sqrt(dxy2[:, None] + (ap.zpos[None, :] - cz) ** 2)  # [a][h]
        Y += amp * sphere_in_ball(ap.radii[None, None, :], d[:, :, None], r)
    return Y
