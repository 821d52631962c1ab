"""Seeded synthetic phantoms and data arrays.

Every generator takes a numpy Generator and returns float64 arrays laid out
[z][y][x] (volumes) or [angle][height][radius] (data). Seeds follow one rule:
1000 + config number for a phantom, 2000 + config number for noise or adjoint
data, 4000 + i for the i-th volume of the differentiation batch.

The partial-volume and centre-voxel rules below decide which voxels a shape
covers. They are input generation only; nothing here integrates over spheres
or circles.
"""
from __future__ import annotations

import numpy as np

from .configs import Aperture


def voxel_centres(ap: Aperture):
    """1-D centre coordinates (x == y, z) of the voxel grid."""
    c = ap.x0 + (np.arange(ap.ms) + 0.5) * ap.dxy
    cz = ap.z0 + (np.arange(ap.mz) + 0.5) * ap.dz
    return c, cz


def _box(ap: Aperture, lo, hi):
    """Index ranges (clipped) of voxels whose cells meet the box [lo, hi]."""
    i0 = max(int(np.floor((lo[0] - ap.x0) / ap.dxy)), 0)
    i1 = min(int(np.floor((hi[0] - ap.x0) / ap.dxy)) + 1, ap.ms)
    j0 = max(int(np.floor((lo[1] - ap.x0) / ap.dxy)), 0)
    j1 = min(int(np.floor((hi[1] - ap.x0) / ap.dxy)) + 1, ap.ms)
    k0 = max(int(np.floor((lo[2] - ap.z0) / ap.dz)), 0)
    k1 = min(int(np.floor((hi[2] - ap.z0) / ap.dz)) + 1, ap.mz)
    return (i0, i1), (j0, j1), (k0, k1)


def balls_params(rng: np.random.Generator, n: int = 3, r_range=(0.1, 0.3),
                 c_range=(-0.6, 0.6), amp_range=(0.5, 1.5)):
    """n balls: rows (cx, cy, cz, radius, amplitude)."""
    r = rng.uniform(*r_range, size=n)
    c = rng.uniform(*c_range, size=(n, 3))
    amp = rng.uniform(*amp_range, size=n)
    return np.column_stack([c, r, amp])


def voxelize_balls(ap: Aperture, balls: np.ndarray, sub: int = 4) -> np.ndarray:
    """Partial-volume voxelisation: each voxel takes amplitude times the
    fraction of its sub^3 regular sub-samples that fall inside a ball."""
    vol = np.zeros(ap.vol_shape)
    off = (np.arange(sub) + 0.5) / sub
    for cx, cy, cz, r, amp in balls:
        (i0, i1), (j0, j1), (k0, k1) = _box(ap, (cx - r, cy - r, cz - r), (cx + r, cy + r, cz + r))
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        xs = ap.x0 + (np.arange(i0, i1)[:, None] + off[None, :]).ravel() * ap.dxy
        ys = ap.x0 + (np.arange(j0, j1)[:, None] + off[None, :]).ravel() * ap.dxy
        zs = ap.z0 + (np.arange(k0, k1)[:, None] + off[None, :]).ravel() * ap.dz
        inside = ((zs[:, None, None] - cz) ** 2 + (ys[None, :, None] - cy) ** 2
                  + (xs[None, None, :] - cx) ** 2) <= r * r
        frac = inside.reshape(k1 - k0, sub, j1 - j0, sub, i1 - i0, sub).mean(axis=(1, 3, 5))
        vol[k0:k1, j0:j1, i0:i1] += amp * frac
    return vol


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices, uniform on SO(3) (normalised Gaussian quaternions)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def ellipsoid_phantom(ap: Aperture, rng: np.random.Generator, n: int = 20,
                      axes_range=(0.02, 0.25), c_range=(-0.6, 0.6),
                      amp_range=(-0.5, 1.0), noise_rng: np.random.Generator | None = None,
                      noise_sigma: float = 0.01) -> np.ndarray:
    """n random ellipsoids (centre-voxel test, additive) plus optional
    i.i.d. N(0, noise_sigma^2) voxel noise."""
    axes = rng.uniform(*axes_range, size=(n, 3))
    rot = random_rotations(rng, n)
    cen = rng.uniform(*c_range, size=(n, 3))
    amp = rng.uniform(*amp_range, size=n)
    cx, cz = voxel_centres(ap)
    vol = np.zeros(ap.vol_shape)
    for e in range(n):
        rmax = axes[e].max()
        lo, hi = cen[e] - rmax, cen[e] + rmax
        (i0, i1), (j0, j1), (k0, k1) = _box(ap, lo, hi)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        Z, Y, X = np.meshgrid(cz[k0:k1], cx[j0:j1], cx[i0:i1], indexing="ij")
        d = np.stack([X - cen[e, 0], Y - cen[e, 1], Z - cen[e, 2]], -1)
        local = d @ rot[e]  # coordinates along the ellipsoid's own axes
        inside = ((local / axes[e]) ** 2).sum(-1) <= 1.0
        vol[k0:k1, j0:j1, i0:i1] += amp[e] * inside
    if noise_rng is not None and noise_sigma > 0:
        vol += noise_rng.normal(0.0, noise_sigma, size=vol.shape)
    return vol


def cylinder_phantom(ap: Aperture, rng: np.random.Generator, n: int = 200,
                     r_range=(0.2, 1.0), len_range=(2.0, 15.0),
                     centre_ball: float | None = None, amp: float = 1.0) -> np.ndarray:
    """n thin random cylinders (vessel-like), centre-voxel test, additive.
    Axes are uniform on the sphere; centres uniform in the ball of radius
    centre_ball (default 0.75 W) about the grid centre."""
    half_w = 0.5 * ap.ms * ap.dxy
    if centre_ball is None:
        centre_ball = 0.75 * half_w
    cx, cz = voxel_centres(ap)
    vol = np.zeros(ap.vol_shape)
    rad = rng.uniform(*r_range, size=n)
    length = rng.uniform(*len_range, size=n)
    axis = rng.standard_normal((n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    direc = rng.standard_normal((n, 3))
    direc /= np.linalg.norm(direc, axis=1, keepdims=True)
    cen = direc * (centre_ball * rng.uniform(0, 1, size=n) ** (1.0 / 3.0))[:, None]
    for e in range(n):
        ext = 0.5 * length[e] * np.abs(axis[e]) + rad[e] * np.sqrt(np.clip(1 - axis[e] ** 2, 0, 1))
        (i0, i1), (j0, j1), (k0, k1) = _box(ap, cen[e] - ext, cen[e] + ext)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        Z, Y, X = np.meshgrid(cz[k0:k1], cx[j0:j1], cx[i0:i1], indexing="ij")
        d = np.stack([X - cen[e, 0], Y - cen[e, 1], Z - cen[e, 2]], -1)
        t = d @ axis[e]
        perp2 = (d * d).sum(-1) - t * t
        inside = (np.abs(t) <= 0.5 * length[e]) & (perp2 <= rad[e] ** 2)
        vol[k0:k1, j0:j1, i0:i1] += amp * inside
    return vol


def phantom(ap: Aperture) -> np.ndarray:
    """The seeded phantom of a named workload (float64, [z][y][x]): three
    balls on the 32^3 grid, ellipsoids plus noise on the 128^3 grid and the
    serving grids, thin cylinders at PACT scale."""
    if ap.name == "grid32":
        return voxelize_balls(ap, balls_params(np.random.default_rng(1001)))
    if ap.name == "grid128":
        return ellipsoid_phantom(ap, np.random.default_rng(1002),
                                 noise_rng=np.random.default_rng(2002))
    if ap.name.startswith("serve"):
        return ellipsoid_phantom(ap, np.random.default_rng(1005),
                                 noise_rng=np.random.default_rng(2005))
    if ap.name == "pact256":
        return cylinder_phantom(ap, np.random.default_rng(1003))
    raise KeyError(ap.name)


def batch_phantoms(ap: Aperture, n: int, seed0: int = 4000) -> np.ndarray:
    """n independent ellipsoid phantoms (seed seed0 + i for volume i)."""
    return np.stack([ellipsoid_phantom(ap, np.random.default_rng(seed0 + i),
                                       noise_rng=np.random.default_rng(seed0 + 100 + i))
                     for i in range(n)])


def gaussian_data(ap: Aperture, rng: np.random.Generator, batch: int | None = None) -> np.ndarray:
    """N(0,1) sensor data of shape [angle][height][radius] (optionally batched)."""
    shape = ap.data_shape if batch is None else (batch,) + ap.data_shape
    return rng.standard_normal(shape)
