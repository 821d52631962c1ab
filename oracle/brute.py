"""Brute-force samplers: independent estimates used to pin the assembly.

* Circle sampling: n equispaced points on an arc, each binned into the cell
  that contains it and weighted by the arc length it represents. A cell's
  sampled weight differs from its exact arc length by less than one sample
  spacing per piece of arc in it.
* Sampled discrete operator: Alg. 1 evaluated with both stages replaced by
  point sampling (circle at each slice height, then half circle over the
  stage-2 image with the same rho cells). No matrices are formed.
* Spherical quadrature of the plain surface integral of Sec. 2 (the
  spherical-coordinate form, measure l^2 sin(theta) dphi dtheta) of the
  voxelised object, to report how far the two-stage method is from the SRT
  of the voxelised object itself.
"""
from __future__ import annotations

import numpy as np

from .geometry import grid_edges, rho_edges

TWO_PI = 2.0 * np.pi


def sampled_arc(cx, cy, r, xe, ye, n, t_end=TWO_PI):
    """Sampled cell weights of one arc: (ix, iy, weight) per sample in the grid."""
    t = t_end * (np.arange(n) + 0.5) / n
    x = cx + r * np.cos(t)
    y = cy + r * np.sin(t)
    ix = np.searchsorted(xe, x, side="right") - 1
    iy = np.searchsorted(ye, y, side="right") - 1
    ok = (ix >= 0) & (ix < xe.size - 1) & (iy >= 0) & (iy < ye.size - 1)
    return ix[ok], iy[ok], np.full(int(ok.sum()), r * t_end / n)


def sampled_a12_row(ap, center, radius, n):
    """Dense sampled row of A12 (length M_s^2)."""
    xe = grid_edges(ap.x0, ap.dxy, ap.ms)
    ix, iy, w = sampled_arc(center[0], center[1], radius, xe, xe, n)
    return np.bincount(iy * ap.ms + ix, weights=w, minlength=ap.ms * ap.ms)


def sampled_a34_row(ap, zc, radius, n):
    """Dense sampled row of A34 (length N_rho M_z)."""
    ze = grid_edges(ap.z0, ap.dz, ap.mz)
    re = rho_edges(ap.rho_grid)
    ik, il, w = sampled_arc(zc, 0.0, radius, ze, re, n, np.pi)
    return np.bincount(il * ap.mz + ik, weights=w, minlength=ap.n_rho * ap.mz)


def sampled_forward(F, ap, n1, n2, angles_idx=None):
    """Alg. 1 with both circular transforms replaced by point sampling.

    Stage 1: for every column a, stage-2 radius rho_l' and slice k, sum F over
    n1 equispaced points of the circle of radius rho_l' about the column
    centre.
    Stage 2: for every height h and radius l, sum the stage-1 image over n2
    equispaced points of the half circle about (z_h, 0), each point taking the
    value of the (rho cell, z slice) that contains it.
    """
    angles_idx = range(ap.n_angles) if angles_idx is None else angles_idx
    xe = grid_edges(ap.x0, ap.dxy, ap.ms)
    ze = grid_edges(ap.z0, ap.dz, ap.mz)
    rgrid = ap.rho_grid
    re = rho_edges(rgrid)
    Fp = F.reshape(ap.mz, -1)  # [k][p]
    out = []
    t2 = np.pi * (np.arange(n2) + 0.5) / n2
    for a in angles_idx:
        cx, cy = ap.column_centers[a]
        G = np.zeros((rgrid.size, ap.mz))
        for lp, rad in enumerate(rgrid):
            ix, iy, w = sampled_arc(cx, cy, rad, xe, xe, n1)
            if ix.size:
                G[lp] = (Fp[:, iy * ap.ms + ix] * w[None, :]).sum(axis=1)
        Y = np.zeros((ap.n_z, ap.n_radii))
        for h, zc in enumerate(ap.zpos):
            z = zc + ap.radii[:, None] * np.cos(t2)[None, :]  # [l][n2]
            rho = ap.radii[:, None] * np.sin(t2)[None, :]
            k = np.searchsorted(ze, z, side="right") - 1
            lp = np.searchsorted(re, rho, side="right") - 1
            ok = (k >= 0) & (k < ap.mz) & (lp >= 0) & (lp < rgrid.size)
            vals = np.where(ok, G[np.clip(lp, 0, rgrid.size - 1), np.clip(k, 0, ap.mz - 1)], 0.0)
            Y[h] = vals.sum(axis=1) * ap.radii * np.pi / n2
        out.append(Y)
    return np.stack(out)


def voxel_lookup(F, ap, x, y, z):
    """Value of the piecewise-constant voxel function at points (0 outside)."""
    i = np.floor((x - ap.x0) / ap.dxy).astype(np.int64)
    j = np.floor((y - ap.x0) / ap.dxy).astype(np.int64)
    k = np.floor((z - ap.z0) / ap.dz).astype(np.int64)
    ok = (i >= 0) & (i < ap.ms) & (j >= 0) & (j < ap.ms) & (k >= 0) & (k < ap.mz)
    return np.where(ok, F[np.clip(k, 0, ap.mz - 1), np.clip(j, 0, ap.ms - 1),
                          np.clip(i, 0, ap.ms - 1)], 0.0)


def spherical_quadrature(F, ap, sensor, radii, n_theta=400, n_phi=800):
    """Surface integral of the voxelised f over spheres about `sensor`
    (Sec. 2, spherical coordinates): Gauss-Legendre in cos(theta) times the
    midpoint rule in phi, measure l^2 sin(theta) dphi dtheta."""
    u, wu = np.polynomial.legendre.leggauss(n_theta)  # u = cos(theta)
    phi = TWO_PI * (np.arange(n_phi) + 0.5) / n_phi
    st = np.sqrt(1.0 - u * u)
    out = np.zeros(len(radii))
    for n, l in enumerate(radii):
        x = sensor[0] + l * st[:, None] * np.cos(phi)[None, :]
        y = sensor[1] + l * st[:, None] * np.sin(phi)[None, :]
        z = sensor[2] + l * u[:, None] * np.ones_like(phi)[None, :]
        f = voxel_lookup(F, ap, x, y, z)
        out[n] = l * l * (wu[:, None] * f).sum() * TWO_PI / n_phi
    return out
