"""Assembly of the two CRT matrices of the cylindrical-aperture SRT (FP64).

Sec. 2 writes the SRT at centre (r1, r2, r3) and radius l as a half-circle
integral, over theta in [0, pi] with measure l dtheta, of f12(r1, r2, z, rho):
the integral of f over the circle of radius rho about (r1, r2) in the plane at
height z, with measure rho dphi. Sec. 3.1 takes f piecewise constant per voxel
and turns each CRT into a sparse matrix (Alg. 1 inputs):

  A12[l, p]           length of the circle |x - c| = l_l inside pixel p
                      (one matrix per sensor column c, N_l x M_s^2);
  A34[(h,l), (l',k)]  length of the half circle (z - z_h)^2 + rho^2 = l_l^2,
                      rho >= 0, inside the (rho, z) cell (l', k)
                      (one matrix shared by all columns, N_h N_l x N_l M_z).

Weights are exact arc lengths (radius times angle), computed from the sorted
angles at which the circle crosses the cell edges or reaches an extreme in x
or y: between two consecutive such angles the arc stays inside one cell,
found from the arc's mid-angle.

Readings of points the paper leaves open:
  * pixel index p = j * M_s + i (i along x); voxel k along z;
  * the rho axis of the stage-2 image reuses the N_l radii: cell l' spans the
    midpoints between neighbouring radii, the outer edges being half a
    spacing beyond the first and last radius (for l_l = l dl the cells are
    [(l'-1/2) dl, (l'+1/2) dl]);
  * that axis may also be a grid of its own, rho_0 < ... < rho_{N_rho - 1}
    (ap.rho_grid): stage 1 then evaluates the circle transform at the rho_m
    (A12 is N_rho x M_s^2) and the cells are built from the rho_m in the same
    way (A34 is N_h N_l x N_rho M_z); without one, rho_m = l_m;
  * row (h, l) of A34 has index h N_l + l, column (l', k) has index l' M_z + k;
  * pieces of zero length are dropped; several pieces of one circle in one
    cell are summed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TWO_PI = 2.0 * np.pi


def grid_edges(x0: float, pitch: float, n: int) -> np.ndarray:
    """The n + 1 cell edges x0 + i * pitch of a uniform axis."""
    return x0 + pitch * np.arange(n + 1, dtype=np.float64)


def rho_edges(radii) -> np.ndarray:
    """Edges of the radial cells of the stage-2 image: midpoints between
    consecutive radii, outer edges half a spacing beyond the end radii."""
    r = np.asarray(radii, dtype=np.float64)
    if r.size == 1:
        return np.array([0.5 * r[0], 1.5 * r[0]])
    mid = 0.5 * (r[1:] + r[:-1])
    return np.concatenate([[r[0] - 0.5 * (r[1] - r[0])], mid,
                           [r[-1] + 0.5 * (r[-1] - r[-2])]])


def arc_pieces(cx: float, cy: float, r: float, xe: np.ndarray, ye: np.ndarray,
               t_end: float = TWO_PI):
    """Pieces of the arc {(cx + r cos t, cy + r sin t) : 0 <= t <= t_end} inside
    the rectangle grid with column edges xe and row edges ye.

    Returns (ix, iy, length): cell column, cell row and arc length of every
    piece whose mid-angle point lies inside the grid (duplicates not merged).
    """
    # the arc's extremes in x and y are cuts as well: every piece is then
    # monotone in both coordinates, and its mid-angle point lies strictly
    # inside one cell even where the arc touches a cell edge tangentially
    ts = [np.array([0.0, t_end]), 0.5 * np.pi * np.arange(5)]
    u = (xe - cx) / r
    u = u[np.abs(u) < 1.0]
    a = np.arccos(u)  # crossings with x = const: cos t = u
    ts += [a, TWO_PI - a]
    v = (ye - cy) / r
    v = v[np.abs(v) < 1.0]
    b = np.arcsin(v)  # crossings with y = const: sin t = v
    ts += [np.mod(b, TWO_PI), np.pi - b]
    t = np.concatenate(ts)
    t = np.unique(t[(t >= 0.0) & (t <= t_end)])  # sorted, distinct
    t0, t1 = t[:-1], t[1:]
    tm = 0.5 * (t0 + t1)
    xm = cx + r * np.cos(tm)
    ym = cy + r * np.sin(tm)
    ix = np.searchsorted(xe, xm, side="right") - 1
    iy = np.searchsorted(ye, ym, side="right") - 1
    ok = (ix >= 0) & (ix < xe.size - 1) & (iy >= 0) & (iy < ye.size - 1) & (t1 > t0)
    return ix[ok], iy[ok], r * (t1 - t0)[ok]


def a12_row(ap, center, radius: float):
    """Row of A12 for one circle: (pixel indices, arc lengths), duplicates summed."""
    xe = grid_edges(ap.x0, ap.dxy, ap.ms)
    ix, iy, w = arc_pieces(center[0], center[1], radius, xe, xe, TWO_PI)
    p = iy * ap.ms + ix
    cols, inv = np.unique(p, return_inverse=True)
    return cols, np.bincount(inv, weights=w, minlength=cols.size)


def assemble_a12(ap, angle: float, rows=None) -> sp.csr_matrix:
    """A12 for the sensor column at angle `angle` on the cylinder (Alg. 1
    input, N_rho x M_s^2). `rows` restricts assembly to a subset of radius
    indices (others empty)."""
    return assemble_a12_at(ap, (ap.radius * np.cos(angle), ap.radius * np.sin(angle)), rows)


def assemble_a12_at(ap, c, rows=None) -> sp.csr_matrix:
    """A12 for the sensor column through (x, y) = c: Sec. 2 only needs the
    sensors of a group on one line parallel to z, wherever that line is."""
    rho = ap.rho_grid
    rows = range(rho.size) if rows is None else rows
    ri, ci, vi = [], [], []
    for l in rows:
        cols, w = a12_row(ap, c, rho[l])
        ri.append(np.full(cols.size, l))
        ci.append(cols)
        vi.append(w)
    ri, ci, vi = (np.concatenate(x) if x else np.zeros(0) for x in (ri, ci, vi))
    return sp.csr_matrix((vi, (ri.astype(np.int64), ci.astype(np.int64))),
                         shape=(rho.size, ap.ms * ap.ms))


def a34_row(ap, zc: float, radius: float):
    """Row of A34 for one half circle centred (z = zc, rho = 0): (cols, lengths)."""
    ze = grid_edges(ap.z0, ap.dz, ap.mz)
    re = rho_edges(ap.rho_grid)
    ik, il, w = arc_pieces(zc, 0.0, radius, ze, re, np.pi)
    col = il * ap.mz + ik
    cols, inv = np.unique(col, return_inverse=True)
    return cols, np.bincount(inv, weights=w, minlength=cols.size)


def assemble_a34(ap, heights=None) -> sp.csr_matrix:
    """A34 (Alg. 1 input, N_h N_l x N_rho M_z), shared by every sensor column.
    `heights` restricts assembly to a subset of sensor-height indices."""
    heights = range(ap.n_z) if heights is None else heights
    ri, ci, vi = [], [], []
    for h in heights:
        for l in range(ap.n_radii):
            cols, w = a34_row(ap, ap.zpos[h], ap.radii[l])
            ri.append(np.full(cols.size, h * ap.n_radii + l))
            ci.append(cols)
            vi.append(w)
    ri, ci, vi = (np.concatenate(x) if x else np.zeros(0) for x in (ri, ci, vi))
    return sp.csr_matrix((vi, (ri.astype(np.int64), ci.astype(np.int64))),
                         shape=(ap.n_z * ap.n_radii, ap.n_rho * ap.mz))


def assemble_all(ap):
    """All per-column A12 matrices and the shared A34."""
    if getattr(ap, "centers", None) is not None:
        return [assemble_a12_at(ap, c) for c in ap.column_centers], assemble_a34(ap)
    return [assemble_a12(ap, a) for a in ap.angles], assemble_a34(ap)
