"""The two CRT matrices for a piecewise-linear voxel basis (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3.1 discretises f on a piecewise-constant voxel basis and notes that the
algorithms carry over to other bases, piecewise-linear ones among them. The
readings taken here:

  * f(x, y, z) = sum_v F_v L_i(x) L_j(y) L_k(z): tent functions centred on the
    voxel centres (x0 + (i + 1/2) h, ...), each of half-width one pitch
    (so f is trilinear between voxel centres and falls to zero half a voxel
    outside the grid);
  * stage 1 (circle transform in a slice) integrates the bilinear
    interpolant: A12[l, (i, j)] = integral over the circle of L_i(x) L_j(y)
    (measure rho dphi); the z dependence stays the coefficient of L_k(z);
  * stage 2 represents f12(z, rho) by tents in z (the same L_k) times tents
    in rho centred on the radii (or on the stage-2 radial grid when the
    aperture has one), with a node of value zero at rho = 0 (the circle
    transform vanishes there) and one past the last radius at the last
    spacing: A34[(h, l), (l', k)] = integral over the upper half circle
    about (z_h, 0) of L_k(z) T_l'(rho) (measure l dtheta).

Each arc is cut at the lines through the nodes, where the interpolant's
pieces change, and at its extremes in x and y; on each piece the four corner weights are integrated by
composite Gauss-Legendre quadrature (the integrand is smooth on a piece).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import TWO_PI

_GL_X, _GL_W = np.polynomial.legendre.leggauss(12)


def node_edges(x0: float, pitch: float, n: int) -> np.ndarray:
    """Positions of the n voxel-centre nodes plus one virtual node (value
    zero) half a voxel outside each end: the breakpoints of the tents."""
    return x0 + pitch * (np.arange(-1, n + 1, dtype=np.float64) + 0.5)


def rho_nodes(radii) -> np.ndarray:
    """rho nodes of stage 2: 0, the radii, and one spacing past the last."""
    r = np.asarray(radii, dtype=np.float64)
    last = r[-1] + (r[-1] - r[-2] if r.size > 1 else r[-1])
    return np.concatenate([[0.0], r, [last]])


def _crossings(c, r, edges):
    """Angles in [0, 2 pi) where c + r cos t (or sin, see caller) meets edges."""
    u = (edges - c) / r
    return u[np.abs(u) < 1.0]


def arc_corner_weights(cx, cy, r, xe, ye, t_end=TWO_PI, max_step=0.05):
    """Integrals over the arc {(cx + r cos t, cy + r sin t): 0 <= t <= t_end}
    (measure r dt) of the bilinear tents on the node lattice xe x ye.
    Returns (node_x, node_y, weight) with node indices into xe / ye
    (duplicates not merged); nodes 0 and len-1 are the virtual ones."""
    a = np.arccos(_crossings(cx, r, xe))
    b = np.arcsin(_crossings(cy, r, ye))
    # the extremes of x and y are cuts too, so that every piece is monotone in
    # both coordinates and its midpoint lies strictly inside one lattice cell
    # (an arc tangent to a node line would otherwise tie at its midpoint)
    extremes = 0.5 * np.pi * np.arange(5)
    t = np.concatenate([[0.0, t_end], extremes, a, TWO_PI - a, np.mod(b, TWO_PI), np.pi - b])
    t = np.unique(t[(t >= 0.0) & (t <= t_end)])
    out_i, out_j, out_w = [], [], []
    for t0, t1 in zip(t[:-1], t[1:]):
        if t1 <= t0:
            continue
        tm = 0.5 * (t0 + t1)
        xm, ym = cx + r * np.cos(tm), cy + r * np.sin(tm)
        ci = np.searchsorted(xe, xm, side="right") - 1  # cell between nodes ci, ci+1
        cj = np.searchsorted(ye, ym, side="right") - 1
        if ci < 0 or ci >= xe.size - 1 or cj < 0 or cj >= ye.size - 1:
            continue
        # composite Gauss-Legendre on [t0, t1]
        m = max(1, int(np.ceil((t1 - t0) / max_step)))
        edges = np.linspace(t0, t1, m + 1)
        ts = (0.5 * (edges[:-1] + edges[1:])[:, None]
              + 0.5 * (edges[1:] - edges[:-1])[:, None] * _GL_X[None, :]).ravel()
        ws = (0.5 * (edges[1:] - edges[:-1])[:, None] * _GL_W[None, :]).ravel() * r
        u = (cx + r * np.cos(ts) - xe[ci]) / (xe[ci + 1] - xe[ci])
        v = (cy + r * np.sin(ts) - ye[cj]) / (ye[cj + 1] - ye[cj])
        for di, dj, f in ((0, 0, (1 - u) * (1 - v)), (1, 0, u * (1 - v)),
                          (0, 1, (1 - u) * v), (1, 1, u * v)):
            out_i.append(ci + di)
            out_j.append(cj + dj)
            out_w.append(float(np.dot(ws, f)))
    return np.array(out_i, int), np.array(out_j, int), np.array(out_w)


def a12_row(ap, center, radius: float):
    """Row of the linear-basis A12: (pixel-node indices j*M_s + i, weights)."""
    xe = node_edges(ap.x0, ap.dxy, ap.ms)
    ni, nj, w = arc_corner_weights(center[0], center[1], radius, xe, xe, TWO_PI)
    ok = (ni >= 1) & (ni <= ap.ms) & (nj >= 1) & (nj <= ap.ms)  # drop virtual nodes
    p = (nj[ok] - 1) * ap.ms + (ni[ok] - 1)
    cols, inv = np.unique(p, return_inverse=True)
    return cols, np.bincount(inv, weights=w[ok], minlength=cols.size)


def assemble_a12_at(ap, c) -> sp.csr_matrix:
    """Linear-basis A12 for the column through (x, y) = c (N_l x M_s^2)."""
    ri, ci, vi = [], [], []
    rho = ap.rho_grid
    for l in range(rho.size):
        cols, w = a12_row(ap, c, rho[l])
        ri.append(np.full(cols.size, l))
        ci.append(cols)
        vi.append(w)
    ri, ci, vi = (np.concatenate(x) for x in (ri, ci, vi))
    return sp.csr_matrix((vi, (ri.astype(np.int64), ci.astype(np.int64))),
                         shape=(rho.size, ap.ms * ap.ms))


def a34_row(ap, zc: float, radius: float):
    """Row of the linear-basis A34: (cols l' * M_z + k, weights)."""
    ze = node_edges(ap.z0, ap.dz, ap.mz)
    re = rho_nodes(ap.rho_grid)
    nk, nl, w = arc_corner_weights(zc, 0.0, radius, ze, re, np.pi)
    ok = (nk >= 1) & (nk <= ap.mz) & (nl >= 1) & (nl <= ap.n_rho)
    col = (nl[ok] - 1) * ap.mz + (nk[ok] - 1)
    cols, inv = np.unique(col, return_inverse=True)
    return cols, np.bincount(inv, weights=w[ok], minlength=cols.size)


def assemble_a34(ap, heights=None) -> sp.csr_matrix:
    heights = range(ap.n_z) if heights is None else heights
    ri, ci, vi = [], [], []
    for h in heights:
        for l in range(ap.n_radii):
            cols, w = a34_row(ap, ap.zpos[h], ap.radii[l])
            ri.append(np.full(cols.size, h * ap.n_radii + l))
            ci.append(cols)
            vi.append(w)
    ri, ci, vi = (np.concatenate(x) for x in (ri, ci, vi))
    return sp.csr_matrix((vi, (ri.astype(np.int64), ci.astype(np.int64))),
                         shape=(ap.n_z * ap.n_radii, ap.n_rho * ap.mz))


def assemble_all(ap):
    """All per-column linear-basis A12 matrices and the shared A34."""
    return [assemble_a12_at(ap, c) for c in ap.column_centers], assemble_a34(ap)
