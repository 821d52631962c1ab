"""Pins of the piecewise-linear-basis operators (oracle/linear.py) against
things other than themselves:

  * exactness on linear data: the bilinear interpolant of a linear function
    is the function itself, so the circle transform of nodal samples of
    a x + b y + c equals 2 pi r (a cx + b cy + c) for circles inside the
    node hull; stage 2 is exact for (a z + b) rho, whose half-circle
    transform is 2 l^2 (a z_h + b);
  * partition of unity: a row's weights sum to the circle's length when it
    lies inside the node hull;
  * point sampling with bilinear weights (brute force) agrees entry by entry
    within the sampling error;
  * end to end, a linear volume has sphere integrals 4 pi l^2 f(sensor)
    (mean value over a sphere) for spheres inside the node hull, which pins
    the hand-over from stage 1 to stage 2 (rho nodes, zero at rho = 0);
  * the composed operator is the constant-basis algorithm's structure: its
    adjoint is the transpose (dot test).
"""
import numpy as np
import pytest

from oracle import linear as lin, srt
from srt_inputs import column_aperture, cylinder_aperture


def _ap():
    return cylinder_aperture("lin", 12, 1.0, 1.4, 6, 5, 24, mz=10)


def _inside_hull(ap, c, r):
    """Circle about c of radius r inside [x_0, x_{M-1}]^2 (the node hull)."""
    lo, hi = ap.x0 + ap.dxy / 2, ap.x0 + (ap.ms - 0.5) * ap.dxy
    return c[0] - r >= lo and c[0] + r <= hi and c[1] - r >= lo and c[1] + r <= hi


def test_stage1_exact_on_linear_data():
    ap = _ap()
    xs = ap.x0 + (np.arange(ap.ms) + 0.5) * ap.dxy
    X, Y = np.meshgrid(xs, xs)  # [j][i]
    a, b, c = 0.7, -1.3, 0.4
    F = (a * X + b * Y + c).reshape(-1)
    checked = 0
    for center in [(0.05, -0.1), (0.3, 0.2)]:
        Gl = lin.assemble_a12_at(ap, center) @ F
        for l, r in enumerate(ap.radii):
            if _inside_hull(ap, center, r):
                ref = 2 * np.pi * r * (a * center[0] + b * center[1] + c)
                assert abs(Gl[l] - ref) <= 1e-12 * max(1.0, abs(ref)), (center, l)
                checked += 1
    assert checked >= 8


def test_stage2_exact_on_linear_data():
    ap = _ap()
    zs = ap.z0 + (np.arange(ap.mz) + 0.5) * ap.dz
    a, b = 0.8, 0.3
    G = np.outer(ap.radii, a * zs + b)  # [l'][k] = (a z_k + b) rho_l'
    A34 = lin.assemble_a34(ap)
    Y = (A34 @ G.reshape(-1)).reshape(ap.n_z, ap.n_radii)
    checked = 0
    for h, zh in enumerate(ap.zpos):
        for l, r in enumerate(ap.radii):
            if zh - r >= zs[0] and zh + r <= zs[-1]:
                ref = 2 * r * r * (a * zh + b)
                assert abs(Y[h, l] - ref) <= 1e-12 * max(1.0, abs(ref)), (h, l)
                checked += 1
    assert checked >= 8


def test_rows_are_partitions_of_unity():
    ap = _ap()
    A = lin.assemble_a12_at(ap, (0.1, 0.05))
    sums = np.asarray(A.sum(axis=1)).ravel()
    checked = 0
    for l, r in enumerate(ap.radii):
        if _inside_hull(ap, (0.1, 0.05), r):
            assert abs(sums[l] - 2 * np.pi * r) <= 1e-12 * r
            checked += 1
    assert checked >= 4


def _sampled_lattice(cx, cy, r, xe, ye, t_end, n):
    """Brute force: n midpoint samples of the arc, each spread over the four
    corners of its lattice cell with bilinear weights. Returns the full
    (len(ye) x len(xe)) node array, virtual nodes included."""
    t = t_end * (np.arange(n) + 0.5) / n
    x, y = cx + r * np.cos(t), cy + r * np.sin(t)
    i = np.searchsorted(xe, x, side="right") - 1
    j = np.searchsorted(ye, y, side="right") - 1
    ok = (i >= 0) & (i < xe.size - 1) & (j >= 0) & (j < ye.size - 1)
    i, j, x, y = i[ok], j[ok], x[ok], y[ok]
    u = (x - xe[i]) / (xe[i + 1] - xe[i])
    v = (y - ye[j]) / (ye[j + 1] - ye[j])
    ds = r * t_end / n
    out = np.zeros(ye.size * xe.size)
    for di, dj, w in ((0, 0, (1 - u) * (1 - v)), (1, 0, u * (1 - v)), (0, 1, (1 - u) * v), (1, 1, u * v)):
        np.add.at(out, (j + dj) * xe.size + (i + di), w * ds)
    return out.reshape(ye.size, xe.size)


def _sampled_row(ap, center, r, n):
    xe = lin.node_edges(ap.x0, ap.dxy, ap.ms)
    full = _sampled_lattice(center[0], center[1], r, xe, xe, 2 * np.pi, n)
    return full[1:-1, 1:-1].reshape(-1)  # drop virtual nodes


@pytest.mark.parametrize("center", [(0.13, -0.41), (1.5, 0.2), (-0.5, -0.5)])
def test_stage1_matches_bilinear_sampling(center):
    ap = column_aperture("s", 8, 1.0, [center], 2, 12, l_max=3.0)
    A = lin.assemble_a12_at(ap, center).toarray()
    n = 1 << 19
    for l, r in enumerate(ap.radii):
        bf = _sampled_row(ap, center, r, n)
        assert np.abs(bf - A[l]).max() <= 8 * r * 2 * np.pi / n, l


def test_stage2_matches_bilinear_sampling():
    ap = cylinder_aperture("s2", 8, 1.0, 1.4, 4, 9, 10, mz=8)
    ze = lin.node_edges(ap.z0, ap.dz, ap.mz)
    re = lin.rho_nodes(ap.radii)
    A = lin.assemble_a34(ap).toarray()
    n = 1 << 19
    for h, zh in enumerate(ap.zpos):
        for l, r in enumerate(ap.radii):
            full = _sampled_lattice(zh, 0.0, r, ze, re, np.pi, n)
            bf = full[1:-1, 1:-1].reshape(-1)  # [l'][k], virtual nodes dropped
            assert np.abs(bf - A[h * ap.n_radii + l]).max() <= 8 * r * np.pi / n, (h, l)


def linear_volume(ap, coef):
    """Nodal values a x + b y + c z + d at the voxel centres, [k][j][i]."""
    a, b, c, d = coef
    xs = ap.x0 + (np.arange(ap.ms) + 0.5) * ap.dxy
    zs = ap.z0 + (np.arange(ap.mz) + 0.5) * ap.dz
    return (a * xs[None, None, :] + b * xs[None, :, None] + c * zs[:, None, None] + d)


def spheres_inside_hull(ap):
    """(a, h, l) of spheres that lie inside the node hull, with radii[l]
    circles about the column inside the xy hull as well."""
    lo, hi = ap.x0 + ap.dxy / 2, ap.x0 + (ap.ms - 0.5) * ap.dxy
    zlo, zhi = ap.z0 + ap.dz / 2, ap.z0 + (ap.mz - 0.5) * ap.dz
    out = []
    for a, (cx, cy) in enumerate(ap.column_centers):
        for h, zh in enumerate(ap.zpos):
            for l, r in enumerate(ap.radii):
                if (cx - r >= lo and cx + r <= hi and cy - r >= lo and cy + r <= hi
                        and zh - r >= zlo and zh + r <= zhi):
                    out.append((a, h, l))
    return out


def test_composed_exact_on_linear_volume():
    ap = column_aperture("ex", 16, 1.0, [(0.1, -0.05), (-0.15, 0.2)], 9, 24, l_max=1.2)
    coef = (0.6, -0.9, 1.1, 0.35)
    a12s, a34 = lin.assemble_all(ap)
    Y = srt.forward(linear_volume(ap, coef), a12s, a34, ap.n_z, ap.n_radii)
    cases = spheres_inside_hull(ap)
    assert len(cases) >= 20
    for a, h, l in cases:
        cx, cy = ap.column_centers[a]
        r = ap.radii[l]
        ref = 4 * np.pi * r * r * (coef[0] * cx + coef[1] * cy + coef[2] * ap.zpos[h] + coef[3])
        assert abs(Y[a, h, l] - ref) <= 1e-12 * max(1.0, abs(ref)), (a, h, l)


def test_linear_basis_dot_product():
    ap = _ap()
    a12s, a34 = lin.assemble_all(ap)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(ap.vol_shape)
    g = rng.standard_normal(ap.data_shape)
    Af = srt.forward(f, a12s, a34, ap.n_z, ap.n_radii)
    Atg = srt.adjoint(g, a12s, a34, ap.ms, ap.mz)
    assert abs(np.vdot(Af, g) - np.vdot(f, Atg)) <= 1e-13 * np.linalg.norm(Af) * np.linalg.norm(g)
