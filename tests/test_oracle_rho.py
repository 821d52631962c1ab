"""Pins of the oracle with a stage-2 radial grid of its own (N_rho != N_l).

The paper ties the rho axis of the stage-2 image to the N_l sphere radii; a
grid of its own changes which circles stage 1 evaluates and which cells
stage 2 integrates over. Checked against things other than the assembly:

  * point sampling of single A12 / A34 rows on uniform and non-uniform grids;
  * Alg. 1 with both transforms done by point sampling (no matrices);
  * convergence: the error against the exact ball transform (spherical cap
    areas) falls as the rho grid is refined;
  * the linear basis stays exact on linear volumes (mean value over spheres)
    on any rho grid;
  * the adjoint is the transpose (dot test), and rho = radii reproduces the
    tied operator exactly.
"""
import dataclasses

import numpy as np
import pytest

from oracle import brute, closed_forms as cf, geometry as geo, linear as lin, srt
from srt_inputs import column_aperture, cylinder_aperture, phantoms, with_rho_grid


def _nonuniform(ap, n):
    """A graded grid: dense at small radii, sparse at large ones."""
    u = np.arange(1, n + 1) / n
    return dataclasses.replace(ap, name=ap.name + "_graded", rho=ap.radii[-1] * u ** 1.5)


def test_rho_equal_to_radii_reproduces_tied_operator():
    ap = cylinder_aperture("t", 12, 1.0, 1.5, 4, 5, 24, l_max=3.5)
    tied = geo.assemble_all(ap)
    own = geo.assemble_all(dataclasses.replace(ap, rho=ap.radii.copy()))
    for A, B in zip(tied[0] + [tied[1]], own[0] + [own[1]]):
        assert A.shape == B.shape and abs(A - B).max() == 0.0


@pytest.mark.parametrize("kind", ["coarse", "fine", "graded"])
def test_rows_match_sampling_on_own_rho_grid(kind):
    ap0 = cylinder_aperture("t", 8, 1.0, 1.2, 3, 5, 16, l_max=3.0)
    ap = {"coarse": lambda: with_rho_grid(ap0, 7), "fine": lambda: with_rho_grid(ap0, 37),
          "graded": lambda: _nonuniform(ap0, 21)}[kind]()
    a12s, a34 = geo.assemble_all(ap)
    assert a12s[0].shape == (ap.n_rho, ap.ms ** 2)
    assert a34.shape == (ap.n_z * ap.n_radii, ap.n_rho * ap.mz)
    n = 1 << 20
    A = a12s[1].toarray()
    c = ap.column_centers[1]
    for m, r in enumerate(ap.rho_grid):
        bf = brute.sampled_a12_row(ap, c, r, n)
        assert np.abs(bf - A[m]).max() <= 4 * r * 2 * np.pi / n, m
    a34 = a34.toarray()
    for h in range(ap.n_z):
        for l, r in enumerate(ap.radii):
            bf = brute.sampled_a34_row(ap, ap.zpos[h], r, n)
            assert np.abs(bf - a34[h * ap.n_radii + l]).max() <= 4 * r * np.pi / n, (h, l)


def test_rows_match_sampling_for_graded_radii():
    """Non-uniform sensor radii with the tied grid: uneven midpoint cells."""
    ap0 = cylinder_aperture("t", 8, 1.0, 1.2, 3, 4, 15, l_max=3.0)
    u = np.arange(1, 16) / 15
    ap = dataclasses.replace(ap0, radii=3.0 * u ** 1.7)
    a12s, a34 = geo.assemble_all(ap)
    n = 1 << 20
    A, c = a12s[2].toarray(), ap.column_centers[2]
    for m, r in enumerate(ap.radii):
        assert np.abs(brute.sampled_a12_row(ap, c, r, n) - A[m]).max() <= 4 * r * 2 * np.pi / n
    a34 = a34.toarray()
    for h in range(ap.n_z):
        for l, r in enumerate(ap.radii):
            bf = brute.sampled_a34_row(ap, ap.zpos[h], r, n)
            assert np.abs(bf - a34[h * ap.n_radii + l]).max() <= 4 * r * np.pi / n, (h, l)


def test_matches_sampled_discrete_operator_on_own_rho_grid():
    ap = _nonuniform(cylinder_aperture("t", 12, 1.0, 1.5, 4, 5, 24, l_max=3.5), 17)
    a12s, a34 = geo.assemble_all(ap)
    F = np.random.default_rng(5).uniform(0, 1, ap.vol_shape)
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    Yb = brute.sampled_forward(F, ap, 100_000, 100_000)
    assert np.linalg.norm(Y - Yb) / np.linalg.norm(Y) <= 1e-4


def test_ball_error_falls_as_rho_grid_refines():
    """Against the exact SRT of three balls at 32^3 with 64 radii: a coarse
    rho grid costs accuracy, refining it recovers the tied grid's error."""
    ap0 = cylinder_aperture("t", 32, 1.0, 1.5, 8, 8, 64, l_max=3.5)
    balls = phantoms.balls_params(np.random.default_rng(1001))
    F = phantoms.voxelize_balls(ap0, balls)
    ex = cf.srt_of_balls(ap0, balls)
    errs = []
    for n_rho in (16, 32, 64, 128):
        ap = with_rho_grid(ap0, n_rho)
        a12s, a34 = geo.assemble_all(ap)
        Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
        errs.append(np.linalg.norm(Y - ex) / np.linalg.norm(ex))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[0] >= 4 * errs[2]
    assert errs[3] <= 6.5e-2


def test_linear_basis_exact_on_linear_volume_with_own_rho_grid():
    ap0 = column_aperture("ex", 16, 1.0, [(0.1, -0.05), (-0.15, 0.2)], 9, 24, l_max=1.2)
    ap = dataclasses.replace(ap0, rho=1.25 * (np.arange(1, 12) / 11) ** 1.3)
    coef = (0.6, -0.9, 1.1, 0.35)
    xs = ap.x0 + (np.arange(ap.ms) + 0.5) * ap.dxy
    zs = ap.z0 + (np.arange(ap.mz) + 0.5) * ap.dz
    F = coef[0] * xs[None, None, :] + coef[1] * xs[None, :, None] + coef[2] * zs[:, None, None] \
        + coef[3]
    a12s, a34 = lin.assemble_all(ap)
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    lo, hi = ap.x0 + ap.dxy / 2, ap.x0 + (ap.ms - 0.5) * ap.dxy
    n = 0
    for a, (cx, cy) in enumerate(ap.column_centers):
        for h, zh in enumerate(ap.zpos):
            for l, r in enumerate(ap.radii):
                # the rho nodes bracketing [0, r] must see circles inside the hull
                top = ap.rho_grid[np.searchsorted(ap.rho_grid, r)]
                if (cx - top >= lo and cx + top <= hi and cy - top >= lo and cy + top <= hi
                        and zh - r >= zs[0] and zh + r <= zs[-1]):
                    ref = 4 * np.pi * r * r * (coef[0] * cx + coef[1] * cy + coef[2] * zh
                                               + coef[3])
                    assert abs(Y[a, h, l] - ref) <= 1e-12 * max(1.0, abs(ref)), (a, h, l)
                    n += 1
    assert n >= 20


@pytest.mark.parametrize("basis", ["constant", "linear"])
def test_dot_product_on_own_rho_grid(basis):
    mod = geo if basis == "constant" else lin
    ap = _nonuniform(cylinder_aperture("t", 10, 1.0, 1.4, 5, 4, 18, l_max=3.0), 13)
    a12s, a34 = mod.assemble_all(ap)
    rng = np.random.default_rng(8)
    f = rng.standard_normal(ap.vol_shape)
    g = rng.standard_normal(ap.data_shape)
    Af = srt.forward(f, a12s, a34, ap.n_z, ap.n_radii)
    Atg = srt.adjoint(g, a12s, a34, ap.ms, ap.mz)
    assert abs(np.vdot(Af, g) - np.vdot(f, Atg)) <= 1e-13 * np.linalg.norm(Af) * np.linalg.norm(g)
