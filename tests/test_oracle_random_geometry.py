"""Pins of the oracle on the seeded random geometries that the GPU parity
sweep uses (srt_inputs.random_aperture): grids that are not centred, voxels
that are not cubes, columns inside and outside the grid, uneven heights and
radii, and stage-2 radial grids of their own.

Rows of A12 and A34 are checked against point sampling of the circles, which
shares nothing with the assembly but the cell edges:
  * constant basis: each sample is binned into the cell that holds it; an
    entry may differ from the exact arc length by one sample spacing per
    piece of arc in the cell, at most 4 pieces;
  * linear basis: each sample is spread over the corners of its lattice cell
    with bilinear weights (the tents' values there), bound 8 spacings.
The adjoint is checked by the dot test on the same geometries.
"""
import numpy as np
import pytest

from oracle import brute, geometry as geo, linear as lin, srt
from srt_inputs import random_aperture
from test_oracle_linear import _sampled_lattice, _sampled_row

N = 1 << 17
SEEDS = (0, 3, 5, 9, 13, 14, 19, 26)


def _columns(ap):
    return sorted({0, ap.n_angles - 1})


@pytest.mark.parametrize("seed", SEEDS)
def test_constant_rows_match_sampling(seed):
    ap = random_aperture(seed)
    a12s, a34 = geo.assemble_all(ap)
    for a in _columns(ap):
        A = a12s[a].toarray()
        c = ap.column_centers[a]
        for m, r in enumerate(ap.rho_grid):
            bf = brute.sampled_a12_row(ap, c, r, N)
            assert np.abs(bf - A[m]).max() <= 4 * r * 2 * np.pi / N, (a, m)
    a34 = a34.toarray()
    for h, zh in enumerate(ap.zpos):
        for l, r in enumerate(ap.radii):
            bf = brute.sampled_a34_row(ap, zh, r, N)
            assert np.abs(bf - a34[h * ap.n_radii + l]).max() <= 4 * r * np.pi / N, (h, l)


@pytest.mark.parametrize("seed", SEEDS)
def test_linear_rows_match_bilinear_sampling(seed):
    ap = random_aperture(seed)
    a12s, a34 = lin.assemble_all(ap)
    for a in _columns(ap):
        A = a12s[a].toarray()
        c = ap.column_centers[a]
        for m, r in enumerate(ap.rho_grid):
            bf = _sampled_row(ap, c, r, N)
            assert np.abs(bf - A[m]).max() <= 8 * r * 2 * np.pi / N, (a, m)
    ze = lin.node_edges(ap.z0, ap.dz, ap.mz)
    re = lin.rho_nodes(ap.rho_grid)
    a34 = a34.toarray()
    for h, zh in enumerate(ap.zpos):
        for l, r in enumerate(ap.radii):
            full = _sampled_lattice(zh, 0.0, r, ze, re, np.pi, N)
            bf = full[1:-1, 1:-1].reshape(-1)  # [rho node][k], virtual nodes dropped
            assert np.abs(bf - a34[h * ap.n_radii + l]).max() <= 8 * r * np.pi / N, (h, l)


@pytest.mark.parametrize("basis", ["constant", "linear"])
def test_dot_product_on_random_geometries(basis):
    mod = geo if basis == "constant" else lin
    for seed in range(8):
        ap = random_aperture(seed)
        a12s, a34 = mod.assemble_all(ap)
        rng = np.random.default_rng(seed)
        f = rng.standard_normal(ap.vol_shape)
        g = rng.standard_normal(ap.data_shape)
        Af = srt.forward(f, a12s, a34, ap.n_z, ap.n_radii)
        Atg = srt.adjoint(g, a12s, a34, ap.ms, ap.mz)
        scale = max(np.linalg.norm(Af) * np.linalg.norm(g), 1e-300)
        assert abs(np.vdot(Af, g) - np.vdot(f, Atg)) <= 1e-13 * scale, seed
