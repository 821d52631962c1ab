"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test fixes one part of the oracle with an independent source: hand
derived exact arcs, brute-force point sampling, closed forms for disks and
balls, the coarea (mass) identity, exact symmetries of the aperture, and the
asymptotic cost stated for Alg. 1. A plausible slip anywhere in the oracle
(a dropped arc-length factor, a wrong sign or index order, a transposed
reshape, a misplaced rho cell) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from srt_inputs import Aperture, config, cylinder_aperture, phantoms
from oracle import brute, closed_forms as cf, geometry as geo, srt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_arcs.json")


def _toy(x0=-1.0, pitch=1.0, m=2, z0=-1.0, dz=1.0, mz=2, radii=(0.5, 1.0)):
    radii = np.asarray(radii, float)
    return Aperture("toy", m, mz, x0, z0, pitch, dz, 0.0, np.zeros(1),
                    np.zeros(1), radii)


def _eval(expr):
    return eval(expr, {"__builtins__": {}}, {"pi": math.pi, "asin": math.asin,
                                             "acos": math.acos, "sqrt": math.sqrt})


@pytest.fixture(scope="module")
def grid32():
    ap = config("grid32")
    a12s, a34 = geo.assemble_all(ap)
    balls = phantoms.balls_params(np.random.default_rng(1001))
    F = phantoms.voxelize_balls(ap, balls)
    return ap, a12s, a34, balls, F


# ---------------------------------------------------------------- exact arcs
def test_golden_exact_arcs():
    """Hand-derived arc lengths (tests/golden/exact_arcs.json)."""
    gold = json.load(open(GOLDEN))
    for case in gold["a12"]:
        ap = _toy(x0=case["x0"], pitch=case["pitch"], m=case["m"])
        cols, w = geo.a12_row(ap, case["center"], case["radius"])
        got = dict(zip(cols.tolist(), w.tolist()))
        exp = {int(k): _eval(v) for k, v in case["expected"].items()}
        assert set(got) == set(exp), case["why"]
        for k in exp:
            assert abs(got[k] - exp[k]) <= 1e-14, case["why"]
    for case in gold["a34"]:
        ap = _toy(z0=case["z0"], dz=case["dz"], mz=case["mz"], radii=case["radii"])
        cols, w = geo.a34_row(ap, case["zc"], case["radius"])
        got = dict(zip(cols.tolist(), w.tolist()))
        exp = {int(k): _eval(v) for k, v in case["expected"].items()}
        assert set(got) == set(exp), case["why"]
        for k in exp:
            assert abs(got[k] - exp[k]) <= 1e-14, case["why"]


def test_rho_edges_midpoints():
    """Uniform radii l*dl give rho cells [(l-1/2)dl, (l+1/2)dl]."""
    dl = 0.37
    e = geo.rho_edges(dl * np.arange(1, 9))
    assert np.allclose(e, dl * (np.arange(9) + 0.5), rtol=0, atol=1e-15)


# ------------------------------------------------------- P1: point sampling
@pytest.mark.parametrize("seed", [0, 1])
def test_a12_entries_match_sampling(seed):
    """Every A12 entry equals the sampled arc length within the sampling
    bound (fewer than 4 sample spacings: at most one per piece)."""
    rng = np.random.default_rng(seed)
    ap = cylinder_aperture("t", 8, 1.0, rng.uniform(0.3, 1.6), 8, 2, 16, l_max=3.2)
    n = 1 << 20
    for a in range(ap.n_angles):
        A = geo.assemble_a12(ap, ap.angles[a]).toarray()
        c = (ap.radius * np.cos(ap.angles[a]), ap.radius * np.sin(ap.angles[a]))
        for l in range(ap.n_radii):
            bf = brute.sampled_a12_row(ap, c, ap.radii[l], n)
            spacing = ap.radii[l] * 2 * np.pi / n
            assert np.abs(bf - A[l]).max() <= 4 * spacing


def test_a12_entries_match_sampling_for_arbitrary_columns():
    """Columns anywhere in the plane (Sec. 2 needs only lines parallel to z):
    inside the grid, on a grid line, on a pixel corner, far outside."""
    from srt_inputs import column_aperture
    centers = [(0.13, -0.41), (0.25, 0.6), (-0.5, -0.5), (2.7, -0.3), (-0.01, 1.9)]
    ap = column_aperture("cols", 8, 1.0, centers, 2, 16, l_max=3.2)
    a12s, _ = geo.assemble_all(ap)
    n = 1 << 20
    for A, c in zip(a12s, centers):
        A = A.toarray()
        for l in range(ap.n_radii):
            bf = brute.sampled_a12_row(ap, c, ap.radii[l], n)
            spacing = ap.radii[l] * 2 * np.pi / n
            assert np.abs(bf - A[l]).max() <= 4 * spacing, (c, l)


def test_a12_entries_match_sampling_for_tangent_circles():
    """Degenerate placements: a column on a voxel-centre line or a grid line,
    with radii that are multiples of the pitch, so that circles touch grid
    lines tangentially with the crossings placed symmetrically about the
    touching point."""
    from srt_inputs import column_aperture
    h = 0.25
    centers = [(h / 2, 0.0), (0.0, h / 2), (h / 2, h / 2), (0.0, 0.0)]
    ap = column_aperture("tan", 8, 1.0, centers, 2, 6, l_max=1.5)
    assert np.allclose(ap.radii / h, np.round(ap.radii / h))
    a12s, _ = geo.assemble_all(ap)
    n = 1 << 20
    for A, c in zip(a12s, centers):
        A = A.toarray()
        for l in range(ap.n_radii):
            bf = brute.sampled_a12_row(ap, c, ap.radii[l], n)
            spacing = ap.radii[l] * 2 * np.pi / n
            assert np.abs(bf - A[l]).max() <= 4 * spacing, (c, l)


def test_a34_entries_match_sampling():
    """Every A34 entry equals the sampled half-circle arc length within the
    sampling bound; rho cells below the first midpoint receive nothing."""
    ap = cylinder_aperture("t", 8, 1.0, 1.2, 1, 5, 16, l_max=3.0)
    a34 = geo.assemble_a34(ap).toarray()
    n = 1 << 20
    for h in range(ap.n_z):
        for l in range(ap.n_radii):
            bf = brute.sampled_a34_row(ap, ap.zpos[h], ap.radii[l], n)
            spacing = ap.radii[l] * np.pi / n
            assert np.abs(bf - a34[h * ap.n_radii + l]).max() <= 4 * spacing


# ------------------------------------------------------ P2/P3: disk closed forms
def _disk_fraction(xe, ye, cx, cy, a, sub=8):
    off = (np.arange(sub) + 0.5) / sub
    xs = (xe[:-1, None] + off[None, :] * np.diff(xe)[:, None]).ravel()
    ys = (ye[:-1, None] + off[None, :] * np.diff(ye)[:, None]).ravel()
    ins = ((xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2) <= a * a
    return ins.reshape(ye.size - 1, sub, xe.size - 1, sub).mean(axis=(1, 3))


def _stage1_disk_error(m, nl):
    ap = cylinder_aperture("t", m, 1.0, 1.5, 4, 2, nl, l_max=3.5, mz=2)
    xe = geo.grid_edges(ap.x0, ap.dxy, ap.ms)
    frac = _disk_fraction(xe, xe, 0.2, -0.1, 0.5)
    F = np.stack([frac, -2.0 * frac])
    errs = []
    for ang in ap.angles:
        G = srt.crt12(geo.assemble_a12(ap, ang), F)
        d = np.hypot(ap.radius * np.cos(ang) - 0.2, ap.radius * np.sin(ang) + 0.1)
        ex = cf.circle_in_disk(ap.radii, d, 0.5)
        assert np.allclose(G[:, 1], -2.0 * G[:, 0], rtol=1e-14, atol=1e-14)
        errs.append(np.linalg.norm(G[:, 0] - ex) / np.linalg.norm(ex))
    return max(errs)


def test_stage1_matches_disk_closed_form():
    """Circle transform of a (partial-volume) disk against the exact arc
    length inside the disk; the error is voxelisation only and halves with h."""
    e64 = _stage1_disk_error(64, 128)
    e128 = _stage1_disk_error(128, 256)
    assert e64 <= 3e-2
    assert e128 <= 0.6 * e64


def _stage2_disk_error(m, nl):
    ap = cylinder_aperture("t", m, 1.0, 1.5, 1, 9, nl, l_max=3.5)
    a34 = geo.assemble_a34(ap)
    G = _disk_fraction(geo.grid_edges(ap.z0, ap.dz, ap.mz), geo.rho_edges(ap.radii),
                       0.1, 1.0, 0.4)
    Y = srt.crt34(a34, G, ap.n_z, ap.n_radii)
    d = np.hypot(ap.zpos - 0.1, 1.0)
    ex = cf.circle_in_disk(ap.radii[None, :], d[:, None], 0.4)
    return np.linalg.norm(Y - ex) / np.linalg.norm(ex)


def test_stage2_matches_disk_closed_form():
    """Half-circle transform of a disk in the (z, rho) plane (away from the
    axis) against the exact arc length inside the disk."""
    e64 = _stage2_disk_error(64, 128)
    e128 = _stage2_disk_error(128, 256)
    assert e64 <= 2.5e-2
    assert e128 <= 0.6 * e64


# ------------------------------------------------------- P4: uniform balls
def test_ball_cap_area_grid32(grid32):
    """Composition of both stages against the exact SRT of three balls
    (spherical cap areas) at the 32^3 workload."""
    ap, a12s, a34, balls, F = grid32
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    ex = cf.srt_of_balls(ap, balls)
    assert np.linalg.norm(Y - ex) / np.linalg.norm(ex) <= 6.5e-2


@pytest.mark.slow
def test_ball_cap_area_refines():
    """The ball error falls when h and the radial step are halved."""
    errs = []
    for m, nl in [(32, 64), (64, 128)]:
        ap = cylinder_aperture("t", m, 1.0, 1.5, 8, 8, nl, l_max=3.5)
        a12s, a34 = geo.assemble_all(ap)
        balls = phantoms.balls_params(np.random.default_rng(1001))
        F = phantoms.voxelize_balls(ap, balls)
        Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
        ex = cf.srt_of_balls(ap, balls)
        errs.append(np.linalg.norm(Y - ex) / np.linalg.norm(ex))
    assert errs[1] <= 0.6 * errs[0]


def test_closed_forms_integrate_to_area_and_volume():
    """Coarea check of the closed forms themselves: integrating the arc length
    over l gives the disk area; integrating the cap area gives the ball volume."""
    a, d = 0.7, 1.1
    l = np.linspace(0, d + a, 200001)
    assert abs(np.trapezoid(cf.circle_in_disk(l, d, a), l) - np.pi * a * a) < 1e-6
    assert abs(np.trapezoid(cf.sphere_in_ball(l, d, a), l) - 4 / 3 * np.pi * a ** 3) < 1e-6
    d = 0.2  # centre inside: the full circle / sphere region
    l = np.linspace(0, d + a, 200001)
    assert abs(np.trapezoid(cf.sphere_in_ball(l, d, a), l) - 4 / 3 * np.pi * a ** 3) < 1e-6


# --------------------------------------------- P5: sampled discrete operator
def test_matches_sampled_discrete_operator():
    """Alg. 1 from assembled matrices equals Alg. 1 with both transforms done
    by point sampling (no matrices), within the sampling error."""
    ap = cylinder_aperture("t", 12, 1.0, 1.5, 6, 5, 24, l_max=3.5)
    a12s, a34 = geo.assemble_all(ap)
    F = np.random.default_rng(5).uniform(0, 1, ap.vol_shape)
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    Yb = brute.sampled_forward(F, ap, 100_000, 100_000)
    assert np.linalg.norm(Y - Yb) / np.linalg.norm(Y) <= 1e-4


# ----------------------------------- P6: distance from the plain surface integral
@pytest.mark.slow
def test_distance_to_plain_srt_shrinks():
    """The two-stage discrete operator approaches the plain SRT of the
    voxelised object (spherical quadrature) as the radial step shrinks."""
    errs = []
    for nl in (32, 128):
        ap = cylinder_aperture("t", 16, 1.0, 1.5, 2, 3, nl, l_max=3.5)
        a12s, a34 = geo.assemble_all(ap)
        F = phantoms.voxelize_balls(ap, np.array([[0.1, -0.2, 0.05, 0.6, 1.0]]))
        Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
        ref = np.stack([[brute.spherical_quadrature(
            F, ap, (ap.radius * np.cos(ap.angles[a]), ap.radius * np.sin(ap.angles[a]),
                    ap.zpos[h]), ap.radii, 300, 600) for h in range(ap.n_z)]
            for a in range(ap.n_angles)])
        errs.append(np.linalg.norm(Y - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.7 * errs[0]


# ------------------------------------------------------------ P7: mass
def test_mass_invariant(grid32):
    """Coarea: the sum over radii of dl * Y equals the mass of the volume for
    every sensor, up to the midpoint rule in l."""
    ap, a12s, a34, balls, F = grid32
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    dl = ap.radii[1] - ap.radii[0]
    rel = np.abs(Y.sum(-1) * dl / (F.sum() * ap.dxy ** 2 * ap.dz) - 1)
    assert rel.mean() <= 2e-2 and rel.max() <= 8e-2


def test_mass_invariant_refines():
    ap = cylinder_aperture("t", 32, 1.0, 1.5, 4, 4, 256, l_max=3.5)
    a12s, a34 = geo.assemble_all(ap)
    F = phantoms.voxelize_balls(ap, phantoms.balls_params(np.random.default_rng(1001)))
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    dl = ap.radii[1] - ap.radii[0]
    rel = np.abs(Y.sum(-1) * dl / (F.sum() * ap.dxy ** 2 * ap.dz) - 1)
    assert rel.max() <= 1e-2


# ------------------------------------------------------------ P8: adjoint
def test_dot_product(grid32):
    """<A f, g> = <f, A^T g> for the aperture-summed Alg. 2."""
    ap, a12s, a34, balls, F = grid32
    g = np.random.default_rng(2001).standard_normal(ap.data_shape)
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    Fp = srt.adjoint(g, a12s, a34, ap.ms, ap.mz)
    rel = abs((Y * g).sum() - (F * Fp).sum()) / (np.linalg.norm(Y) * np.linalg.norm(g))
    assert rel <= 1e-13
    # results in C order, as the device layouts expect them
    assert Y.flags.c_contiguous and Fp.flags.c_contiguous


def test_adjoint_is_explicit_transpose(grid32):
    """Alg. 2 applied to unit data vectors reproduces the rows of the forward
    operator (explicit transpose on a few entries)."""
    ap, a12s, a34, balls, F = grid32
    rng = np.random.default_rng(3)
    for _ in range(5):
        a, h, l = rng.integers(ap.n_angles), rng.integers(ap.n_z), rng.integers(20, ap.n_radii)
        e = np.zeros(ap.data_shape)
        e[a, h, l] = 1.0
        row = srt.adjoint(e, a12s, a34, ap.ms, ap.mz)
        Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
        assert abs((row * F).sum() - Y[a, h, l]) <= 1e-13 * max(1.0, abs(Y[a, h, l]))


# ------------------------------------------------------------ P9: symmetries
def test_symmetries(grid32):
    """Rotating the object 90 deg about z shifts the sensor angle by N_a/4;
    mirroring y maps angle a to -a; flipping z reverses the sensor heights;
    A34 does not depend on the sensor column."""
    ap, a12s, a34, balls, _ = grid32
    F = np.random.default_rng(7).uniform(0, 1, ap.vol_shape)
    M = ap.ms
    Y = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    i = np.arange(M)
    Frot = F[:, (M - 1 - i)[None, :], i[:, None]]  # Frot[k, j, i] = F[k, M-1-i, j]
    Yrot = srt.forward(Frot, a12s, a34, ap.n_z, ap.n_radii)
    q = ap.n_angles // 4
    scale = np.abs(Y).max()
    assert np.abs(Yrot - np.roll(Y, q, axis=0)).max() <= 1e-12 * scale
    Ym = srt.forward(F[:, ::-1, :], a12s, a34, ap.n_z, ap.n_radii)
    assert np.abs(Ym - Y[(-np.arange(ap.n_angles)) % ap.n_angles]).max() <= 1e-12 * scale
    Yz = srt.forward(F[::-1], a12s, a34, ap.n_z, ap.n_radii)
    assert np.abs(Yz - Y[:, ::-1, :]).max() <= 1e-12 * scale


# ------------------------------------------------------------ P10: sanity
def test_linearity_and_sign(grid32):
    ap, a12s, a34, balls, F = grid32
    rng = np.random.default_rng(11)
    F2 = rng.uniform(0, 1, ap.vol_shape)
    Y1 = srt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    Y2 = srt.forward(F2, a12s, a34, ap.n_z, ap.n_radii)
    Y12 = srt.forward(2.0 * F - 3.0 * F2, a12s, a34, ap.n_z, ap.n_radii)
    assert np.abs(Y12 - (2 * Y1 - 3 * Y2)).max() <= 1e-12 * np.abs(Y12).max()
    assert (Y1 >= 0).all() and (Y2 >= 0).all()
    # spheres that cannot reach the grid see nothing
    near = ap.radius - np.sqrt(2) * 1.0
    assert np.all(Y2[:, :, ap.radii < near - 1e-9] == 0)


def test_cost_exponent():
    """Alg. 1 costs O(M^(4/3)) multiply-adds for M voxels when the numbers of
    sensors and radii grow like M^(1/3) (Sec. 3.1)."""
    Ms, cost = [], []
    for m in (12, 16, 24, 32):
        ap = cylinder_aperture("t", m, 1.0, 1.3, m, m, 4 * m)
        a12s, a34 = geo.assemble_all(ap)
        Ms.append(m ** 3)
        cost.append(srt.flops(a12s, a34, ap.mz))
    slope = np.polyfit(np.log(Ms), np.log(cost), 1)[0]
    assert abs(slope - 4 / 3) <= 0.08
