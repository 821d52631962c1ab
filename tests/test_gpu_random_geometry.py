"""Parity sweep over seeded random geometries (srt_inputs.random_aperture):
grids that are not centred, voxels that are not cubes, columns inside and
outside the grid, uneven heights and radii, both voxel bases, and for one
seed in three a stage-2 radial grid of its own. Seeds 100-107 are drawn at
three times the size (up to 90^2 x 60 voxels, 21 columns, 75 radii): several
row blocks and chunks per operator, dense widths off the vector width.

Bars as in the fixed-geometry tests: operator entries (FP64) 1e-12 * pitch
per entry; forward and adjoint relative L2 1e-12 (FP64) and 1e-5 (FP32)
against the oracle; with 16-bit stored weights (the packed entry layout;
BF16 on odd seeds, F16 on even ones) 5e-3.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry as geo, linear as lin, srt as osrt
from srt_inputs import random_aperture
from oracle_cache import rel_l2, stacked

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [(s, 1) for s in range(32)] + [(s, 3) for s in range(100, 108)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2402_15641_amd import binding
    binding.lib()


def _t(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _np(t):
    return t.detach().to("cpu", torch.float64).numpy()


@pytest.mark.parametrize("seed,scale", CASES)
def test_random_geometry_matches_oracle(seed, scale):
    from paper_2402_15641_amd import SRTPlan
    ap = random_aperture(seed, scale)
    basis = "constant" if seed % 2 == 0 else "linear"
    a12s, a34 = (geo if basis == "constant" else lin).assemble_all(ap)
    print(f"seed {seed}: {ap.ms}^2 x {ap.mz}, {ap.n_angles} columns, {ap.n_z} heights, "
          f"{ap.n_radii} radii, n_rho {ap.n_rho}, {basis}", flush=True)
    tol_w = 1e-12 * min(ap.dxy, ap.dz)
    plan = SRTPlan.from_geometry(ap, value_dtype="f64", basis=basis)
    assert plan.info["n_rho"] == ap.n_rho
    r, c, v = plan.export_coo(0)
    A = sp.csr_matrix((v, (r, c)), shape=(ap.n_angles * ap.n_rho, ap.ms ** 2))
    assert abs(A - stacked(a12s)).max() <= tol_w
    live = plan.info["live_radii"]
    rows = np.concatenate([m.tocoo().row for m in a12s])
    assert (rows.max() < live if rows.size else live == 0) and live <= ap.n_rho
    if live:
        r, c, v = plan.export_coo(1)
        B = sp.csr_matrix((v, (r, c)), shape=(ap.n_z * ap.n_radii, live * ap.mz))
        assert abs(B - a34[:, :live * ap.mz]).max() <= tol_w
    rng = np.random.default_rng(1000 + seed)
    vols = rng.uniform(-1, 1, (2,) + ap.vol_shape)
    data = rng.standard_normal((2,) + ap.data_shape)
    fwd = np.stack([osrt.forward(x, a12s, a34, ap.n_z, ap.n_radii) for x in vols])
    adj = np.stack([osrt.adjoint(g, a12s, a34, ap.ms, ap.mz) for g in data])
    w16 = "bf16" if seed % 2 else "f16"
    for value, weight, tol in (("f64", "f64", 1e-12), ("f32", "f32", 1e-5), ("f32", w16, 5e-3)):
        dt = torch.float64 if value == "f64" else torch.float32
        p = plan if value == "f64" else SRTPlan.from_geometry(ap, value_dtype=value,
                                                              weight_dtype=weight, basis=basis)
        assert rel_l2(_np(p.forward(_t(vols, dt))), fwd) <= tol, weight
        assert rel_l2(_np(p.adjoint(_t(data, dt))), adj) <= tol, weight
