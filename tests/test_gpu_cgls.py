"""Least-squares reconstruction on the GPU (srt_cgls through the C ABI)
against the oracle's CGLS with the oracle's operators.

Tolerances:
  FP64 plan, 8 iterations: 1e-9 relative L2 on the iterate and on every
  residual norm (the operators agree to 1e-12 and CG amplifies the
  difference by far less than 1e3 in 8 steps).
  FP32 plan, 5 iterations: the normal equations are badly conditioned, and
  CG carries the ~1e-7 rounding of each FP32 apply into the iterate along the
  smallest singular directions, where it is barely constrained: at 6
  iterations the iterate differed from the FP64 oracle by 2.2e-4 and the
  last residual norm by 1.0e-3 (measured; the earlier norms by <= 1.1e-6).
  The iterate is held to 1e-3, the residual norms of 5 iterations to 1e-4,
  and the data misfit ||A f - g||, the quantity CG minimises and first-order
  insensitive to those directions, to 1e-5. A wrong step length or sign
  shows at the 1e-1 level in all three.
"""
import numpy as np
import pytest

from oracle import cgls as ocg, srt as osrt
from oracle_cache import operators, rel_l2
from srt_inputs import phantoms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


def _plan(ap, value):
    from paper_2402_15641_amd import SRTPlan
    return SRTPlan.from_geometry(ap, value_dtype=value)


def _oracle(ap, a12s, a34, g, n_iter):
    fwd = lambda f: osrt.forward(f, a12s, a34, ap.n_z, ap.n_radii)  # noqa: E731
    adj = lambda y: osrt.adjoint(y, a12s, a34, ap.ms, ap.mz)  # noqa: E731
    return ocg.cgls(fwd, adj, g, np.zeros(ap.vol_shape), n_iter)


def test_cgls_fp64_matches_oracle():
    ap, a12s, a34 = operators("grid32")
    rng = np.random.default_rng(31)
    F = phantoms.phantom(ap)
    g = osrt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    g = g + 0.01 * np.abs(g).max() * rng.standard_normal(g.shape)
    plan = _plan(ap, "f64")
    f, resid = plan.cgls(torch.from_numpy(g).cuda(), 8)
    ref, hist = _oracle(ap, a12s, a34, g, 8)
    assert rel_l2(f.cpu().numpy(), ref) <= 1e-9
    assert np.allclose(resid[:, 0], hist, rtol=1e-9, atol=0)


def test_cgls_fp32_matches_oracle_and_batch_items_are_independent():
    ap, a12s, a34 = operators("grid128")
    F = phantoms.batch_phantoms(ap, 2, seed0=4100)
    rng = np.random.default_rng(32)
    g = np.stack([osrt.forward(F[i], a12s, a34, ap.n_z, ap.n_radii) for i in range(2)])
    g += 0.01 * np.abs(g).max() * rng.standard_normal(g.shape)
    plan = _plan(ap, "f32")
    gt = torch.from_numpy(g).float().cuda()
    n = 5
    f, resid = plan.cgls(gt, n)
    assert resid.shape == (n + 1, 2)
    g0 = gt[0].double().cpu().numpy()
    ref, hist = _oracle(ap, a12s, a34, g0, n)
    f0 = f[0].double().cpu().numpy()
    assert rel_l2(f0, ref) <= 1e-3
    dev = np.abs(resid[:, 0] - np.asarray(hist)) / np.asarray(hist)
    assert dev.max() <= 1e-4, (resid[:, 0].tolist(), list(map(float, hist)))
    mis = np.linalg.norm(osrt.forward(f0, a12s, a34, ap.n_z, ap.n_radii) - g0)
    mis_ref = np.linalg.norm(osrt.forward(ref, a12s, a34, ap.n_z, ap.n_radii) - g0)
    assert abs(mis - mis_ref) <= 1e-5 * mis_ref
    # the second item alone gives bitwise the same iterate (independent problems)
    f1, resid1 = plan.cgls(gt[1:2].contiguous(), n)
    assert torch.equal(f1[0], f[1])
    assert np.array_equal(resid1[:, 0], resid[:, 1])


def test_cgls_data_residual_never_increases():
    ap, a12s, a34 = operators("grid128")
    F = phantoms.phantom(ap)
    plan = _plan(ap, "f32")
    g = plan.forward(torch.from_numpy(F).float().cuda())
    g = g + 0.01 * g.abs().max() * torch.randn(g.shape, generator=torch.Generator().manual_seed(33)).cuda()
    prev = float("inf")
    for k in (0, 2, 4, 8, 12):
        f, _ = plan.cgls(g, k)
        res = float((plan.forward(f) - g).double().norm())
        assert res <= prev * (1 + 1e-6), k
        prev = res


def test_cgls_ragged_fp64_batch():
    """Vector lengths that are not a multiple of the 16-byte vector width
    (13 x 13 x 7 voxels, 5 x 3 x 11 samples) and a batch of 3: the scalar
    paths of the update and reduction kernels."""
    from srt_inputs import cylinder_aperture
    from oracle import geometry as geo
    ap = cylinder_aperture("ragged", 13, 1.0, 0.9, 5, 3, 11, mz=7)
    a12s, a34 = geo.assemble_all(ap)
    rng = np.random.default_rng(34)
    g = rng.standard_normal((3,) + ap.data_shape)
    plan = _plan(ap, "f64")
    f, resid = plan.cgls(torch.from_numpy(g).cuda(), 4)
    for b in range(3):
        ref, hist = _oracle(ap, a12s, a34, g[b], 4)
        assert rel_l2(f[b].cpu().numpy(), ref) <= 1e-9, b
        assert np.allclose(resid[:, b], hist, rtol=1e-9, atol=0), b
