"""Nonnegative least squares on the GPU (srt_nnls and srt_opnorm2 through the
C ABI) against the oracle's FISTA and power method with the oracle's
operators. The data carry enough noise that the constraint is active.

Tolerances:
  FP64 plan: 1e-12 relative on the ||A||^2 estimate, the iterate and every
  misfit (the operators agree to 1e-12; a projected gradient step does not
  amplify differences, and entries that the projection sets to zero on one
  side only are as small as the rounding that decides them). Measured:
  6e-16, 4e-15 and 2e-16.
  FP32 plan: 1e-6 on the estimate and on the misfits, 1e-5 on the iterate
  (the FP32 applies round at ~1e-7 per step and the extrapolation weights
  approach 1, so differences add up over the iterations). Measured: 2e-8,
  8e-10 and 1.9e-7 after 6 iterations at 128^3.
  A wrong step, sign or weight shows at the 1e-2 level or more.
"""
import numpy as np
import pytest

from oracle import nnls as onn, srt as osrt
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


def _ops(ap, a12s, a34):
    fwd = lambda f: osrt.forward(f, a12s, a34, ap.n_z, ap.n_radii)  # noqa: E731
    adj = lambda y: osrt.adjoint(y, a12s, a34, ap.ms, ap.mz)  # noqa: E731
    return fwd, adj


def _noisy_data(ap, a12s, a34, F, seed, level):
    g = osrt.forward(F, a12s, a34, ap.n_z, ap.n_radii)
    return g + level * np.abs(g).max() * np.random.default_rng(seed).standard_normal(g.shape)


def test_opnorm2_matches_oracle():
    ap, a12s, a34 = operators("grid32")
    fwd, adj = _ops(ap, a12s, a34)
    ref = onn.opnorm2(fwd, adj, ap.vol_shape, 20)
    est64 = _plan(ap, "f64").opnorm2(20)
    est32 = _plan(ap, "f32").opnorm2(20)
    print(f"opnorm2: oracle {ref:.12e}, f64 rel {abs(est64 - ref) / ref:.2e}, "
          f"f32 rel {abs(est32 - ref) / ref:.2e}", flush=True)
    assert abs(est64 - ref) <= 1e-12 * ref
    assert abs(est32 - ref) <= 1e-6 * ref
    assert _plan(ap, "f64").opnorm2(0) == 0.0


def test_nnls_fp64_matches_oracle():
    ap, a12s, a34 = operators("grid32")
    fwd, adj = _ops(ap, a12s, a34)
    g = _noisy_data(ap, a12s, a34, phantoms.phantom(ap), 41, 0.05)
    step = 1.0 / (1.05 * onn.opnorm2(fwd, adj, ap.vol_shape, 30))
    n = 12
    f, resid, used = _plan(ap, "f64").nnls(torch.from_numpy(g).cuda(), n, step=step)
    assert used == step and resid.shape == (n, 1)
    ref, hist = onn.fista_nn(fwd, adj, g, np.zeros(ap.vol_shape), step, n)
    fn = f.cpu().numpy()
    print(f"nnls f64: iterate rel {rel_l2(fn, ref):.2e}, misfit rel "
          f"{np.max(np.abs(resid[:, 0] - hist) / np.asarray(hist)):.2e}, zeros "
          f"{np.mean(ref == 0):.2f}", flush=True)
    assert fn.min() >= 0.0 and np.mean(ref == 0) > 0.05  # the constraint is active
    assert rel_l2(fn, ref) <= 1e-12
    assert np.allclose(resid[:, 0], hist, rtol=1e-12, atol=0)


def test_nnls_fp32_matches_oracle_and_batch_items_are_independent():
    ap, a12s, a34 = operators("grid128")
    fwd, adj = _ops(ap, a12s, a34)
    F = phantoms.batch_phantoms(ap, 2, seed0=4200)
    g = np.stack([_noisy_data(ap, a12s, a34, F[i], 42 + i, 0.05) for i in range(2)])
    gt = torch.from_numpy(g).float().cuda()
    plan = _plan(ap, "f32")
    L = plan.opnorm2(30)
    step = 1.0 / (1.05 * L)
    n = 6
    f, resid, _ = plan.nnls(gt, n, step=step)
    assert resid.shape == (n, 2)
    g0 = gt[0].double().cpu().numpy()
    ref, hist = onn.fista_nn(fwd, adj, g0, np.zeros(ap.vol_shape), float(np.float32(step)), n)
    f0 = f[0].double().cpu().numpy()
    dev = np.abs(resid[:, 0] - np.asarray(hist)) / np.asarray(hist)
    print(f"nnls f32: iterate rel {rel_l2(f0, ref):.2e}, misfit rel {dev.max():.2e}, zeros "
          f"{np.mean(ref == 0):.2f}", flush=True)
    assert f0.min() >= 0.0 and np.mean(ref == 0) > 0.05
    assert rel_l2(f0, ref) <= 1e-5
    assert dev.max() <= 1e-6
    # the second item alone gives bitwise the same iterate (independent problems)
    f1, resid1, _ = plan.nnls(gt[1:2].contiguous(), n, step=step)
    assert torch.equal(f1[0], f[1])
    assert np.array_equal(resid1[:, 0], resid[:, 1])


def test_nnls_ragged_fp64_batch_and_start():
    """Vector lengths that are not a multiple of the 16-byte vector width, a
    batch of 3 and a start that is partly negative (the first projection
    clears it)."""
    from srt_inputs import cylinder_aperture
    from oracle import geometry as geo
    ap = cylinder_aperture("ragged", 13, 1.0, 0.9, 5, 3, 11, mz=7)
    a12s, a34 = geo.assemble_all(ap)
    fwd, adj = _ops(ap, a12s, a34)
    rng = np.random.default_rng(43)
    g = rng.standard_normal((3,) + ap.data_shape)
    f0 = rng.uniform(-0.5, 1.0, (3,) + ap.vol_shape)
    step = 1.0 / (1.05 * onn.opnorm2(fwd, adj, ap.vol_shape, 30))
    f, resid, _ = _plan(ap, "f64").nnls(torch.from_numpy(g).cuda(), 5, step=step,
                                        vol0=torch.from_numpy(f0).cuda())
    for b in range(3):
        ref, hist = onn.fista_nn(fwd, adj, g[b], f0[b], step, 5)
        assert rel_l2(f[b].cpu().numpy(), ref) <= 1e-12, b
        assert np.allclose(resid[:, b], hist, rtol=1e-12, atol=0), b


def test_nnls_default_step_and_argument_errors():
    from paper_2402_15641_amd import binding as B
    ap, _, _ = operators("grid32")
    plan = _plan(ap, "f32")
    g = torch.rand(ap.data_shape, device="cuda")
    L = plan.opnorm2(30)
    f, resid, step = plan.nnls(g, 3)
    assert step == pytest.approx(1.0 / (1.05 * L), rel=1e-12)
    assert resid.shape == (3, 1) and float(f.min()) >= 0.0
    f0, r0, _ = plan.nnls(g, 0)
    assert r0.shape == (0, 1) and float(f0.abs().max()) == 0.0
    L_ = B.lib()
    ws = torch.empty(B.srt_nnls_workspace(plan.handle, 1, 2) + 64, dtype=torch.uint8,
                     device="cuda")
    vol = torch.zeros(ap.vol_shape, device="cuda")
    nb = ws.numel() - 64
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        st = L_.srt_nnls(plan.handle, vol.data_ptr(), g.data_ptr(), 1, 2, bad, None,
                         ws.data_ptr(), nb, None)
        assert st == B.SRT_EINVAL and "step" in B.srt_last_error()
    st = L_.srt_nnls(plan.handle, vol.data_ptr(), g.data_ptr(), 1, 2, 1e-3, None,
                     ws.data_ptr(), nb - 256, None)
    assert st == B.SRT_EINVAL and "workspace" in B.srt_last_error()
    st = L_.srt_nnls(plan.handle, vol.data_ptr(), g.data_ptr(), 1, 2, 1e-3, None,
                     ws.data_ptr() + 8, nb, None)
    assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()
    import ctypes
    d = ctypes.c_double()
    st = L_.srt_opnorm2(plan.handle, 2, ctypes.byref(d), ws.data_ptr(), 16, None)
    assert st == B.SRT_EINVAL and "workspace" in B.srt_last_error()
