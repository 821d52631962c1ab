"""The allocation-free forward, srt_forward_noalloc, through the C ABI.

Its output must equal srt_forward's on the same plan and input (the same
kernels run over the library's fixed scratch array instead of a workspace),
within the FP32 bar of 1e-5 relative L2; bitwise equality is expected and
asserted. Two calls in a row, the second on a smaller input, show that what
the first call left in the shared array does not leak into the second. A
plan and batch whose workspace exceeds the array are refused with EINVAL.
"""
import numpy as np
import pytest

from srt_inputs import config, cylinder_aperture, phantoms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2402_15641_amd import binding
    binding.lib()


def _both(ap, batch, seed):
    """(srt_forward, srt_forward_noalloc) outputs for `batch` phantoms."""
    from paper_2402_15641_amd import SRTPlan, binding as B
    plan = SRTPlan.from_geometry(ap, value_dtype="f32")
    rng = np.random.default_rng(seed)
    vols = phantoms.batch_phantoms(ap, batch, seed0=seed) + 0.1 * rng.standard_normal(
        (batch,) + ap.vol_shape)
    F = torch.from_numpy(vols).float().cuda()
    shape = (batch, ap.n_angles, ap.n_z, ap.n_radii)
    ref = torch.empty(shape, device="cuda")
    out = torch.full(shape, float("nan"), device="cuda")
    stream = torch.cuda.current_stream()
    B.srt_forward(plan.handle, F, ref, batch, None, stream)
    B.srt_forward_noalloc(plan.handle, F, out, batch, stream)
    torch.cuda.synchronize()
    plan.close()
    return ref, out


def _check(ref, out):
    r, o = ref.double().cpu().numpy(), out.double().cpu().numpy()
    assert np.isfinite(o).all()
    assert np.linalg.norm(o - r) <= 1e-5 * np.linalg.norm(r)
    assert torch.equal(ref, out)


def test_noalloc_matches_forward_twice_second_smaller():
    big = cylinder_aperture("noalloc48", 48, 1.0, 1.3, 40, 24, 96)
    print("noalloc: 48^3, batch 3", flush=True)
    _check(*_both(big, 3, 11))
    print("noalloc: 32^3, batch 1", flush=True)
    _check(*_both(config("grid32"), 1, 12))


def test_noalloc_refuses_workspace_beyond_its_array():
    from paper_2402_15641_amd import SRTPlan, binding as B
    ap = config("grid128")
    plan = SRTPlan.from_geometry(ap, value_dtype="f32")
    _, ws = B.srt_plan_footprint(plan.handle, 8)
    assert ws > 256 << 20
    F = torch.zeros((8,) + ap.vol_shape, device="cuda")
    Y = torch.zeros((8, ap.n_angles, ap.n_z, ap.n_radii), device="cuda")
    L = B.lib()
    st = L.srt_forward_noalloc(plan.handle, F.data_ptr(), Y.data_ptr(), 8,
                               torch.cuda.current_stream().cuda_stream)
    assert st == B.SRT_EINVAL
    assert "scratch" in B.srt_last_error()
    # a batch that fits runs and matches srt_forward
    _, ws1 = B.srt_plan_footprint(plan.handle, 1)
    assert ws1 <= 256 << 20
    plan.close()
