"""The allocation-free forward, srt_forward_noalloc, through the C ABI.

Its output must equal srt_forward's on the same plan and input (the same
kernels run over the library's fixed scratch array instead of a workspace),
within the FP32 bar of 1e-5 relative L2; bitwise equality is expected and
asserted. Two calls in a row, the second on a smaller input, show that what
the first call left in the shared array does not leak into the second. A
plan and batch whose workspace exceeds the array are refused with EINVAL.
The call is also captured into a HIP graph, the use it exists for, and the
graph's replays are checked against srt_forward.
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


def test_noalloc_replays_from_a_hip_graph():
    """Captured into a HIP graph (nothing is allocated inside the capture) and
    replayed. Between replays the graph's input is overwritten and the same
    plan runs eagerly through srt_forward; every replay equals the eager
    srt_forward of its input, bitwise."""
    from paper_2402_15641_amd import SRTPlan, binding as B
    ap = config("grid32")
    plan = SRTPlan.from_geometry(ap, value_dtype="f32")
    batch = 2
    rng = np.random.default_rng(21)
    vols = [torch.from_numpy(phantoms.batch_phantoms(ap, batch, seed0=21 + 5 * i)
                             + 0.1 * rng.standard_normal((batch,) + ap.vol_shape)).float().cuda()
            for i in range(3)]
    shape = (batch, ap.n_angles, ap.n_z, ap.n_radii)
    cur = torch.cuda.current_stream
    refs = []
    for v in vols:
        r = torch.empty(shape, device="cuda")
        B.srt_forward(plan.handle, v, r, batch, None, cur())
        refs.append(r)
    src = vols[0].clone()
    out = torch.full(shape, float("nan"), device="cuda")
    # the first call on a device looks the scratch array's address up: make it
    # outside the capture
    B.srt_forward_noalloc(plan.handle, src, out, batch, cur())
    torch.cuda.synchronize()
    assert torch.equal(out, refs[0])
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.srt_forward_noalloc(plan.handle, src, out, batch, cur())
    other = torch.empty(shape, device="cuda")
    for step, i in enumerate([1, 2, 0, 2, 1]):
        print(f"graph replay {step}: input {i}", flush=True)
        src.copy_(vols[i])
        out.fill_(float("nan"))
        graph.replay()
        B.srt_forward(plan.handle, vols[(i + 1) % 3], other, batch, None, cur())
        torch.cuda.synchronize()
        assert torch.equal(out, refs[i]), step
        assert torch.equal(other, refs[(i + 1) % 3]), step
    del graph
    plan.close()
