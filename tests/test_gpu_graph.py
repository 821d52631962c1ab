"""srt_forward and srt_adjoint captured into a HIP graph (through torch's
CUDAGraph on ROCm) and replayed: with a caller workspace an apply only
launches kernels, so every replay must reproduce the eager result bitwise.

Each replay follows eager work of its own on the same plan (another input,
the plan's own workspace) and a synchronisation, and the graph's outputs are
overwritten with NaN before it, so a replay that skipped or reordered a node
would show. The degenerate plan whose spheres all miss the grid clears its
outputs with a kernel, which the graph must hold too.
"""
import numpy as np
import pytest

from oracle_cache import operators
from srt_inputs import cylinder_aperture

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


def _plan(ap, value="f32", weight=None):
    from paper_2402_15641_amd import SRTPlan
    return SRTPlan.from_geometry(ap, value_dtype=value, weight_dtype=weight)


def _capture_pair(plan, vol, data, back, ws):
    side = torch.cuda.Stream()  # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up off the capturing stream
        plan.forward(vol, out=data, workspace=ws)
        plan.adjoint(data, out=back, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(vol, out=data, workspace=ws)
        plan.adjoint(data, out=back, workspace=ws)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("weight", ["f32", "bf16"])
def test_captured_pair_replays_bitwise(weight):
    ap, _, _ = operators("grid32")
    plan = _plan(ap, "f32", weight)
    rng = np.random.default_rng(51)
    vol = torch.from_numpy(rng.uniform(0, 1, (2,) + ap.vol_shape)).float().cuda()
    Y0 = plan.forward(vol)
    F0 = plan.adjoint(Y0)
    torch.cuda.synchronize()
    ws = plan.workspace(2)
    data = torch.empty_like(Y0)
    back = torch.empty_like(F0)
    g = _capture_pair(plan, vol, data, back, ws)
    for i in range(4):
        data.fill_(float("nan"))
        back.fill_(float("nan"))
        other = plan.adjoint(plan.forward(vol * (i + 2)))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(data, Y0), i
        assert torch.equal(back, F0), i
        assert torch.isfinite(other).all()


def test_captured_degenerate_plan_clears_its_outputs():
    ap = cylinder_aperture("far", 8, 1.0, 50.0, 4, 3, 5, l_max=2.0)
    plan = _plan(ap, "f32")
    assert plan.info["live_radii"] == 0
    vol = torch.ones(ap.vol_shape, device="cuda")
    ws = plan.workspace(1)
    data = torch.empty(ap.data_shape, device="cuda")
    back = torch.empty(ap.vol_shape, device="cuda")
    g = _capture_pair(plan, vol, data, back, ws)
    for i in range(3):
        data.fill_(float("nan"))
        back.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(data.abs().max()) == 0.0 and float(back.abs().max()) == 0.0, i
