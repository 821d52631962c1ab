"""On-the-fly plans (SRT_OP_ONTHEFLY) against stored plans, through the C ABI.

An on-the-fly plan keeps only its geometry; every apply regenerates the two
operators its direction needs and releases them afterwards. It must report
the same operator sizes, export the same entries, and give results bitwise
equal to a stored plan's (the same builder and the same kernels), for the
forward, the adjoint and a reconstruction that applies both repeatedly.
"""
import ctypes
import time

import numpy as np
import pytest

from srt_inputs import config, phantoms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2402_15641_amd import binding
    binding.lib()


def _pair(ap, value, weight=None):
    from paper_2402_15641_amd import SRTPlan
    st = SRTPlan.from_geometry(ap, value_dtype=value, weight_dtype=weight, mode="stored")
    otf = SRTPlan.from_geometry(ap, value_dtype=value, weight_dtype=weight, mode="onthefly")
    return st, otf


def test_grid32_fp64_same_operators_and_results():
    from paper_2402_15641_amd import binding as B
    ap = config("grid32")
    st, otf = _pair(ap, "f64")
    assert st.info["mode"] == B.MODES["stored"] and otf.info["mode"] == B.MODES["onthefly"]
    for k in ("nnz_a12", "nnz_a34", "live_radii", "operator_bytes"):
        assert st.info[k] == otf.info[k], k
    res_st, _ = B.srt_plan_footprint(st.handle, 1)
    res_otf, _ = B.srt_plan_footprint(otf.handle, 1)
    assert res_otf < res_st and res_st - res_otf == st.info["operator_bytes"]
    for which in range(4):
        a, b = st.export_coo(which), otf.export_coo(which)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), which
    rng = np.random.default_rng(21)
    F = torch.from_numpy(rng.uniform(-1, 1, (2,) + ap.vol_shape)).cuda()
    g = torch.from_numpy(rng.standard_normal((2,) + ap.data_shape)).cuda()
    assert torch.equal(st.forward(F), otf.forward(F))
    assert torch.equal(st.adjoint(g), otf.adjoint(g))
    st.close()
    otf.close()


def test_grid128_bf16_results_and_cgls_bitwise():
    ap = config("grid128")
    st, otf = _pair(ap, "f32", "bf16")
    F = torch.from_numpy(phantoms.phantom(ap)).float().cuda()
    Y = st.forward(F)
    assert torch.equal(Y, otf.forward(F))
    assert torch.equal(st.adjoint(Y), otf.adjoint(Y))
    f1, r1 = st.cgls(Y, 2)
    f2, r2 = otf.cgls(Y, 2)
    assert torch.equal(f1, f2) and np.array_equal(r1, r2)
    # the cost of regenerating: one forward each way, after warm-up
    for p in (st, otf):
        p.forward(F)
    torch.cuda.synchronize()
    t = []
    for p in (st, otf):
        t0 = time.perf_counter()
        p.forward(F)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    print(f"128^3 forward: stored {t[0] * 1e3:.2f} ms, on the fly {t[1] * 1e3:.2f} ms")
    st.close()
    otf.close()


def test_auto_keeps_operators_that_fit_and_noalloc_refuses_onthefly():
    from paper_2402_15641_amd import SRTPlan, binding as B
    ap = config("grid32")
    auto = SRTPlan.from_geometry(ap, value_dtype="f32", mode="auto")
    assert auto.info["mode"] == B.MODES["stored"]
    otf = SRTPlan.from_geometry(ap, value_dtype="f32", mode="onthefly")
    F = torch.zeros((1,) + ap.vol_shape, device="cuda")
    Y = torch.zeros((1, ap.n_angles, ap.n_z, ap.n_radii), device="cuda")
    st = B.lib().srt_forward_noalloc(otf.handle, F.data_ptr(), Y.data_ptr(), 1,
                                     torch.cuda.current_stream().cuda_stream)
    assert st == B.SRT_EINVAL and "on-the-fly" in B.srt_last_error()
    auto.close()
    otf.close()


@pytest.mark.parametrize("seed", [3, 8, 14])
def test_widened_operators_onthefly_equal_stored(seed):
    """Seeded random geometries (columns anywhere, uneven heights and radii,
    some with a stage-2 radial grid of their own) on the linear basis: an
    on-the-fly plan's forward and adjoint equal a stored plan's bitwise."""
    from paper_2402_15641_amd import SRTPlan
    from srt_inputs import random_aperture
    ap = random_aperture(seed, scale=2)
    plans = [SRTPlan.from_geometry(ap, value_dtype="f32", basis="linear", mode=m)
             for m in ("stored", "onthefly")]
    rng = np.random.default_rng(seed)
    F = torch.from_numpy(rng.uniform(-1, 1, ap.vol_shape)).float().cuda()
    g = torch.from_numpy(rng.standard_normal(ap.data_shape)).float().cuda()
    assert torch.equal(plans[0].forward(F), plans[1].forward(F))
    assert torch.equal(plans[0].adjoint(g), plans[1].adjoint(g))
    for p in plans:
        p.close()
