"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative L2 over a whole output unless stated):
  FP64 values and weights   1e-12
  FP32 values and weights   1e-5
  BF16 / FP16 weights       5e-3
  adjoint dot test          1e-6 of |<A f, g>| (the Cauchy-Schwarz form,
                            |<Af,g> - <f,A^T g>| / (||A f|| ||g||), is printed beside it)
  operator entries (FP64)   1e-12 * pitch per entry
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry as geo, srt as osrt
from srt_inputs import config, cylinder_aperture, phantoms
from oracle_cache import operators, oracle_adjoint, oracle_forward, rel_l2, stacked

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2402_15641_amd import binding
    binding.lib()


def _plan(ap, value="f32", weight=None):
    from paper_2402_15641_amd import SRTPlan
    return SRTPlan.from_geometry(ap, value_dtype=value, weight_dtype=weight)


def _t(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _np(t):
    return t.detach().to("cpu", torch.float64).numpy()


def _dot(Y, g, F, Fg):
    """Dot test on device results, inner products in FP64: the error
    |<A f, g> - <f, A^T g>| relative to |<A f, g>| (asserted), and relative to
    the Cauchy-Schwarz bound ||A f|| ||g|| (a weaker measure, printed)."""
    lhs = float((Y.double() * g.double()).sum())
    rhs = float((F.double() * Fg.double()).sum())
    rel = abs(lhs - rhs) / abs(lhs)
    cs = abs(lhs - rhs) / (float(Y.double().norm()) * float(g.double().norm()))
    print(f"dot test: relative {rel:.2e}, Cauchy-Schwarz {cs:.2e}")
    return rel


# ------------------------------------------------------------------ operators
def test_operators_match_oracle_grid32():
    """Every stored weight equals the oracle's arc length (FP64 plan), the
    transposes hold the same entries, and dropped rho cells are empty."""
    ap, a12s, a34 = operators("grid32")
    plan = _plan(ap, "f64")
    h = ap.dxy
    r, c, v = plan.export_coo(0)
    A = sp.csr_matrix((v, (r, c)), shape=(ap.n_angles * ap.n_radii, ap.ms ** 2))
    assert abs(A - stacked(a12s)).max() <= 1e-12 * h
    live = plan.info["live_radii"]
    r, c, v = plan.export_coo(1)
    B = sp.csr_matrix((v, (r, c)), shape=(ap.n_z * ap.n_radii, live * ap.mz))
    assert abs(B - a34[:, :live * ap.mz]).max() <= 1e-12 * h
    # rho cells at or beyond `live` receive no stage-1 value from any column
    rows_l = np.concatenate([A.tocoo().row for A in a12s])
    assert rows_l.size == 0 or rows_l.max() < live
    # stored transposes are exact transposes
    for which, M in ((2, A), (3, B)):
        r, c, v = plan.export_coo(which)
        T = sp.csr_matrix((v, (r, c)), shape=M.T.shape)
        D = (T - M.T.tocsr())
        assert D.nnz == 0 or abs(D).max() == 0.0


@pytest.mark.parametrize("weight", ["bf16", "f16"])
def test_rounded_weights_are_nearest(weight):
    """16-bit weights are the FP64 arc lengths rounded once to nearest."""
    ap, a12s, a34 = operators("grid32")
    plan = _plan(ap, "f32", weight)
    r, c, v = plan.export_coo(1)
    B = sp.csr_matrix((v, (r, c)), shape=(ap.n_z * ap.n_radii, plan.info["live_radii"] * ap.mz))
    ref = a34[:, :B.shape[1]].tocsr()
    scale = plan.info["weight_scale_a34"]
    ulp = 2.0 ** -8 if weight == "bf16" else 2.0 ** -11  # half ulp bound, relative
    diff = abs(B - ref).tocoo()
    refv = np.asarray(ref[diff.row, diff.col]).ravel()
    tiny = 2.0 ** (-133 if weight == "bf16" else -24) / scale
    assert np.all(diff.data <= ulp * refv + tiny)


# ------------------------------------------------------------------ grid32
@pytest.mark.parametrize("value,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_grid32_forward_adjoint(value, tol):
    ap, a12s, a34 = operators("grid32")
    F = phantoms.phantom(ap)
    g = phantoms.gaussian_data(ap, np.random.default_rng(2001))
    dt = torch.float64 if value == "f64" else torch.float32
    Ft, gt = _t(F, dt), _t(g, dt)
    Fin, gin = _np(Ft), _np(gt)  # the exact values the device sees
    plan = _plan(ap, value)
    Y = plan.forward(Ft)
    assert rel_l2(_np(Y), osrt.forward(Fin, a12s, a34, ap.n_z, ap.n_radii)) <= tol
    Fp = plan.adjoint(gt)
    assert rel_l2(_np(Fp), osrt.adjoint(gin, a12s, a34, ap.ms, ap.mz)) <= tol


# ------------------------------------------------------------------ ragged / degenerate
RAGGED = [
    # ms, mz, R, na, nh, nl, batch: tails in every dimension, odd dense widths
    (13, 7, 0.9, 5, 3, 11, 3),
    (24, 65, 1.7, 7, 9, 70, 2),
    (9, 3, 0.0, 4, 2, 6, 1),     # columns on the cylinder axis, inside the grid
]


@pytest.mark.parametrize("ms,mz,R,na,nh,nl,batch", RAGGED)
@pytest.mark.parametrize("value", ["f64", "f32"])
def test_ragged_shapes(ms, mz, R, na, nh, nl, batch, value):
    ap = cylinder_aperture("ragged", ms, 1.0, R, na, nh, nl, mz=mz)
    a12s, a34 = geo.assemble_all(ap)
    rng = np.random.default_rng(ms * 1000 + mz)
    vols = rng.uniform(-1, 1, (batch,) + ap.vol_shape)
    data = rng.standard_normal((batch,) + ap.data_shape)
    dt = torch.float64 if value == "f64" else torch.float32
    tol = 1e-12 if value == "f64" else 1e-5
    vt, dtt = _t(vols, dt), _t(data, dt)
    plan = _plan(ap, value)
    assert rel_l2(_np(plan.forward(vt)), oracle_forward(ap, a12s, a34, _np(vt))) <= tol
    assert rel_l2(_np(plan.adjoint(dtt)), oracle_adjoint(ap, a12s, a34, _np(dtt))) <= tol


MINIMAL = [
    # ms, mz, R, na, nh, nl: single-element axes
    (1, 1, 0.7, 1, 1, 1),
    (2, 1, 1.5, 1, 1, 1),
    (5, 1, 1.2, 3, 1, 2),
    (1, 4, 0.3, 2, 3, 1),
    (3, 2, 0.0, 1, 2, 3),
]


@pytest.mark.parametrize("ms,mz,R,na,nh,nl", MINIMAL)
@pytest.mark.parametrize("basis", ["constant", "linear"])
def test_minimal_shapes(ms, mz, R, na, nh, nl, basis):
    """One pixel, one slice, one radius, one height or one column, on both
    bases (FP64, batch 2) against the oracle."""
    from oracle import linear as lin
    from paper_2402_15641_amd import SRTPlan
    ap = cylinder_aperture("min", ms, 1.0, R, na, nh, nl, l_max=2.5, mz=mz)
    a12s, a34 = (geo if basis == "constant" else lin).assemble_all(ap)
    rng = np.random.default_rng(ms * 100 + mz * 10 + nl)
    vols = rng.uniform(-1, 1, (2,) + ap.vol_shape)
    data = rng.standard_normal((2,) + ap.data_shape)
    plan = SRTPlan.from_geometry(ap, value_dtype="f64", basis=basis)
    assert rel_l2(_np(plan.forward(_t(vols, torch.float64))),
                  oracle_forward(ap, a12s, a34, vols)) <= 1e-12
    assert rel_l2(_np(plan.adjoint(_t(data, torch.float64))),
                  oracle_adjoint(ap, a12s, a34, data)) <= 1e-12


def test_empty_batch():
    """batch 0 is an argument error at the C ABI; the torch wrapper returns an
    empty result without calling it."""
    import ctypes
    from paper_2402_15641_amd import binding as B
    ap, _, _ = operators("grid32")
    plan = _plan(ap, "f32")
    vol = torch.zeros((0,) + ap.vol_shape, device="cuda")
    assert plan.forward(vol).shape == (0,) + ap.data_shape
    assert plan.adjoint(torch.zeros((0,) + ap.data_shape, device="cuda")).shape == vol.shape
    out = torch.empty(ap.data_shape, device="cuda")
    one = torch.zeros(ap.vol_shape, device="cuda")
    st = B.lib().srt_forward(plan.handle, one.data_ptr(), out.data_ptr(), 0, None, 0, None)
    assert st == B.SRT_EINVAL and "batch" in B.srt_last_error()


def test_no_sphere_reaches_the_grid():
    """Sensors far away with short radii: both transforms are exactly zero."""
    ap = cylinder_aperture("far", 8, 1.0, 50.0, 4, 3, 5, l_max=2.0)
    plan = _plan(ap, "f32")
    assert plan.info["live_radii"] == 0 and plan.info["nnz_a12"] == 0
    Y = plan.forward(torch.ones(ap.vol_shape, device="cuda"))
    F = plan.adjoint(torch.ones(ap.data_shape, device="cuda"))
    assert float(Y.abs().max()) == 0.0 and float(F.abs().max()) == 0.0


def test_batch_and_workspace_are_bitwise_stable():
    ap, a12s, a34 = operators("grid32")
    plan = _plan(ap, "f32")
    rng = np.random.default_rng(9)
    vols = _t(rng.uniform(0, 1, (3,) + ap.vol_shape), torch.float32)
    Yb = plan.forward(vols)
    for i in range(3):
        assert torch.equal(plan.forward(vols[i].contiguous()), Yb[i])
    ws = plan.workspace(3)
    assert torch.equal(plan.forward(vols, workspace=ws), Yb)
    Fb = plan.adjoint(Yb, workspace=ws)
    assert torch.equal(plan.adjoint(Yb), Fb)
    from paper_2402_15641_amd.binding import SRTError, SRT_EINVAL
    with pytest.raises(SRTError) as e:
        plan.forward(vols, workspace=ws[:1024])
    assert e.value.status == SRT_EINVAL


def test_wrapper_rejects_outputs_and_workspaces_it_cannot_use():
    """The torch wrapper refuses an output (or CGLS start) holding another
    number of items than the input, and a workspace that is not a contiguous
    tensor on the plan's device, before the library is called; a batch of
    one is accepted with or without its batch axis, and an empty CGLS batch
    returns at once."""
    ap, _, _ = operators("grid32")
    plan = _plan(ap, "f32")
    vols = _t(np.random.default_rng(6).uniform(0, 1, (3,) + ap.vol_shape), torch.float32)
    data = torch.zeros((3,) + ap.data_shape, device="cuda")
    for bad in ((2,) + ap.data_shape, ap.data_shape, (4,) + ap.data_shape):
        with pytest.raises(ValueError, match="item"):
            plan.forward(vols, out=torch.empty(bad, device="cuda"))
    with pytest.raises(ValueError, match="item"):
        plan.adjoint(data, out=torch.empty(ap.vol_shape, device="cuda"))
    with pytest.raises(ValueError, match="item"):
        plan.cgls(data, 1, vol0=torch.zeros(ap.vol_shape, device="cuda"))
    ws = plan.workspace(3)
    for bad in (ws.cpu(), ws[::2]):
        with pytest.raises(ValueError, match="workspace"):
            plan.forward(vols, workspace=bad)
        with pytest.raises(ValueError, match="workspace"):
            plan.adjoint(data, workspace=bad)
    with pytest.raises(ValueError, match="workspace"):
        plan.cgls(data, 1, workspace=ws.cpu())
    Y1 = plan.forward(vols[0])
    out = torch.empty((1,) + ap.data_shape, device="cuda")
    assert torch.equal(plan.forward(vols[0], out=out)[0], Y1)
    out = torch.empty(ap.data_shape, device="cuda")
    assert torch.equal(plan.forward(vols[:1], out=out), Y1)
    f, r = plan.cgls(torch.zeros((0,) + ap.data_shape, device="cuda"), 2)
    assert f.shape == (0,) + ap.vol_shape and r.shape == (3, 0)


def test_misaligned_arrays_are_rejected():
    """A caller workspace off 16-byte alignment, or a volume or data array off
    its element size, is an argument error caught before anything runs (apply
    and CGLS); a 16-byte offset is accepted and gives the same result."""
    from paper_2402_15641_amd import binding as B
    ap, _, _ = operators("grid32")
    plan = _plan(ap, "f32")
    L = B.lib()
    vol = _t(np.random.default_rng(4).uniform(0, 1, ap.vol_shape), torch.float32)
    data = torch.zeros(ap.data_shape, device="cuda")
    n = plan.workspace(1).numel()
    big = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    for off in (4, 8):
        st = L.srt_forward(plan.handle, vol.data_ptr(), data.data_ptr(), 1,
                           big.data_ptr() + off, n, None)
        assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()
    st = L.srt_adjoint(plan.handle, data.data_ptr(), vol.data_ptr() + 2, 1, None, 0, None)
    assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()
    st = L.srt_forward(plan.handle, vol.data_ptr() + 1, data.data_ptr(), 1, None, 0, None)
    assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()
    Y0 = plan.forward(vol)
    torch.cuda.synchronize()
    st = L.srt_forward(plan.handle, vol.data_ptr(), data.data_ptr(), 1, big.data_ptr() + 16, n,
                       None)
    torch.cuda.synchronize()
    assert st == B.SRT_OK and torch.equal(data, Y0)
    nb = B.srt_cgls_workspace(plan.handle, 1, 2)
    cw = torch.zeros(nb + 64, dtype=torch.uint8, device="cuda")
    st = L.srt_cgls(plan.handle, vol.data_ptr(), data.data_ptr(), 1, 2, None, cw.data_ptr() + 8,
                    nb, None)
    assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()
    st = L.srt_cgls(plan.handle, vol.data_ptr() + 2, data.data_ptr(), 1, 2, None, cw.data_ptr(),
                    nb, None)
    assert st == B.SRT_EINVAL and "aligned" in B.srt_last_error()


# ------------------------------------------------------------------ grid128
@pytest.fixture(scope="module")
def grid128():
    ap, a12s, a34 = operators("grid128")
    F = phantoms.phantom(ap)
    Ft = _t(F, torch.float32)
    Fin = _np(Ft)[None]
    Y = oracle_forward(ap, a12s, a34, Fin)
    g = phantoms.gaussian_data(ap, np.random.default_rng(2002))[None]
    gt = _t(g, torch.float32)
    Fp = oracle_adjoint(ap, a12s, a34, _np(gt))
    return ap, Ft, gt, Y, Fp


def test_grid128_forward_adjoint_f32(grid128):
    ap, Ft, gt, Y, Fp = grid128
    plan = _plan(ap, "f32")
    Yg = plan.forward(Ft[None].contiguous())
    assert rel_l2(_np(Yg), Y) <= 1e-5
    Fg = plan.adjoint(gt)
    assert rel_l2(_np(Fg), Fp) <= 1e-5
    # dot tests: N(0,1) data, and its absolute value (no cancellation in <Af, g>)
    assert _dot(Yg, gt, Ft[None], Fg) <= 1e-6
    assert _dot(Yg, gt.abs(), Ft[None], plan.adjoint(gt.abs())) <= 1e-6


@pytest.mark.parametrize("weight", ["bf16", "f16"])
def test_grid128_rounded_weights(grid128, weight):
    ap, Ft, gt, Y, Fp = grid128
    plan = _plan(ap, "f32", weight)
    Yg = plan.forward(Ft[None].contiguous())
    Fg = plan.adjoint(gt)
    assert rel_l2(_np(Yg), Y) <= 5e-3
    assert rel_l2(_np(Fg), Fp) <= 5e-3
    # the same rounded weights on both sides: the dot test holds as in FP32
    assert _dot(Yg, gt, Ft[None], Fg) <= 1e-6
    assert _dot(Yg, gt.abs(), Ft[None], plan.adjoint(gt.abs())) <= 1e-6


# ------------------------------------------------------------------ pact256 (full size)
# 32 columns spread over the whole angle range, three heights
PACT_COLS = list(range(5, 512, 16))
PACT_HEIGHTS = [10, 128, 245]


@pytest.fixture(scope="module")
def pact256_oracle():
    """The FP32-cast 256^3 phantom, the oracle's A12 of 32 columns and its
    A34 rows of three heights, the forward planes of those (column, height)
    pairs, and the adjoint of N(0,1) data on all of them."""
    ap = config("pact256")
    Ft = _t(phantoms.phantom(ap), torch.float32)
    Fin = _np(Ft)
    a34 = geo.assemble_a34(ap, heights=PACT_HEIGHTS)
    a12 = {a: geo.assemble_a12(ap, ap.angles[a]) for a in PACT_COLS}
    fwd = {}
    for a in PACT_COLS:
        G = osrt.crt12(a12[a], Fin).reshape(-1)
        for h in PACT_HEIGHTS:
            fwd[a, h] = a34[h * ap.n_radii:(h + 1) * ap.n_radii] @ G
    rng = np.random.default_rng(2003)
    data = np.zeros(ap.data_shape)
    for a in PACT_COLS:
        for h in PACT_HEIGHTS:
            data[a, h] = rng.standard_normal(ap.n_radii)
    dt = _t(data, torch.float32)
    din = _np(dt)
    adj = np.zeros(ap.vol_shape)
    for a in PACT_COLS:
        adj += osrt.crt12_t(a12[a], osrt.crt34_t(a34, din[a], ap.mz), ap.ms)
    return ap, Ft, fwd, dt, adj


@pytest.mark.parametrize("weight,tol", [("f32", 1e-5), ("bf16", 5e-3)])
def test_pact256_sampled_forward_and_adjoint(pact256_oracle, weight, tol):
    """At the 256^3 PACT-scale workload, in the launch configuration the
    benchmark times: the forward's [h][l] planes of 32 columns spread over
    the angle range at three heights each (96 planes) against the oracle, and
    the whole adjoint volume of data that is non-zero on those 96 planes
    (the oracle needs only their rows)."""
    ap, Ft, fwd, dt, adj = pact256_oracle
    plan = _plan(ap, "f32", weight)
    Y = _np(plan.forward(Ft))
    for (a, h), ref in fwd.items():
        assert rel_l2(Y[a, h], ref) <= tol, (a, h)
    assert rel_l2(_np(plan.adjoint(dt)), adj) <= tol


@pytest.mark.parametrize("weight", ["f32", "bf16"])
def test_pact256_dot_test(weight):
    """At 256^3, the device's forward and adjoint agree as a transpose pair:
    <A f, g> = <f, A^T g> to 1e-6 of |<A f, g>| for the phantom f and N(0,1)
    data g on every column, height and radius, and for |g|. Inner products
    in FP64; no oracle."""
    ap = config("pact256")
    F = _t(phantoms.phantom(ap), torch.float32)
    plan = _plan(ap, "f32", weight)
    g = _t(np.random.default_rng(2013).standard_normal(ap.data_shape), torch.float32)
    Y = plan.forward(F)
    assert _dot(Y, g, F, plan.adjoint(g)) <= 1e-6
    assert _dot(Y, g.abs(), F, plan.adjoint(g.abs())) <= 1e-6


def test_pact256_sampled_adjoint_f16_weights(pact256_oracle):
    """At 256^3 with F16 weights (the packed entry layout): the adjoint of data
    on the 96 sampled planes against the FP64 oracle, within 5e-3."""
    ap, Ft, fwd, dt, adj = pact256_oracle
    plan = _plan(ap, "f32", "f16")
    assert rel_l2(_np(plan.adjoint(dt)), adj) <= 5e-3


@pytest.mark.parametrize("weight", ["bf16", "f16"])
def test_pact256_sampled_forward_16bit_weights(weight):
    """At 256^3 with 16-bit weights (the packed entry layout, in the launch
    configuration the benchmark times): sampled forward outputs against the
    FP64 oracle within the 16-bit-weight bar, 5e-3 relative L2."""
    ap = config("pact256")
    Ft = _t(phantoms.phantom(ap), torch.float32)
    Fin = _np(Ft)
    plan = _plan(ap, "f32", weight)
    Y = _np(plan.forward(Ft))
    angles, heights = [3, 260], [17, 200]
    a34 = geo.assemble_a34(ap, heights=heights)
    for a in angles:
        G = osrt.crt12(geo.assemble_a12(ap, ap.angles[a]), Fin).reshape(-1)
        for h in heights:
            rows = a34[h * ap.n_radii:(h + 1) * ap.n_radii]
            assert rel_l2(Y[a, h], rows @ G) <= 5e-3, (a, h)


def test_pact256_batch_over_4gib_matches_single():
    """A batch of 11 at 256^3 makes every stage's dense operand span 4 GiB or
    more except stage 1's forward input, so those stages stage their rows by
    global rather than buffer copies (32-bit offsets would overflow). Batch
    items must equal the single applies bitwise."""
    ap = config("pact256")
    F = _t(phantoms.phantom(ap), torch.float32)
    plan = _plan(ap, "f32")
    Y1 = plan.forward(F)
    Fp1 = plan.adjoint(Y1)
    n = 11
    L = plan.info["live_radii"]
    assert L * ap.mz * n * ap.n_angles * 4 >= 1 << 32  # stage-2 forward operand
    Fb = torch.stack([F * (1.0 + 0.25 * i) for i in range(n)])
    Fb[0] = F
    Fb[-1] = F
    Yb = plan.forward(Fb)
    assert torch.equal(Yb[0], Y1) and torch.equal(Yb[-1], Y1)
    Fpb = plan.adjoint(Yb)
    assert torch.equal(Fpb[0], Fp1) and torch.equal(Fpb[-1], Fp1)
    # the scaled items are scaled copies up to FP32 rounding
    assert rel_l2(_np(Yb[4]), 2.0 * _np(Y1)) <= 1e-6


# ------------------------------------------------------------------ tangent circles
def test_tangent_circles_match_oracle():
    """Circles that touch grid lines tangentially, with the edge crossings
    symmetric about the touching point (columns on voxel-centre and grid
    lines, radii multiples of the pitch): FP64 operator entries."""
    from srt_inputs import column_aperture
    h = 0.125
    centers = [(h / 2, 0.0), (0.0, h / 2), (h / 2, h / 2), (0.0, 0.0), (1.5, 0.0)]
    ap = column_aperture("tan", 16, 1.0, centers, 9, 24, l_max=3.0)
    assert np.allclose(ap.radii / h, np.round(ap.radii / h))
    a12s, a34 = geo.assemble_all(ap)
    plan = _plan(ap, "f64")
    r, c, v = plan.export_coo(0)
    A = sp.csr_matrix((v, (r, c)), shape=(ap.n_angles * ap.n_radii, ap.ms ** 2))
    assert abs(A - stacked(a12s)).max() <= 1e-12 * h
    live = plan.info["live_radii"]
    r, c, v = plan.export_coo(1)
    B = sp.csr_matrix((v, (r, c)), shape=(ap.n_z * ap.n_radii, live * ap.mz))
    assert abs(B - a34[:, :live * ap.mz]).max() <= 1e-12 * h


def test_pact256_square_columns_sampled():
    """At 256^3 with the 512 columns spaced along a square instead of the
    cylinder (the bench's --aperture square): sampled forward outputs and the
    adjoint of data on two columns against the oracle (FP32 plan)."""
    from srt_inputs import square_columns
    ap0 = config("pact256")
    ap = square_columns(ap0, ap0.radius)
    F = _t(phantoms.phantom(ap0), torch.float32)
    Fin = _np(F)
    plan = _plan(ap, "f32")
    Y = _np(plan.forward(F))
    cols, heights = [0, 130, 333], [40, 220]
    a34 = geo.assemble_a34(ap, heights=heights)
    a12 = {a: geo.assemble_a12_at(ap, ap.column_centers[a]) for a in cols}
    for a in cols:
        G = osrt.crt12(a12[a], Fin).reshape(-1)
        for h in heights:
            rows = a34[h * ap.n_radii:(h + 1) * ap.n_radii]
            assert rel_l2(Y[a, h], rows @ G) <= 1e-5, (a, h)
    data = np.zeros(ap.data_shape)
    rng = np.random.default_rng(2007)
    for a in cols[:2]:
        for h in heights:
            data[a, h] = rng.standard_normal(ap.n_radii)
    dt = _t(data, torch.float32)
    Fp = _np(plan.adjoint(dt))
    din = _np(dt)
    ref = np.zeros(ap.vol_shape)
    for a in cols[:2]:
        ref += osrt.crt12_t(a12[a], osrt.crt34_t(a34, din[a], ap.mz), ap.ms)
    assert rel_l2(Fp, ref) <= 1e-5


# ------------------------------------------------------------------ columns anywhere
COLUMN_SETS = {
    # a linear array below the grid, and a scatter with columns inside the
    # grid, on a grid line and on a pixel corner
    "linear": [(x, -1.45) for x in np.linspace(-1.2, 1.2, 12)],
    "scatter": [(0.13, -0.41), (0.25, 0.5), (-0.5, -0.5), (2.7, -0.3), (-0.01, 1.9),
                (1.2, 1.1), (-1.6, 0.2)],
}


@pytest.mark.parametrize("which", sorted(COLUMN_SETS))
def test_arbitrary_columns_match_oracle(which):
    """srt_plan_create_columns: operator entries (FP64) and FP64 / FP32
    forward and adjoint against the oracle for columns off any cylinder."""
    from srt_inputs import column_aperture
    ap = column_aperture(which, 24, 1.0, COLUMN_SETS[which], 9, 40, mz=20)
    a12s, a34 = geo.assemble_all(ap)
    plan = _plan(ap, "f64")
    r, c, v = plan.export_coo(0)
    A = sp.csr_matrix((v, (r, c)), shape=(ap.n_angles * ap.n_radii, ap.ms ** 2))
    assert abs(A - stacked(a12s)).max() <= 1e-12 * ap.dxy
    rng = np.random.default_rng(41)
    vols = rng.uniform(-1, 1, (2,) + ap.vol_shape)
    data = rng.standard_normal((2,) + ap.data_shape)
    for value, tol in (("f64", 1e-12), ("f32", 1e-5)):
        dt = torch.float64 if value == "f64" else torch.float32
        p = plan if value == "f64" else _plan(ap, value)
        vt, dtt = _t(vols, dt), _t(data, dt)
        assert rel_l2(_np(p.forward(vt)), oracle_forward(ap, a12s, a34, _np(vt))) <= tol
        assert rel_l2(_np(p.adjoint(dtt)), oracle_adjoint(ap, a12s, a34, _np(dtt))) <= tol
