"""Pins of the oracle's nonnegative least squares (oracle/nnls.py) against
things other than itself, on a tiny SRT problem whose matrix is assembled
explicitly (64 voxels, 72 sensor samples) and data with negative values, so
that the constraint is active:

  * the power estimate of ||A||^2 never exceeds the largest eigenvalue of
    A^T A from a dense symmetric eigensolver (Rayleigh quotient bound) and
    converges to it;
  * the extrapolation weights come from a sequence with t_{k+1}^2 - t_{k+1}
    = t_k^2 and t_k >= (k + 1) / 2, the two facts the convergence proof uses;
  * every FISTA iterate is nonnegative and its objective gap to the solution
    of scipy.optimize.nnls (Lawson-Hanson active set, a different method)
    stays below the published bound 2 L ||f0 - f*||^2 / (k + 1)^2;
  * after many steps the iterate meets the optimality conditions (f >= 0,
    gradient >= 0 and f * gradient = 0) and the nnls objective;
  * the reported misfit of the first step is ||A f0 - g||.
"""
import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls

from oracle import geometry as geo, nnls as onn, srt
from srt_inputs import cylinder_aperture


@pytest.fixture(scope="module")
def tiny():
    ap = cylinder_aperture("tiny", 4, 1.0, 1.5, 3, 3, 8)
    a12s, a34 = geo.assemble_all(ap)
    fwd = lambda f: srt.forward(f, a12s, a34, ap.n_z, ap.n_radii)  # noqa: E731
    adj = lambda y: srt.adjoint(y, a12s, a34, ap.ms, ap.mz)  # noqa: E731
    n = int(np.prod(ap.vol_shape))
    A = np.stack([fwd(np.eye(n)[i].reshape(ap.vol_shape)).reshape(-1) for i in range(n)], axis=1)
    rng = np.random.default_rng(21)
    g = A @ rng.uniform(0, 1, n) + 0.5 * rng.standard_normal(A.shape[0])
    return ap, fwd, adj, A, g.reshape(ap.data_shape)


def _objective(A, f, g):
    r = A @ f.reshape(-1) - g.reshape(-1)
    return 0.5 * float(r @ r)


def test_power_estimate_bounded_by_and_converging_to_lambda_max(tiny):
    ap, fwd, adj, A, g = tiny
    lam = np.linalg.eigvalsh(A.T @ A)[-1]
    prev = 0.0
    for k in (1, 2, 3, 5, 10, 20, 40):
        est = onn.opnorm2(fwd, adj, ap.vol_shape, k)
        assert est <= lam * (1 + 1e-12), k
        assert est >= prev * (1 - 1e-12), k  # the power method's quotients rise
        prev = est
    assert abs(onn.opnorm2(fwd, adj, ap.vol_shape, 200) - lam) <= 1e-10 * lam


def test_momentum_sequence():
    w = onn.momentum(60)
    t = 1.0
    for k, beta in enumerate(w, start=1):
        # recover t_{k+1} from beta = (t_k - 1) / t_{k+1} (beta_1 = 0: t_2 is the
        # positive root of t^2 - t = 1)
        t_next = (t - 1.0) / beta if beta > 0 else (1.0 + np.sqrt(5.0)) / 2.0
        assert abs(t_next * t_next - t_next - t * t) <= 1e-9 * t * t, k
        assert t_next >= (k + 2) / 2.0, k
        t = t_next
    assert w[0] == 0.0 and all(0.0 <= b < 1.0 for b in w)


def test_objective_gap_within_published_bound(tiny):
    ap, fwd, adj, A, g = tiny
    L = np.linalg.eigvalsh(A.T @ A)[-1]
    f_star, _ = scipy_nnls(A, g.reshape(-1))
    F_star = _objective(A, f_star, g)
    f0 = np.zeros(ap.vol_shape)
    R2 = float(np.sum((f0.reshape(-1) - f_star) ** 2))
    for k in (1, 2, 3, 5, 10, 20, 50, 100, 200, 400):
        fk, hist = onn.fista_nn(fwd, adj, g, f0, 1.0 / L, k)
        assert fk.min() >= 0.0, k
        assert len(hist) == k
        gap = _objective(A, fk, g) - F_star
        assert gap <= 2.0 * L * R2 / (k + 1) ** 2 + 1e-12 * F_star, (k, gap)


def test_converges_to_the_nonnegative_least_squares_solution(tiny):
    ap, fwd, adj, A, g = tiny
    L = np.linalg.eigvalsh(A.T @ A)[-1]
    f_star, _ = scipy_nnls(A, g.reshape(-1))
    x_ls, *_ = np.linalg.lstsq(A, g.reshape(-1), rcond=None)
    assert x_ls.min() < -1e-3 and (f_star == 0).any()  # the constraint is active
    f, hist = onn.fista_nn(fwd, adj, g, np.zeros(ap.vol_shape), 1.0 / L, 4000)
    F, F_star = _objective(A, f, g), _objective(A, f_star, g)
    assert F - F_star <= 1e-9 * F_star
    grad = A.T @ (A @ f.reshape(-1) - g.reshape(-1))
    scale = np.abs(A.T @ g.reshape(-1)).max()
    fv = f.reshape(-1)
    assert fv.min() >= 0.0
    assert grad.min() >= -1e-6 * scale
    assert np.abs(fv * grad).max() <= 1e-6 * scale * max(fv.max(), 1e-300)
    assert hist[0] == pytest.approx(np.linalg.norm(g), rel=1e-15)  # y_1 = f0 = 0


def test_first_misfit_is_that_of_the_start(tiny):
    ap, fwd, adj, A, g = tiny
    f0 = np.random.default_rng(22).uniform(0, 1, ap.vol_shape)
    _, hist = onn.fista_nn(fwd, adj, g, f0, 1e-3, 3)
    assert hist[0] == pytest.approx(np.linalg.norm(A @ f0.reshape(-1) - g.reshape(-1)), rel=1e-12)
