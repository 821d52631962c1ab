"""Pins of the oracle's least-squares reconstruction (oracle/cgls.py) against
things other than itself, on a tiny SRT problem whose matrix is assembled
explicitly (64 voxels, 72 sensor samples):

  * the k-step iterate is the least-squares minimiser over f0 plus the Krylov
    space span{s0, (A^T A) s0, ...}, solved here by a dense least-squares
    routine on an explicit basis (the defining property of CG on the normal
    equations);
  * the data residual ||g - A f_k|| never increases;
  * the reported residual norms equal ||A^T (g - A f_k)|| recomputed from f_k;
  * from f0 = 0 the iterates converge to the minimum-norm least-squares
    solution given by the SVD.
"""
import numpy as np
import pytest

from oracle import cgls as ocg, geometry as geo, srt
from srt_inputs import cylinder_aperture


@pytest.fixture(scope="module")
def tiny():
    ap = cylinder_aperture("tiny", 4, 1.0, 1.5, 3, 3, 8)
    a12s, a34 = geo.assemble_all(ap)
    fwd = lambda f: srt.forward(f, a12s, a34, ap.n_z, ap.n_radii)  # noqa: E731
    adj = lambda y: srt.adjoint(y, a12s, a34, ap.ms, ap.mz)  # noqa: E731
    n = int(np.prod(ap.vol_shape))
    A = np.stack([fwd(np.eye(n)[i].reshape(ap.vol_shape)).reshape(-1) for i in range(n)], axis=1)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(ap.data_shape)
    return ap, fwd, adj, A, g


def test_iterate_minimises_over_krylov_space(tiny):
    ap, fwd, adj, A, g = tiny
    rng = np.random.default_rng(12)
    f0 = rng.standard_normal(ap.vol_shape)
    gv = g.reshape(-1)
    s0 = A.T @ (gv - A @ f0.reshape(-1))
    for k in (1, 2, 3):
        fk, _ = ocg.cgls(fwd, adj, g, f0, k)
        basis = [s0]
        for _ in range(k - 1):
            basis.append(A.T @ (A @ basis[-1]))
        K = np.stack(basis, axis=1)
        K /= np.linalg.norm(K, axis=0)
        c, *_ = np.linalg.lstsq(A @ K, gv - A @ f0.reshape(-1), rcond=None)
        ref = f0.reshape(-1) + K @ c
        assert np.linalg.norm(fk.reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref), k


def test_data_residual_never_increases(tiny):
    ap, fwd, adj, A, g = tiny
    prev = np.inf
    for k in range(0, 12):
        fk, _ = ocg.cgls(fwd, adj, g, np.zeros(ap.vol_shape), k)
        res = np.linalg.norm(g - fwd(fk))
        assert res <= prev * (1 + 1e-12), k
        prev = res


def test_reported_residuals_match_recomputation(tiny):
    ap, fwd, adj, A, g = tiny
    for k in (0, 3, 7):
        fk, hist = ocg.cgls(fwd, adj, g, np.zeros(ap.vol_shape), k)
        assert len(hist) == k + 1
        direct = np.linalg.norm(adj(g - fwd(fk)))
        assert abs(hist[-1] - direct) <= 1e-9 * max(direct, hist[0]), k


def test_converges_to_minimum_norm_solution(tiny):
    ap, fwd, adj, A, g = tiny
    x_mn, *_ = np.linalg.lstsq(A, g.reshape(-1), rcond=None)
    f, hist = ocg.cgls(fwd, adj, g, np.zeros(ap.vol_shape), 400)
    assert hist[-1] <= 1e-8 * hist[0]
    assert np.linalg.norm(f.reshape(-1) - x_mn) <= 1e-6 * np.linalg.norm(x_mn)
