"""Alg. 1 (forward) and Alg. 2 (matched adjoint) of the discrete SRT, FP64.

Layouts: volume F[k][j][i] (z, y, x); data Y[a][h][l] (sensor column, sensor
height, sphere radius, radius fastest). The paper states the per-column output
once as N_h x N_l and once as N_l x N_h; the reading here is [h][l], matching
the row order h N_l + l of A34.

The full-aperture adjoint is the sum over columns of Alg. 2 applied to each
column's data, which is exactly the transpose of the stacked forward.
"""
from __future__ import annotations

import numpy as np


def stage1(a12, F: np.ndarray) -> np.ndarray:
    """Alg. 1, first product: reshape F to M_s^2 x M_z (pixel by slice) and
    apply the circle transform in every slice: G = A12 F, N_rho x M_z."""
    mz = F.shape[0]
    F2 = F.reshape(mz, -1).T
    return np.asarray(a12 @ F2)


def stage2(a34, G: np.ndarray, n_z: int, n_radii: int) -> np.ndarray:
    """Alg. 1, second product: flatten G to a vector of length N_rho M_z,
    apply the half-circle transform and reshape to N_h x N_l."""
    return np.asarray(a34 @ G.reshape(-1)).reshape(n_z, n_radii)


def column_srt(F: np.ndarray, a12, a34, n_z: int, n_radii: int) -> np.ndarray:
    """Alg. 1 (ColumnSRT) for one sensor column."""
    return stage2(a34, stage1(a12, F), n_z, n_radii)


def forward(F: np.ndarray, a12s, a34, n_z: int, n_radii: int) -> np.ndarray:
    """Alg. 1 over every column of the aperture: Y[a][h][l]."""
    return np.stack([column_srt(F, a, a34, n_z, n_radii) for a in a12s])


def adj_stage2(a34, Y_a: np.ndarray, mz: int) -> np.ndarray:
    """Alg. 2, first product: G' = (A34)^T y, reshaped to N_rho x M_z (the
    radial axis of the stage-2 image; N_rho = N_l unless it has its own)."""
    return np.asarray(a34.T @ Y_a.reshape(-1)).reshape(-1, mz)


def adj_stage1(a12, Gp: np.ndarray, ms: int) -> np.ndarray:
    """Alg. 2, second product: F' = (A12)^T G', reshaped to M_z x M_s x M_s."""
    Fp = np.asarray(a12.T @ Gp)  # [p][k]
    return Fp.T.reshape(Gp.shape[1], ms, ms)


def column_adjoint(Y_a: np.ndarray, a12, a34, ms: int, mz: int) -> np.ndarray:
    """Alg. 2 (AdjColumnSRT) for one sensor column."""
    return adj_stage1(a12, adj_stage2(a34, Y_a, mz), ms)


def adjoint(Y: np.ndarray, a12s, a34, ms: int, mz: int) -> np.ndarray:
    """Alg. 2 summed over the columns of the aperture: F'[k][j][i]."""
    out = np.zeros((mz, ms, ms))
    for a, A in enumerate(a12s):
        out += column_adjoint(Y[a], A, a34, ms, mz)
    return out


def flops(a12s, a34, mz: int) -> int:
    """Multiply-adds of one forward (the adjoint does the same number)."""
    return int(sum(A.nnz for A in a12s) * mz + a34.nnz * len(a12s))
