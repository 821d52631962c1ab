"""The discrete SRT of a cylindrical aperture and its adjoint, FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline call this module; the library never does.

Sec. 2 factors the SRT of the sensors on one z-parallel column into two
circular Radon transforms. CRT12 integrates the volume over circles about the
column in every z-plane, giving an image f12 on the (rho, z) half-plane of
that column; CRT34 integrates f12 over half circles about each sensor of the
column. With the voxel basis of Sec. 3.1 both are sparse matrices
(oracle.geometry): A12_a (N_rho x M_s^2) for column a, and A34
(N_h N_l x N_rho M_z), the same for every column. So

    SRT_a f = A34 vec(A12_a F),    F[p][k] = f at pixel p of slice k,
    f12_a[m][k] = (A12_a F)[m][k], vec(f12_a)[m M_z + k] = f12_a[m][k],

and the adjoint of the whole aperture is the transpose of the map from f to
all columns' data: sum over a of (A12_a)^T unvec((A34)^T y_a). The products
below are scipy sparse products; nothing is blocked or reordered beyond
stacking the columns, so that a reader can check each line against these
formulas. The GPU path (Alg. 1 and Alg. 2) is checked against it.

Layouts: volume F[k][j][i] (z, y, x), pixel p = j M_s + i; data Y[a][h][l]
(column, sensor height, sphere radius, radius fastest), row h N_l + l of A34.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def pixels_by_slice(F: np.ndarray) -> np.ndarray:
    """F[k][j][i] as the matrix F[p][k] (pixel p = j M_s + i, slice k)."""
    return F.reshape(F.shape[0], -1).T


def crt12(a12, F: np.ndarray) -> np.ndarray:
    """CRT12 of one column: its circle transform in every z-plane,
    f12[m][k] = sum over p of A12[m, p] F[k, p] (N_rho x M_z)."""
    return np.asarray(a12 @ pixels_by_slice(F))


def crt34(a34, f12: np.ndarray, n_z: int, n_radii: int) -> np.ndarray:
    """CRT34 of one column's image: the half-circle integrals of f12 about
    every sensor, Y[h][l] = sum over (m, k) of A34[(h, l), (m, k)] f12[m][k]."""
    return np.asarray(a34 @ f12.reshape(-1)).reshape(n_z, n_radii)


def crt34_t(a34, y: np.ndarray, mz: int) -> np.ndarray:
    """Transpose of crt34: f12'[m][k] = sum over (h, l) of A34[(h, l), (m, k)] y[h][l]."""
    return np.asarray(a34.T @ y.reshape(-1)).reshape(-1, mz)


def crt12_t(a12, f12p: np.ndarray, ms: int) -> np.ndarray:
    """Transpose of crt12: F'[k][j][i] = sum over m of A12[m, p] f12'[m][k]."""
    Fp = np.asarray(a12.T @ f12p)  # [p][k]
    return np.ascontiguousarray(Fp.T).reshape(f12p.shape[1], ms, ms)


def forward(F: np.ndarray, a12s, a34, n_z: int, n_radii: int) -> np.ndarray:
    """SRT of every column of the aperture, Y[a][h][l] = SRT_a f: the
    columns' circle transforms as one product with the stacked A12, then A34
    applied to every column's image at once."""
    na, mz = len(a12s), F.shape[0]
    f12 = np.asarray(sp.vstack(a12s).tocsr() @ pixels_by_slice(F))  # [a N_rho + m][k]
    images = f12.reshape(na, -1)  # row a: vec(f12_a)
    Y = np.ascontiguousarray(np.asarray(a34 @ images.T).T)  # [a][h N_l + l]
    return Y.reshape(na, n_z, n_radii)


def adjoint(Y: np.ndarray, a12s, a34, ms: int, mz: int) -> np.ndarray:
    """The transpose of forward: F'[k][j][i] = sum over a of
    (A12_a)^T unvec((A34)^T y_a), as two products with the transposed
    operators (the sum over columns is the product with the stacked A12)."""
    na = len(a12s)
    images = np.asarray(a34.T @ Y.reshape(na, -1).T).T  # row a: vec(f12'_a)
    Fp = np.asarray(sp.vstack(a12s).tocsr().T @ images.reshape(-1, mz))  # [p][k]
    return np.ascontiguousarray(Fp.T).reshape(mz, ms, ms)


def flops(a12s, a34, mz: int) -> int:
    """Multiply-adds of one forward (the adjoint does the same number)."""
    return int(sum(A.nnz for A in a12s) * mz + a34.nnz * len(a12s))
