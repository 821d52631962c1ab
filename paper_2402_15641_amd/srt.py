"""Plan object over the C ABI: torch tensors in, torch tensors out.

The plan holds both CRT operators (and their transposes) resident on the
device. forward() is Alg. 1 over every sensor column, adjoint() is Alg. 2
summed over columns. All arithmetic happens in libsrt; this file checks
shapes and dtypes and allocates outputs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B

_TORCH = {"f32": torch.float32, "f64": torch.float64}


class SRTPlan:
    """SRT operator for sensor columns parallel to z, on one device.

    Geometry: voxel (i, j, k) covers [x0 + i dxy, ...) x [x0 + j dxy, ...) x
    [z0 + k dz, ...); sensor column a sits at (R cos angles[a], R sin angles[a])
    on a cylinder, or at col_xy[a] anywhere in the plane, with heights z_pos
    and sphere radii `radii` (strictly increasing).
    Volumes are [B][mz][ms][ms]; data are [B][n_angles][n_z][n_radii].
    """

    def __init__(self, ms, mz, x0, z0, dxy, dz, cyl_radius, angles, z_pos, radii,
                 value_dtype: str = "f32", weight_dtype: str | None = None,
                 device=None, mode: str = "auto", col_xy=None, basis: str = "constant",
                 rho=None):
        """col_xy (n x 2), when given, places the sensor columns at arbitrary
        (x, y) positions; cyl_radius and angles are then ignored. basis is
        "constant" (piecewise-constant voxels) or "linear" (volumes hold
        values at voxel centres, interpolated trilinearly). rho, when given,
        is a radial grid of the stage-2 image of its own (strictly
        increasing, > 0); by default it is the radii."""
        if weight_dtype is None:
            weight_dtype = value_dtype
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("SRTPlan needs a ROCm device")
        self.device = dev
        self.value_dtype, self.weight_dtype = value_dtype, weight_dtype
        self.dtype = _TORCH[value_dtype]
        self.ms, self.mz = int(ms), int(mz)
        n_cols = len(angles) if col_xy is None else len(col_xy)
        self.n_angles, self.n_z, self.n_radii = n_cols, len(z_pos), len(radii)
        self.basis = basis
        with torch.cuda.device(dev):
            if basis != "constant" or rho is not None:
                self.handle = B.srt_plan_create_desc(
                    ms, mz, x0, z0, dxy, dz, z_pos, radii, basis=basis, cyl_radius=cyl_radius,
                    angles=angles if col_xy is None else None, col_xy=col_xy, rho=rho,
                    value_dtype=value_dtype, weight_dtype=weight_dtype, mode=mode,
                    device=dev.index or 0)
            elif col_xy is None:
                self.handle = B.srt_plan_create(ms, mz, x0, z0, dxy, dz, cyl_radius, angles,
                                                z_pos, radii, value_dtype, weight_dtype, mode,
                                                dev.index or 0)
            else:
                self.handle = B.srt_plan_create_columns(ms, mz, x0, z0, dxy, dz, col_xy, z_pos,
                                                        radii, value_dtype, weight_dtype, mode,
                                                        dev.index or 0)
        self.info = B.srt_plan_get_info(self.handle)

    @classmethod
    def from_geometry(cls, g, **kw) -> "SRTPlan":
        """From any object with ms, mz, x0, z0, dxy, dz, radius, angles, zpos,
        radii (and optionally centers: columns at arbitrary (x, y); rho: a
        stage-2 radial grid of its own)."""
        kw.setdefault("col_xy", getattr(g, "centers", None))
        kw.setdefault("rho", getattr(g, "rho", None))
        return cls(g.ms, g.mz, g.x0, g.z0, g.dxy, g.dz, g.radius, g.angles, g.zpos, g.radii,
                   **kw)

    @property
    def vol_shape(self):
        return (self.mz, self.ms, self.ms)

    @property
    def data_shape(self):
        return (self.n_angles, self.n_z, self.n_radii)

    def _check(self, t: torch.Tensor, shape, name):
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} must be {self.dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if tuple(t.shape[-len(shape):]) != tuple(shape) or t.dim() not in (len(shape), len(shape) + 1):
            raise ValueError(f"{name} must have shape [B,]{tuple(shape)}, got {tuple(t.shape)}")
        return 1 if t.dim() == len(shape) else t.shape[0]

    def _check_out(self, out: torch.Tensor, shape, batch: int, name: str):
        # the library writes `batch` items: a smaller output would be overrun
        if self._check(out, shape, name) != batch:
            raise ValueError(f"{name} must hold {batch} item(s) of shape {tuple(shape)}, "
                             f"got {tuple(out.shape)}")

    def _check_workspace(self, ws):
        # passed on as a raw device pointer and byte count
        if ws is None:
            return
        if not isinstance(ws, torch.Tensor) or ws.device != self.device or not ws.is_contiguous():
            raise ValueError(f"workspace must be a contiguous tensor on {self.device}")

    def forward(self, vol: torch.Tensor, out: torch.Tensor | None = None, workspace=None,
                stream=None) -> torch.Tensor:
        batch = self._check(vol, self.vol_shape, "vol")
        shape = self.data_shape if vol.dim() == 3 else (batch,) + self.data_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        else:
            self._check_out(out, self.data_shape, batch, "out")
        self._check_workspace(workspace)
        if batch > 0:
            B.srt_forward(self.handle, vol, out, batch, workspace, stream)
        return out

    def adjoint(self, data: torch.Tensor, out: torch.Tensor | None = None, workspace=None,
                stream=None) -> torch.Tensor:
        batch = self._check(data, self.data_shape, "data")
        shape = self.vol_shape if data.dim() == 3 else (batch,) + self.vol_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        else:
            self._check_out(out, self.vol_shape, batch, "out")
        self._check_workspace(workspace)
        if batch > 0:
            B.srt_adjoint(self.handle, data, out, batch, workspace, stream)
        return out

    def footprint(self, batch: int = 1):
        return B.srt_plan_footprint(self.handle, batch)

    def workspace(self, batch: int = 1) -> torch.Tensor:
        """A caller-owned workspace tensor large enough for `batch` items."""
        _, ws = self.footprint(batch)
        return torch.empty(ws, dtype=torch.uint8, device=self.device)

    def cgls(self, data: torch.Tensor, n_iter: int, vol0: torch.Tensor | None = None,
             workspace=None, want_resid: bool = True, stream=None):
        """Least-squares reconstruction: n_iter CGLS iterations for
        min ||A f - data||, starting from vol0 (zeros if None). Returns
        (f, residual norms ||A^T (data - A f_k)|| per iteration and batch item)."""
        batch = self._check(data, self.data_shape, "data")
        shape = self.vol_shape if data.dim() == 3 else (batch,) + self.vol_shape
        if vol0 is None:
            f = torch.zeros(shape, dtype=self.dtype, device=self.device)
        else:
            self._check_out(vol0, self.vol_shape, batch, "vol0")
            f = vol0.clone()
        if batch == 0:
            return f, (np.zeros((int(n_iter) + 1, 0)) if want_resid else None)
        self._check_workspace(workspace)
        if workspace is None:
            workspace = torch.empty(B.srt_cgls_workspace(self.handle, batch, n_iter),
                                    dtype=torch.uint8, device=self.device)
        resid = B.srt_cgls(self.handle, f, data, batch, n_iter, workspace, want_resid, stream)
        return f, resid

    def opnorm2(self, n_iter: int = 30, workspace=None, stream=None) -> float:
        """Power-method estimate of ||A||_2^2 (largest eigenvalue of A^T A),
        a lower bound that rises towards it with n_iter."""
        self._check_workspace(workspace)
        if workspace is None:
            workspace = torch.empty(B.srt_nnls_workspace(self.handle, 1, 0), dtype=torch.uint8,
                                    device=self.device)
        return B.srt_opnorm2(self.handle, n_iter, workspace, stream)

    def nnls(self, data: torch.Tensor, n_iter: int, step: float | None = None,
             vol0: torch.Tensor | None = None, workspace=None, want_resid: bool = True,
             stream=None, power_iters: int = 30, margin: float = 1.05):
        """Nonnegative least squares min ||A f - data||^2, f >= 0: n_iter
        FISTA iterations from vol0 (zeros if None). Without a step, the step
        is 1 / (margin * opnorm2(power_iters)). Returns (f, misfits
        ||A y_k - data|| per iteration and batch item, step used)."""
        batch = self._check(data, self.data_shape, "data")
        shape = self.vol_shape if data.dim() == 3 else (batch,) + self.vol_shape
        if vol0 is None:
            f = torch.zeros(shape, dtype=self.dtype, device=self.device)
        else:
            self._check_out(vol0, self.vol_shape, batch, "vol0")
            f = vol0.clone()
        self._check_workspace(workspace)
        if step is None:
            L = self.opnorm2(power_iters, stream=stream)
            if not L > 0:
                raise ValueError("the operator is zero: no step can be derived")
            step = 1.0 / (margin * L)
        if batch == 0:
            return f, (np.zeros((int(n_iter), 0)) if want_resid else None), step
        if workspace is None:
            workspace = torch.empty(B.srt_nnls_workspace(self.handle, batch, n_iter),
                                    dtype=torch.uint8, device=self.device)
        resid = B.srt_nnls(self.handle, f, data, batch, n_iter, step, workspace, want_resid,
                           stream)
        return f, resid, step

    def export_coo(self, which: int):
        return B.srt_plan_export_coo(self.handle, which)

    def flops(self, batch: int = 1) -> int:
        """Multiply-adds of one forward (the adjoint does as many)."""
        return batch * (self.info["nnz_a12"] * self.mz + self.info["nnz_a34"] * self.n_angles)

    def close(self):
        if getattr(self, "handle", None):
            B.srt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
