"""Thin Python binding of libsrt (include/srt.h): argument marshalling only.

The functions below carry the C ABI's names. Tensors are torch tensors on a
ROCm device; only their data pointers and the current HIP stream cross the
boundary. Every arithmetic step runs in the HIP library; if the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrt.so")

SRT_OK, SRT_EINVAL, SRT_ENOMEM, SRT_EDEVICE, SRT_ENOTSUP = range(5)
STATUS_NAMES = {0: "SRT_OK", 1: "SRT_EINVAL", 2: "SRT_ENOMEM", 3: "SRT_EDEVICE", 4: "SRT_ENOTSUP"}
DTYPES = {"f32": 0, "f64": 1, "bf16": 2, "f16": 3}
MODES = {"auto": 0, "stored": 1, "onthefly": 2}
BASES = {"constant": 0, "linear": 1}

# Every entry point declared in include/srt.h.
SYMBOLS = ("srt_plan_create", "srt_plan_create_columns", "srt_plan_create_desc", "srt_forward", "srt_adjoint", "srt_forward_noalloc", "srt_plan_destroy",
           "srt_plan_footprint", "srt_plan_get_info", "srt_plan_export_coo",
           "srt_plan_set_timing", "srt_plan_stage_times", "srt_cgls", "srt_cgls_workspace",
           "srt_nnls", "srt_nnls_workspace", "srt_opnorm2", "srt_last_error")
STAGES = 5


class SrtGrid(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_int32), ("mz", ctypes.c_int32), ("x0", ctypes.c_double),
                ("z0", ctypes.c_double), ("dxy", ctypes.c_double), ("dz", ctypes.c_double)]


class SrtPlanInfo(ctypes.Structure):
    _fields_ = [("nnz_a12", ctypes.c_int64), ("nnz_a34", ctypes.c_int64),
                ("live_radii", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("n_z", ctypes.c_int32), ("n_radii", ctypes.c_int32),
                ("weight_scale_a12", ctypes.c_double), ("weight_scale_a34", ctypes.c_double),
                ("basis", ctypes.c_int32), ("n_rho", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("operator_bytes", ctypes.c_int64)]


class SrtPlanDesc(ctypes.Structure):
    _fields_ = [("grid", SrtGrid), ("basis", ctypes.c_int), ("cyl_radius", ctypes.c_double),
                ("angles", ctypes.c_void_p), ("col_xy", ctypes.c_void_p),
                ("n_cols", ctypes.c_int32), ("z_pos", ctypes.c_void_p), ("n_z", ctypes.c_int32),
                ("radii", ctypes.c_void_p), ("n_radii", ctypes.c_int32),
                ("rho", ctypes.c_void_p), ("n_rho", ctypes.c_int32),
                ("value_dtype", ctypes.c_int), ("weight_dtype", ctypes.c_int),
                ("mode", ctypes.c_int), ("device", ctypes.c_int32)]


class SRTError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libsrt.so (built by paper_2402_15641_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2402_15641_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I32, I64, SZ = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                          ctypes.c_size_t)
    L.srt_plan_create.argtypes = [ctypes.POINTER(SrtGrid), D, P, I32, P, I32, P, I32, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, I32, P, ctypes.POINTER(P)]
    L.srt_plan_create_columns.argtypes = [ctypes.POINTER(SrtGrid), P, I32, P, I32, P, I32,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, I32, P,
                                          ctypes.POINTER(P)]
    L.srt_plan_create_desc.argtypes = [ctypes.POINTER(SrtPlanDesc), P, ctypes.POINTER(P)]
    L.srt_forward.argtypes = [P, P, P, I32, P, SZ, P]
    L.srt_adjoint.argtypes = [P, P, P, I32, P, SZ, P]
    L.srt_forward_noalloc.argtypes = [P, P, P, I32, P]
    L.srt_plan_destroy.argtypes = [P]
    L.srt_plan_footprint.argtypes = [P, I32, ctypes.POINTER(SZ), ctypes.POINTER(SZ)]
    L.srt_plan_get_info.argtypes = [P, ctypes.POINTER(SrtPlanInfo)]
    L.srt_plan_export_coo.argtypes = [P, I32, I64, ctypes.POINTER(I64), P, P, P]
    L.srt_plan_set_timing.argtypes = [P, I32]
    L.srt_plan_stage_times.argtypes = [P, I32, I32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(I32)]
    L.srt_cgls.argtypes = [P, P, P, I32, I32, P, P, SZ, P]
    L.srt_cgls_workspace.argtypes = [P, I32, I32, ctypes.POINTER(SZ)]
    L.srt_nnls.argtypes = [P, P, P, I32, I32, D, P, P, SZ, P]
    L.srt_nnls_workspace.argtypes = [P, I32, I32, ctypes.POINTER(SZ)]
    L.srt_opnorm2.argtypes = [P, I32, ctypes.POINTER(D), P, SZ, P]
    for name in SYMBOLS[:-1]:
        getattr(L, name).restype = ctypes.c_int
    L.srt_last_error.argtypes = []
    L.srt_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def srt_last_error() -> str:
    return lib().srt_last_error().decode(errors="replace")


def _check(status: int, where: str):
    if status != SRT_OK:
        raise SRTError(status, where, srt_last_error())


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def srt_plan_create(ms, mz, x0, z0, dxy, dz, cyl_radius, angles, z_pos, radii,
                    value_dtype="f32", weight_dtype="f32", mode="auto", device=0,
                    stream=None) -> int:
    """Builds a plan; returns its opaque handle (an integer)."""
    L = lib()
    grid = SrtGrid(int(ms), int(mz), float(x0), float(z0), float(dxy), float(dz))
    ang, zp, rad = _f64(angles), _f64(z_pos), _f64(radii)
    out = ctypes.c_void_p()
    st = L.srt_plan_create(ctypes.byref(grid), float(cyl_radius), ang.ctypes.data, ang.size,
                           zp.ctypes.data, zp.size, rad.ctypes.data, rad.size,
                           DTYPES[value_dtype], DTYPES[weight_dtype], MODES[mode], int(device),
                           _stream_ptr(stream) if stream is not False else None,
                           ctypes.byref(out))
    _check(st, "srt_plan_create")
    return out.value


def srt_plan_create_columns(ms, mz, x0, z0, dxy, dz, col_xy, z_pos, radii,
                            value_dtype="f32", weight_dtype="f32", mode="auto", device=0,
                            stream=None) -> int:
    """Builds a plan for sensor columns at arbitrary (x, y) positions
    (col_xy: n x 2); returns its opaque handle."""
    L = lib()
    grid = SrtGrid(int(ms), int(mz), float(x0), float(z0), float(dxy), float(dz))
    xy, zp, rad = _f64(col_xy).reshape(-1, 2), _f64(z_pos), _f64(radii)
    xy = np.ascontiguousarray(xy)
    out = ctypes.c_void_p()
    st = L.srt_plan_create_columns(ctypes.byref(grid), xy.ctypes.data, xy.shape[0],
                                   zp.ctypes.data, zp.size, rad.ctypes.data, rad.size,
                                   DTYPES[value_dtype], DTYPES[weight_dtype], MODES[mode],
                                   int(device), _stream_ptr(stream) if stream is not False else None,
                                   ctypes.byref(out))
    _check(st, "srt_plan_create_columns")
    return out.value


def srt_plan_create_desc(ms, mz, x0, z0, dxy, dz, z_pos, radii, basis="constant",
                         cyl_radius=0.0, angles=None, col_xy=None, rho=None,
                         value_dtype="f32", weight_dtype="f32", mode="auto", device=0,
                         stream=None) -> int:
    """Builds a plan from a full description: voxel basis ("constant" or
    "linear"), a cylinder aperture (cyl_radius, angles) or columns at col_xy
    (n x 2), and optionally a stage-2 radial grid rho of its own."""
    L = lib()
    keep = []  # host arrays must outlive the call

    def arr(a, shape=None):
        if a is None:
            return None, 0
        v = _f64(a) if shape is None else np.ascontiguousarray(_f64(a).reshape(shape))
        keep.append(v)
        return v.ctypes.data, (v.shape[0] if v.ndim > 1 else v.size)

    ang, n_ang = arr(angles)
    xy, n_xy = arr(col_xy, (-1, 2))
    zp, n_z = arr(z_pos)
    rad, n_rad = arr(radii)
    rh, n_rh = arr(rho)
    d = SrtPlanDesc(SrtGrid(int(ms), int(mz), float(x0), float(z0), float(dxy), float(dz)),
                    BASES[basis], float(cyl_radius), ang, xy, n_ang if ang is not None else n_xy,
                    zp, n_z, rad, n_rad, rh, n_rh, DTYPES[value_dtype], DTYPES[weight_dtype],
                    MODES[mode], int(device))
    out = ctypes.c_void_p()
    st = L.srt_plan_create_desc(ctypes.byref(d),
                                _stream_ptr(stream) if stream is not False else None,
                                ctypes.byref(out))
    _check(st, "srt_plan_create_desc")
    return out.value


def srt_plan_destroy(plan: int) -> None:
    _check(lib().srt_plan_destroy(plan), "srt_plan_destroy")


def srt_forward(plan: int, vol, data, batch: int, workspace=None, stream=None) -> None:
    """data[b][a][h][l] <- Alg. 1 of vol[b][k][j][i] (device tensors)."""
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(),
                                                              workspace.numel() * workspace.element_size())
    _check(lib().srt_forward(plan, vol.data_ptr(), data.data_ptr(), int(batch), ws_ptr, ws_bytes,
                             _stream_ptr(stream)), "srt_forward")


def srt_adjoint(plan: int, data, vol, batch: int, workspace=None, stream=None) -> None:
    """vol[b][k][j][i] <- Alg. 2 (summed over columns) of data[b][a][h][l]."""
    ws_ptr, ws_bytes = (None, 0) if workspace is None else (workspace.data_ptr(),
                                                              workspace.numel() * workspace.element_size())
    _check(lib().srt_adjoint(plan, data.data_ptr(), vol.data_ptr(), int(batch), ws_ptr, ws_bytes,
                             _stream_ptr(stream)), "srt_adjoint")


def srt_forward_noalloc(plan: int, vol, data, batch: int, stream=None) -> None:
    """srt_forward over the library's own fixed scratch array (no allocation)."""
    _check(lib().srt_forward_noalloc(plan, vol.data_ptr(), data.data_ptr(), int(batch),
                                     _stream_ptr(stream)), "srt_forward_noalloc")


def srt_plan_footprint(plan: int, batch: int):
    """(resident bytes, workspace bytes for `batch` items)."""
    r, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().srt_plan_footprint(plan, int(batch), ctypes.byref(r), ctypes.byref(w)),
           "srt_plan_footprint")
    return r.value, w.value


def srt_plan_get_info(plan: int) -> dict:
    info = SrtPlanInfo()
    _check(lib().srt_plan_get_info(plan, ctypes.byref(info)), "srt_plan_get_info")
    return {k: getattr(info, k) for k, _ in SrtPlanInfo._fields_}


def srt_plan_export_coo(plan: int, which: int):
    """One stored operator as host COO arrays (rows, cols, arc lengths)."""
    L = lib()
    nnz = ctypes.c_int64()
    _check(L.srt_plan_export_coo(plan, int(which), 0, ctypes.byref(nnz), None, None, None),
           "srt_plan_export_coo")
    n = nnz.value
    rows = np.zeros(n, np.int32)
    cols = np.zeros(n, np.int32)
    vals = np.zeros(n, np.float64)
    if n:
        _check(L.srt_plan_export_coo(plan, int(which), n, ctypes.byref(nnz), rows.ctypes.data,
                                     cols.ctypes.data, vals.ctypes.data), "srt_plan_export_coo")
    return rows, cols, vals


def srt_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().srt_plan_set_timing(plan, 1 if enable else 0), "srt_plan_set_timing")


def srt_plan_stage_times(plan: int, adjoint: bool):
    """(summed milliseconds per stage, number of timed applies)."""
    tot = (ctypes.c_double * STAGES)()
    n = ctypes.c_int32()
    _check(lib().srt_plan_stage_times(plan, 1 if adjoint else 0, STAGES, tot, ctypes.byref(n)),
           "srt_plan_stage_times")
    return list(tot), n.value


def srt_cgls_workspace(plan: int, batch: int, n_iter: int) -> int:
    """Workspace bytes srt_cgls needs."""
    b = ctypes.c_size_t()
    _check(lib().srt_cgls_workspace(plan, int(batch), int(n_iter), ctypes.byref(b)),
           "srt_cgls_workspace")
    return b.value


def srt_cgls(plan: int, vol, data, batch: int, n_iter: int, workspace, want_resid=True,
             stream=None):
    """n_iter CGLS iterations in place on vol (device tensors); returns the
    residual norms ||A^T (g - A f_k)|| as an (n_iter + 1, batch) array, or
    None when want_resid is False (then the call is asynchronous)."""
    resid = np.zeros((int(n_iter) + 1, int(batch)), np.float64) if want_resid else None
    _check(lib().srt_cgls(plan, vol.data_ptr(), data.data_ptr(), int(batch), int(n_iter),
                          None if resid is None else resid.ctypes.data, workspace.data_ptr(),
                          workspace.numel() * workspace.element_size(), _stream_ptr(stream)),
           "srt_cgls")
    return resid


def srt_nnls_workspace(plan: int, batch: int, n_iter: int) -> int:
    """Workspace bytes srt_nnls needs (batch 1, n_iter 0: what srt_opnorm2 needs)."""
    b = ctypes.c_size_t()
    _check(lib().srt_nnls_workspace(plan, int(batch), int(n_iter), ctypes.byref(b)),
           "srt_nnls_workspace")
    return b.value


def srt_nnls(plan: int, vol, data, batch: int, n_iter: int, step: float, workspace,
             want_resid=True, stream=None):
    """n_iter FISTA steps for min ||A f - g||^2, f >= 0, in place on vol;
    returns the misfits ||A y_k - g|| as an (n_iter, batch) array, or None
    when want_resid is False (then the call is asynchronous)."""
    resid = np.zeros((int(n_iter), int(batch)), np.float64) if want_resid else None
    _check(lib().srt_nnls(plan, vol.data_ptr(), data.data_ptr(), int(batch), int(n_iter),
                          float(step), None if resid is None else resid.ctypes.data,
                          workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                          _stream_ptr(stream)), "srt_nnls")
    return resid


def srt_opnorm2(plan: int, n_iter: int, workspace, stream=None) -> float:
    """Power-method estimate of ||A||_2^2 after n_iter steps (waits for the stream)."""
    out = ctypes.c_double()
    _check(lib().srt_opnorm2(plan, int(n_iter), ctypes.byref(out), workspace.data_ptr(),
                             workspace.numel() * workspace.element_size(), _stream_ptr(stream)),
           "srt_opnorm2")
    return out.value
