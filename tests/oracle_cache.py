"""Per-process cache of oracle operators for the parity tests (test helper)."""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp

from oracle import geometry as geo, srt
from srt_inputs import config


@functools.lru_cache(maxsize=4)
def operators(name: str):
    ap = config(name)
    a12s, a34 = geo.assemble_all(ap)
    return ap, a12s, a34


def rel_l2(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (n if n > 0 else 1.0))


def oracle_forward(ap, a12s, a34, vols):
    """vols: [B][mz][ms][ms] float64 -> [B][na][nh][nl]."""
    return np.stack([srt.forward(v, a12s, a34, ap.n_z, ap.n_radii) for v in vols])


def oracle_adjoint(ap, a12s, a34, data):
    return np.stack([srt.adjoint(d, a12s, a34, ap.ms, ap.mz) for d in data])


def stacked(a12s):
    return sp.vstack(a12s).tocsr()
