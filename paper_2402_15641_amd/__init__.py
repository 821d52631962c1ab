"""MI355X library for the discrete spherical Radon transform on a cylindrical
aperture: two circular Radon transforms (Sec. 2) held as sparse operators on
the device, a forward (Alg. 1) and its exactly matched adjoint (Alg. 2).

    from paper_2402_15641_amd import SRTPlan
    plan = SRTPlan.from_geometry(aperture, value_dtype="f32", weight_dtype="bf16")
    data = plan.forward(vol)          # [B][n_angles][n_z][n_radii]
    back = plan.adjoint(data)         # [B][mz][ms][ms]

binding.py mirrors the C ABI of include/srt.h function by function.
"""
from . import binding  # noqa: F401


def __getattr__(name):
    # torch-dependent pieces load lazily so the ABI can be inspected without torch
    if name == "SRTPlan":
        from .srt import SRTPlan
        return SRTPlan
    raise AttributeError(name)
