"""Voxel grids and cylindrical sensor apertures of the synthetic workloads.

A cylindrical aperture is a set of sensor columns parallel to the z axis on a
circle of radius R about the z axis (Sec. 2: sensors on one z-parallel line
share the first circular transform). Column a sits at angle alpha_a; every
column carries the same sensor heights z_h and the same sphere radii l_l
(Alg. 1 inputs).

Readings of what the paper leaves open (all stated once here):
  * voxels are cell-centred on the cube [-W, W]^3 with M voxels per axis;
  * alpha_a = 2*pi*a/N_a (uniform on [0, 2*pi));
  * z_h = linspace(-W, W, N_h), end points included;
  * l_l = l * l_max / N_l for l = 1..N_l (uniform on (0, l_max]);
  * where a workload gives no l_max, l_max is the distance from a sensor to
    the farthest voxel corner, sqrt((R + sqrt(2) W)^2 + (2W)^2).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Aperture:
    """A voxel grid plus a cylindrical aperture. Lengths share one unit."""

    name: str
    ms: int  # voxels along x and along y
    mz: int  # voxels along z
    x0: float  # lower corner of the grid in x and in y
    z0: float  # lower corner of the grid in z
    dxy: float  # voxel pitch in x and y
    dz: float  # voxel pitch in z
    radius: float  # cylinder radius R
    angles: np.ndarray = field(repr=False)  # [N_a] radians
    zpos: np.ndarray = field(repr=False)  # [N_h]
    radii: np.ndarray = field(repr=False)  # [N_l], strictly increasing, > 0
    # Columns anywhere in the (x, y) plane ([N_a][2]); None: on the cylinder
    # at (R cos alpha_a, R sin alpha_a).
    centers: np.ndarray | None = field(default=None, repr=False)
    # Radial grid of the stage-2 image ([N_rho], strictly increasing, > 0);
    # None: the sphere radii themselves (the paper's choice).
    rho: np.ndarray | None = field(default=None, repr=False)

    @property
    def rho_grid(self) -> np.ndarray:
        """[N_rho] radii at which stage 1 evaluates the circle transform."""
        return np.asarray(self.radii if self.rho is None else self.rho, dtype=np.float64)

    @property
    def n_rho(self) -> int:
        return int(self.rho_grid.size)

    @property
    def column_centers(self) -> np.ndarray:
        """[N_a][2] (x, y) of every sensor column."""
        if self.centers is not None:
            return np.asarray(self.centers, dtype=np.float64)
        return np.stack([self.radius * np.cos(self.angles), self.radius * np.sin(self.angles)], axis=1)

    @property
    def n_angles(self) -> int:
        return int(self.angles.size)

    @property
    def n_z(self) -> int:
        return int(self.zpos.size)

    @property
    def n_radii(self) -> int:
        return int(self.radii.size)

    @property
    def vol_shape(self):
        return (self.mz, self.ms, self.ms)

    @property
    def data_shape(self):
        return (self.n_angles, self.n_z, self.n_radii)

    def summary(self) -> dict:
        return {
            "workload": self.name,
            "grid": [self.ms, self.ms, self.mz],
            "pitch": self.dxy,
            "cyl_radius": self.radius,
            "n_angles": self.n_angles,
            "n_z": self.n_z,
            "n_radii": self.n_radii,
            "l_max": float(self.radii[-1]),
        }


def farthest_corner(radius: float, half_width: float) -> float:
    """Distance from a sensor on the cylinder to the farthest grid corner."""
    return float(np.hypot(radius + np.sqrt(2.0) * half_width, 2.0 * half_width))


def cylinder_aperture(name: str, m: int, half_width: float, radius: float,
                      n_angles: int, n_z: int, n_radii: int,
                      l_max: float | None = None, mz: int | None = None) -> Aperture:
    """Cubic grid [-W, W]^3 (M^3 voxels) with a uniform cylindrical aperture."""
    mz = m if mz is None else mz
    h = 2.0 * half_width / m
    hz = 2.0 * half_width / mz
    if l_max is None:
        l_max = farthest_corner(radius, half_width)
    angles = 2.0 * np.pi * np.arange(n_angles, dtype=np.float64) / n_angles
    zpos = np.linspace(-half_width, half_width, n_z, dtype=np.float64)
    radii = l_max * np.arange(1, n_radii + 1, dtype=np.float64) / n_radii
    return Aperture(name=name, ms=m, mz=mz, x0=-half_width, z0=-half_width,
                    dxy=h, dz=hz, radius=float(radius), angles=angles,
                    zpos=zpos, radii=radii)


def with_rho_grid(ap: Aperture, n_rho: int, rho_max: float | None = None) -> Aperture:
    """The same aperture with a stage-2 radial grid of its own: N_rho uniform
    values rho_m = m * rho_max / N_rho, m = 1..N_rho (rho_max defaults to the
    largest sphere radius)."""
    rho_max = float(ap.radii[-1]) if rho_max is None else float(rho_max)
    rho = rho_max * np.arange(1, n_rho + 1, dtype=np.float64) / n_rho
    return replace(ap, name=f"{ap.name}_rho{n_rho}", rho=rho)


def square_columns(ap: Aperture, half_side: float) -> Aperture:
    """The same grid, heights and radii with the N_a sensor columns placed
    evenly along the perimeter of the square [-s, s]^2 (s = half_side)
    instead of on a circle: columns anywhere (Sec. 2 only needs z-parallel
    lines), at the size of a given workload."""
    n, s = ap.n_angles, float(half_side)
    t = 8.0 * s * (np.arange(n, dtype=np.float64) + 0.5) / n  # arc length along the perimeter
    side, u = np.divmod(t, 2.0 * s)
    u = u - s
    # counter-clockwise: side 0 x = s, y = u; side 1 y = s, x = -u;
    # side 2 x = -s, y = -u; side 3 y = -s, x = u
    xy = np.empty((n, 2))
    sides = [(np.full(n, s), u), (-u, np.full(n, s)), (np.full(n, -s), -u), (u, np.full(n, -s))]
    for k, (x, y) in enumerate(sides):
        sel = side == k
        xy[sel, 0], xy[sel, 1] = x[sel], y[sel]
    return replace(ap, name=f"{ap.name}_square", radius=float("nan"),
                   angles=np.arctan2(xy[:, 1], xy[:, 0]), centers=xy)


def column_aperture(name: str, m: int, half_width: float, centers, n_z: int, n_radii: int,
                    l_max: float | None = None, mz: int | None = None) -> Aperture:
    """Cubic grid [-W, W]^3 with sensor columns at arbitrary (x, y) positions
    (each a line of N_h sensors parallel to z, Sec. 2), sharing the heights
    and radii of a cylindrical aperture; l_max defaults to the largest
    distance from a column to a grid corner."""
    mz = m if mz is None else mz
    c = np.asarray(centers, dtype=np.float64).reshape(-1, 2)
    if l_max is None:
        corners = np.array([[sx * half_width, sy * half_width] for sx in (-1, 1) for sy in (-1, 1)])
        dxy = np.max(np.hypot(c[:, None, 0] - corners[None, :, 0], c[:, None, 1] - corners[None, :, 1]))
        l_max = float(np.hypot(dxy, 2.0 * half_width))
    ap = cylinder_aperture(name, m, half_width, 0.0, c.shape[0], n_z, n_radii, l_max=l_max, mz=mz)
    return Aperture(name=name, ms=ap.ms, mz=ap.mz, x0=ap.x0, z0=ap.z0, dxy=ap.dxy, dz=ap.dz,
                    radius=float("nan"), angles=np.arctan2(c[:, 1], c[:, 0]), zpos=ap.zpos,
                    radii=ap.radii, centers=c)


def random_aperture(seed: int, scale: int = 1) -> Aperture:
    """A small seeded geometry off every regular case, for parity sweeps:
    a grid that is not centred, with voxels that are not cubes (dz != dxy);
    1-7 columns, on a circle of random radius (inside or outside the grid)
    or scattered anywhere; 1-6 heights and 1-25 radii, unevenly spaced; and
    for one seed in three a stage-2 radial grid of its own. scale > 1
    multiplies the largest grid and sample counts (more operator tiles)."""
    rng = np.random.default_rng(seed)
    ms, mz = int(rng.integers(2, 30 * scale + 1)), int(rng.integers(1, 20 * scale + 1))
    dxy = float(rng.uniform(0.5, 1.5))
    dz = dxy * float(rng.uniform(0.6, 1.7))
    x0 = -0.5 * ms * dxy + float(rng.uniform(-2.0, 2.0)) * dxy
    z0 = -0.5 * mz * dz + float(rng.uniform(-2.0, 2.0)) * dz
    half = 0.5 * ms * dxy
    n_cols = int(rng.integers(1, 7 * scale + 1))
    if rng.uniform() < 0.5:
        R = half * float(rng.uniform(0.3, 1.6))
        ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, n_cols))
        xy = np.stack([R * np.cos(ang), R * np.sin(ang)], axis=1)
    else:
        xy = rng.uniform(-1.5 * half, 1.5 * half, (n_cols, 2))
    zlo, zhi = z0 - dz, z0 + (mz + 1) * dz
    zpos = np.sort(rng.uniform(zlo, zhi, int(rng.integers(1, 6 * scale + 1))))
    # farthest grid corner from any column, over the height range
    cx = np.array([x0, x0 + ms * dxy])
    far_xy = max(float(np.hypot(np.max(np.abs(cx - c[0])), np.max(np.abs(cx - c[1]))))
                 for c in xy)
    l_max = float(np.hypot(far_xy, zhi - zlo))

    def increasing(n, hi):
        while True:
            v = np.sort(rng.uniform(0.02 * hi, hi, n))
            if n == 1 or np.min(np.diff(v)) > 1e-6 * hi:
                return v

    radii = increasing(int(rng.integers(1, 25 * scale + 1)), l_max)
    rho = increasing(int(rng.integers(1, 30 * scale + 1)), 1.05 * l_max) if rng.uniform() < 1 / 3 else None
    return Aperture(name=f"random{seed}" + (f"x{scale}" if scale > 1 else ""), ms=ms, mz=mz, x0=x0, z0=z0, dxy=dxy, dz=dz,
                    radius=float("nan"), angles=np.arctan2(xy[:, 1], xy[:, 0]), zpos=zpos,
                    radii=radii, centers=xy, rho=rho)


CONFIG_NAMES = ("grid32", "grid128", "pact256", "serve64", "serve128", "serve192")


def config(name: str) -> Aperture:
    """The named workload geometries.

    grid32    32^3 on [-1,1]^3, R=1.5, 16 angles x 16 heights x 64 radii, l_max=3.5
    grid128   128^3 on [-1,1]^3, R=1.3, 128 x 128 x 512
    pact256   256^3 at 0.1 mm (W=12.8 mm), R=1.2 W, 512 x 256 x 1024 (PACT scale)
    serveN    N^3 on [-1,1]^3, R=1.3, N x N x 4N (serving mix, N in 64/128/192)
    """
    if name == "grid32":
        return cylinder_aperture("grid32", 32, 1.0, 1.5, 16, 16, 64, l_max=3.5)
    if name == "grid128":
        return cylinder_aperture("grid128", 128, 1.0, 1.3, 128, 128, 512)
    if name == "pact256":
        w = 12.8
        return cylinder_aperture("pact256", 256, w, 1.2 * w, 512, 256, 1024)
    if name.startswith("serve"):
        n = int(name[len("serve"):])
        return cylinder_aperture(name, n, 1.0, 1.3, n, n, 4 * n)
    raise KeyError(name)
