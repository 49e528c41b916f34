"""Scan geometries, phantom recipes and solver parameters for the DECT workloads.

Conventions (a specification shared by the GPU library and the CPU oracle,
each of which implements it in its own code):

* Image pixel (r, c): r is the row (y), c the column (x), stored row-major with
  c fastest.  Pixel centres sit at x_c = (c - (nx-1)/2) * pixel and
  y_r = (r - (ny-1)/2) * pixel, so the image is centred on the isocentre.
* View v has angle theta_v = 2*pi*v / n_views (counter-clockwise, theta_0 = 0)
  unless explicit angles are given.
* Source at sod * (cos theta, sin theta).  Flat detector line centred at
  -(sdd - sod) * (cos theta, sin theta) with axis e_u = (-sin theta, cos theta);
  bin b is centred at u_b = (b - (n_bins-1)/2) * bin + det_offset.
* Sinogram layout [n_views][n_bins], bin fastest.

The paper's real scanner (Sec. 3) is a cone-beam CBCT of which only the central
slice is used: a 2-D fan beam onto a flat 1-D detector line.  The workloads
below are synthetic stand-ins of that shape.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

# Linear attenuation coefficients in 1/mm of the two basis materials at the two
# tube energies (Eq. 12 notation: eta_{material, energy}).
MU_WATER_HIGH = 0.0180
MU_WATER_LOW = 0.0227
MU_BONE_HIGH = 0.048
MU_BONE_LOW = 0.080


@dataclasses.dataclass(frozen=True)
class Geometry:
    """2-D fan-beam geometry with a flat detector line (Sec. 2.1, Fig. 1; Sec. 3)."""

    nx: int
    ny: int
    pixel_mm: float
    n_views: int
    n_bins: int
    bin_mm: float
    sod_mm: float
    sdd_mm: float
    det_offset_mm: float = 0.0
    angles_rad: Optional[Sequence[float]] = None
    model: int = 0  # ray model of A: 0 Joseph (interpolating), 1 Siddon (pixel intersection lengths)

    @property
    def n_pixels(self) -> int:
        return self.nx * self.ny

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_bins

    def angles(self):
        if self.angles_rad is not None:
            return [float(a) for a in self.angles_rad]
        return [2.0 * math.pi * v / self.n_views for v in range(self.n_views)]

    def fov_radius_mm(self) -> float:
        """Radius of the circle every ray fan covers (the measured field of view)."""
        half = 0.5 * self.n_bins * self.bin_mm + abs(self.det_offset_mm)
        return self.sod_mm * math.sin(math.atan(half / self.sdd_mm))

    def with_views(self, n_views: int) -> "Geometry":
        return dataclasses.replace(self, n_views=n_views, angles_rad=None)


@dataclasses.dataclass(frozen=True)
class ConeGeometry:
    """3-D circular cone beam with a flat detector panel (the scanner of Sec. 3;
    Geometry is its central plane).  Volume [nz][ny][nx] of cubic voxels
    centred on the isocentre; projections [n_views][n_rows][n_bins]; detector
    rows along z, row j at (j - (n_rows-1)/2) * row_mm."""

    nx: int
    ny: int
    nz: int
    voxel_mm: float
    n_views: int
    n_bins: int
    n_rows: int
    bin_mm: float
    row_mm: float
    sod_mm: float
    sdd_mm: float
    det_offset_mm: float = 0.0
    angles_rad: Optional[Sequence[float]] = None

    def central_plane(self) -> "Geometry":
        """The 2-D fan-beam geometry of the source's plane (z = 0)."""
        return Geometry(nx=self.nx, ny=self.ny, pixel_mm=self.voxel_mm, n_views=self.n_views,
                        n_bins=self.n_bins, bin_mm=self.bin_mm, sod_mm=self.sod_mm,
                        sdd_mm=self.sdd_mm, det_offset_mm=self.det_offset_mm,
                        angles_rad=self.angles_rad)


@dataclasses.dataclass(frozen=True)
class AdmParams:
    """Parameters of the TV-regularised ADM reconstruction (Eqs. 3-10, Sec. 2.4).

    mu weights the data term (Eq. 4), rho is the augmented-Lagrangian penalty
    (Eq. 6), xi is the multiplier step (Eq. 7), beta_high/beta_low are the
    noise-balancing scalars of Eq. 3.
    """

    mu: float
    rho: float
    xi: float
    beta_high: float = 1.0
    beta_low: float = 1.0
    max_iter: int = 50
    tol: float = 0.0
    nonneg: bool = False  # project every f-step onto f >= 0
    coupled_tv: bool = False  # TV over both energies' gradients jointly (tol must be 0)
    step: str = "bb1"  # Barzilai-Borwein rule: "bb1", "bb2" or "abb" (adaptive)


@dataclasses.dataclass(frozen=True)
class PlsParams:
    """Parameters of the penalised least-squares decomposition (Eqs. 11-15)."""

    eta_water_high: float = MU_WATER_HIGH
    eta_bone_high: float = MU_BONE_HIGH
    eta_water_low: float = MU_WATER_LOW
    eta_bone_low: float = MU_BONE_LOW
    gamma: float = 1.0
    edge_eps: float = 0.1
    edge_tau: float = 0.25
    max_iter: int = 500
    tol: float = 1e-6
    mode: int = 0  # 0: Eq. 15 as printed (image space), 1: |x - Du|^2 + gamma R (attenuation space)


# --- Workload geometries -----------------------------------------------------

# Plain method, tiny: 128x128, 1 mm pixels, 60 views over 360 degrees,
# 192 bins of 1.2 mm, SOD 500 mm, SDD 1000 mm.
TINY = Geometry(nx=128, ny=128, pixel_mm=1.0, n_views=60, n_bins=192,
                bin_mm=1.2, sod_mm=500.0, sdd_mm=1000.0)
TINY_OBJECT_RADIUS_MM = 51.5


def paper_geometry(n: int = 512, n_views: int = 360, n_bins: Optional[int] = None) -> Geometry:
    """Paper-scale fan geometry: the tiny fan with its lengths doubled.

    SOD 1000 mm, SDD 2000 mm, 2.4 mm bins, 1 mm pixels; 736 bins at 512^2 and
    round(1.4375 * n) bins for other image sides.
    """
    if n_bins is None:
        n_bins = int(round(1.4375 * n))
    return Geometry(nx=n, ny=n, pixel_mm=1.0, n_views=n_views, n_bins=n_bins,
                    bin_mm=2.4, sod_mm=1000.0, sdd_mm=2000.0)


def object_radius_mm(geom: Geometry) -> float:
    """Radius scale of the ellipse phantoms drawn for a geometry."""
    if geom.sod_mm == TINY.sod_mm and geom.nx == 128:
        return TINY_OBJECT_RADIUS_MM
    return 230.0 * geom.nx / 512.0


def paper_cone_geometry(n: int = 512, nz: int = 64, n_views: int = 360,
                        n_rows: int = 64) -> ConeGeometry:
    """Multi-row version of paper_geometry: the same fan (SOD 1000 mm, SDD
    2000 mm, 2.4 mm bins, 1 mm voxels) with n_rows rows of 2.4 mm, which
    cover n_rows * 1.2 mm of height at the isocentre, and nz slices."""
    return ConeGeometry(nx=n, ny=n, nz=nz, voxel_mm=1.0, n_views=n_views,
                        n_bins=int(round(1.4375 * n)), n_rows=n_rows, bin_mm=2.4, row_mm=2.4,
                        sod_mm=1000.0, sdd_mm=2000.0)


METRIC = paper_geometry(512, 360)          # ADM-TV iterations/s are quoted here
PAPER_SPARSE = paper_geometry(512, 90)
PAPER_FULL = paper_geometry(512, 720)
UNROLLED = paper_geometry(512, 180)
CONE = paper_cone_geometry(512, 64, 360, 64)  # cone-beam projector pair timings

BATCH_SIZES = (256, 384, 512)
BATCH_VIEWS = (60, 90, 180, 360)


def default_adm_params(geom: Geometry, max_iter: int = 50) -> AdmParams:
    """Frozen ADM parameters.

    rho is in the paper's 2^2..2^10 range (Sec. 2.4) and mu grows as the view
    count falls (mu = 45 / V at paper scale, mu = 1 for the 128^2 fan); xi =
    rho / 4 keeps the BB iteration stable under FP32 rounding;
    beta_low/beta_high = sigma_high/sigma_low of the synthetic noise.
    """
    mu = 45.0 / geom.n_views
    if geom.nx == 128 and geom.sod_mm == TINY.sod_mm:
        mu = 1.0
    return AdmParams(mu=mu, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79,
                     max_iter=max_iter)
