"""Seeded synthetic inputs: water/bone ellipse phantoms and their sinograms.

This module is the only code that both the GPU library's tests and the CPU
oracle's tests share.  It holds none of the reconstruction method's
arithmetic (no projector, no ADM, no decomposition): it draws ellipse
phantoms, rasterises them by supersampled area fractions, and integrates them
analytically along the fan-beam rays of a geometry (chord length times
attenuation), then adds Gaussian noise.

Phantom recipe (stand-in for the paper's head phantom, Sec. 3):
* one water body ellipse, semi-axes U(0.55, 0.8) * R_obj, centre offset
  U(-0.05, 0.05) * R_obj, rotation U(0, pi);
* non-overlapping bone inserts fully inside 0.8x the body, semi-axes
  U(0.03, 0.15) * R_obj, rotation U(0, pi); an insert's value replaces water;
* attenuation of water/bone at the high/low energy from ``configs``.
Seeds: phantom = slice id; noise = 10000 + 2 * slice + energy (0 high, 1 low).
Noise sigma per energy is 0.5 % of that energy's largest clean line integral.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

from . import configs as C


@dataclasses.dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    a: float           # semi-axis along the ellipse's own x' axis (mm)
    b: float           # semi-axis along y' (mm)
    phi: float         # rotation of x' from the x axis (rad)
    mu_high: float     # attenuation added inside, 1/mm, high energy
    mu_low: float      # same, low energy
    material: int      # 1 = water, 2 = bone (for the ground-truth maps)


def _inside(el: Ellipse, x: np.ndarray, y: np.ndarray, scale: float = 1.0) -> np.ndarray:
    cp, sp = math.cos(el.phi), math.sin(el.phi)
    dx, dy = x - el.cx, y - el.cy
    xp = cp * dx + sp * dy
    yp = -sp * dx + cp * dy
    return (xp / (el.a * scale)) ** 2 + (yp / (el.b * scale)) ** 2 <= 1.0


def _boundary_points(el: Ellipse, n: int = 64) -> Tuple[np.ndarray, np.ndarray]:
    t = np.linspace(0.0, 2.0 * math.pi, n, endpoint=False)
    cp, sp = math.cos(el.phi), math.sin(el.phi)
    xp, yp = el.a * np.cos(t), el.b * np.sin(t)
    return el.cx + cp * xp - sp * yp, el.cy + sp * xp + cp * yp


def make_phantom(seed: int, r_obj: float, n_inserts=None) -> List[Ellipse]:
    """Draw a water body plus bone inserts (replacing water) from ``seed``.

    ``n_inserts`` None draws U{9..19} inserts (10-20 ellipses in all).
    Ellipse values are *differences*: the body carries water, each insert
    carries bone - water, so a ray's integral is a plain sum over ellipses.
    """
    rng = np.random.default_rng(seed)
    if n_inserts is None:
        n_inserts = int(rng.integers(9, 20))
    a = rng.uniform(0.55, 0.8) * r_obj
    b = rng.uniform(0.55, 0.8) * r_obj
    cx, cy = rng.uniform(-0.05, 0.05, size=2) * r_obj
    phi = rng.uniform(0.0, math.pi)
    body = Ellipse(cx, cy, a, b, phi, C.MU_WATER_HIGH, C.MU_WATER_LOW, 1)
    inserts: List[Ellipse] = []
    tries = 0
    while len(inserts) < n_inserts and tries < 20000:
        tries += 1
        ia = rng.uniform(0.03, 0.15) * r_obj
        ib = rng.uniform(0.03, 0.15) * r_obj
        iphi = rng.uniform(0.0, math.pi)
        # centre drawn uniformly in the 0.8x body's bounding box, then tested
        u, v = rng.uniform(-0.8, 0.8, size=2)
        cpb, spb = math.cos(phi), math.sin(phi)
        icx = cx + cpb * u * a - spb * v * b
        icy = cy + spb * u * a + cpb * v * b
        cand = Ellipse(icx, icy, ia, ib, iphi,
                       C.MU_BONE_HIGH - C.MU_WATER_HIGH, C.MU_BONE_LOW - C.MU_WATER_LOW, 2)
        bx, by = _boundary_points(cand)
        if not np.all(_inside(body, bx, by, 0.8)):
            continue
        rad = max(ia, ib)
        if any(math.hypot(icx - o.cx, icy - o.cy) < rad + max(o.a, o.b) + 1.0 for o in inserts):
            continue
        inserts.append(cand)
    return [body] + inserts


def coverage(el: Ellipse, geom: C.Geometry, supersample: int = 8) -> np.ndarray:
    """Fraction of each pixel inside the ellipse, by supersample^2 point tests.

    Pixels whose centre is farther than half a pixel diagonal from the
    boundary (measured conservatively in the ellipse's scaled frame) are
    entirely inside or outside and are not supersampled.
    """
    nx, ny, d = geom.nx, geom.ny, geom.pixel_mm
    s = supersample
    xc = (np.arange(nx) - (nx - 1) / 2.0) * d
    yc = (np.arange(ny) - (ny - 1) / 2.0) * d
    X, Y = np.meshgrid(xc, yc)
    cp, sp = math.cos(el.phi), math.sin(el.phi)
    dx, dy = X - el.cx, Y - el.cy
    rad = np.sqrt(((cp * dx + sp * dy) / el.a) ** 2 + ((-sp * dx + cp * dy) / el.b) ** 2)
    margin = 0.7072 * d / min(el.a, el.b)
    out = (rad <= 1.0 - margin).astype(np.float64)
    amb = np.nonzero((rad > 1.0 - margin) & (rad < 1.0 + margin))
    if amb[0].size:
        off = ((np.arange(s) + 0.5) / s - 0.5) * d
        ox, oy = np.meshgrid(off, off)
        px = X[amb][:, None] + ox.reshape(-1)[None, :]
        py = Y[amb][:, None] + oy.reshape(-1)[None, :]
        out[amb] = _inside(el, px, py).sum(axis=1) / float(s * s)
    return out


def rasterize(ellipses: Sequence[Ellipse], geom: C.Geometry, energy: int,
              supersample: int = 8) -> np.ndarray:
    """Pixel images of attenuation by area fraction (supersample x supersample).

    energy 0 = high, 1 = low.  Returns float64 [ny][nx] in 1/mm.
    """
    img = np.zeros((geom.ny, geom.nx))
    for el in ellipses:
        img += (el.mu_high if energy == 0 else el.mu_low) * coverage(el, geom, supersample)
    return img


def material_maps(ellipses: Sequence[Ellipse], geom: C.Geometry,
                  supersample: int = 8) -> Tuple[np.ndarray, np.ndarray]:
    """Ground-truth unitless water and bone fraction maps (Eq. 11's u)."""
    water = np.zeros((geom.ny, geom.nx))
    bone = np.zeros((geom.ny, geom.nx))
    for el in ellipses:
        cov = coverage(el, geom, supersample)
        if el.material == 1:
            water += cov
        else:
            water -= cov
            bone += cov
    return water, bone


def ray_endpoints(geom: C.Geometry) -> Tuple[np.ndarray, np.ndarray]:
    """Source and detector-bin positions of every ray, float64 [V][B][2]."""
    th = np.asarray(geom.angles(), dtype=np.float64)
    ct, st = np.cos(th), np.sin(th)
    R, D = geom.sod_mm, geom.sdd_mm
    u = (np.arange(geom.n_bins) - (geom.n_bins - 1) / 2.0) * geom.bin_mm + geom.det_offset_mm
    src = np.stack([R * ct, R * st], axis=-1)[:, None, :].repeat(geom.n_bins, axis=1)
    det = np.stack([-(D - R) * ct[:, None] - u[None, :] * st[:, None],
                    -(D - R) * st[:, None] + u[None, :] * ct[:, None]], axis=-1)
    return src, det


def chord_lengths(el: Ellipse, src: np.ndarray, det: np.ndarray) -> np.ndarray:
    """Length of the segment of each source->detector line inside the ellipse.

    The line p(t) = s + t d (|d| = 1) is mapped into the ellipse frame and
    scaled to the unit circle; the roots of A t^2 + B t + C = 0 give the
    chord sqrt(B^2 - 4AC) / A.
    """
    d = det - src
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    cp, sp = math.cos(el.phi), math.sin(el.phi)
    px, py = src[..., 0] - el.cx, src[..., 1] - el.cy
    P0x = (cp * px + sp * py) / el.a
    P0y = (-sp * px + cp * py) / el.b
    Dx = (cp * d[..., 0] + sp * d[..., 1]) / el.a
    Dy = (-sp * d[..., 0] + cp * d[..., 1]) / el.b
    A = Dx * Dx + Dy * Dy
    B = 2.0 * (P0x * Dx + P0y * Dy)
    Cc = P0x * P0x + P0y * P0y - 1.0
    disc = B * B - 4.0 * A * Cc
    return np.where(disc > 0.0, np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)


def analytic_sinogram(ellipses: Sequence[Ellipse], geom: C.Geometry, energy: int) -> np.ndarray:
    """Exact line integrals of the continuous phantom, float64 [V][B]."""
    src, det = ray_endpoints(geom)
    out = np.zeros((geom.n_views, geom.n_bins))
    for el in ellipses:
        out += (el.mu_high if energy == 0 else el.mu_low) * chord_lengths(el, src, det)
    return out


@dataclasses.dataclass
class Slice:
    """One synthetic dual-energy slice: truth images, maps and noisy sinograms."""

    geom: C.Geometry
    ellipses: List[Ellipse]
    x_true: np.ndarray        # [2][ny][nx] float64 (high, low) 1/mm
    u_true: np.ndarray        # [2][ny][nx] float64 (water, bone)
    sino_clean: np.ndarray    # [2][V][B] float64
    sino: np.ndarray          # [2][V][B] float64, with noise
    sigma: Tuple[float, float]


def make_slice(geom: C.Geometry, slice_id: int, n_inserts=None, r_obj=None,
               noise_frac: float = 0.005, supersample: int = 8) -> Slice:
    """Seeded phantom + analytic sinograms + Gaussian noise for both energies."""
    if r_obj is None:
        r_obj = C.object_radius_mm(geom)
    if n_inserts is None and geom.nx == 128:
        n_inserts = 5
    els = make_phantom(slice_id, r_obj, n_inserts)
    x = np.stack([rasterize(els, geom, e, supersample) for e in (0, 1)])
    u = np.stack(material_maps(els, geom, supersample))
    clean = np.stack([analytic_sinogram(els, geom, e) for e in (0, 1)])
    noisy = np.empty_like(clean)
    sig = []
    for e in (0, 1):
        s = noise_frac * float(clean[e].max())
        rng = np.random.default_rng(10000 + 2 * slice_id + e)
        noisy[e] = clean[e] + rng.normal(0.0, s, size=clean[e].shape)
        sig.append(s)
    return Slice(geom, els, x, u, clean, noisy, (sig[0], sig[1]))


def random_image(geom: C.Geometry, seed: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((geom.ny, geom.nx)).astype(dtype)


def random_sino(geom: C.Geometry, seed: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((geom.n_views, geom.n_bins)).astype(dtype)


def cone_volume(geom: C.ConeGeometry, seed: int, supersample: int = 4) -> np.ndarray:
    """Seeded 3-D test object [nz][ny][nx] (high-energy attenuation, 1/mm):
    the in-plane phantom of make_phantom, extruded over the central 70% of
    the volume's height (flat ends), zero above and below."""
    g2 = geom.central_plane()
    img = rasterize(make_phantom(seed, C.object_radius_mm(g2)), g2, 0, supersample)
    z = (np.arange(geom.nz) - (geom.nz - 1) / 2.0) * geom.voxel_mm
    on = (np.abs(z) <= 0.35 * geom.nz * geom.voxel_mm).astype(np.float64)
    return on[:, None, None] * img[None]
