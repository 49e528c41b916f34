"""Pins of the oracle's cone-beam Joseph projector pair (the 3-D scanner of
Sec. 3) against what fixes it independently of its 3-D code:

* the central detector row (odd row count, odd slice count) sees only the
  central slice, at zero z-weight, and equals the pinned fan-beam projector
  of that slice;
* an object constant along z is seen by a tilted row as the fan-beam
  projection scaled by the ray's 3-D length over its in-plane length, while
  the ray stays inside the volume (the bilinear z-weights sum to one);
* the dense matrices of A and A^T on a small volume are transposes, and the
  adjoint identity holds on a larger one.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

G3 = C.ConeGeometry(nx=40, ny=36, nz=21, voxel_mm=1.0, n_views=24, n_bins=70, n_rows=9,
                    bin_mm=1.3, row_mm=1.1, sod_mm=150.0, sdd_mm=300.0, det_offset_mm=0.4)


def test_central_row_is_the_fan_beam_projection():
    g = G3
    rng = np.random.default_rng(1)
    vol = rng.random((g.nz, g.ny, g.nx))
    p3 = O.project3(g, vol)
    p2 = O.project(g.central_plane(), vol[g.nz // 2])
    assert np.abs(p3[:, g.n_rows // 2, :] - p2).max() <= 1e-12 * np.abs(p2).max()


def test_z_invariant_object_scales_with_the_ray_length():
    g = C.ConeGeometry(nx=40, ny=36, nz=61, voxel_mm=1.0, n_views=12, n_bins=70, n_rows=5,
                       bin_mm=1.3, row_mm=0.7, sod_mm=150.0, sdd_mm=300.0)
    img = P.random_image(g.central_plane(), 2)
    vol = np.repeat(img[None], g.nz, axis=0)
    p3 = O.project3(g, vol)
    p2 = O.project(g.central_plane(), img)
    src, det = P.ray_endpoints(g.central_plane())
    d2 = np.linalg.norm(det - src, axis=-1)  # in-plane length source -> bin
    for j in range(g.n_rows):
        w = (j - (g.n_rows - 1) / 2.0) * g.row_mm
        scale = np.sqrt(d2 ** 2 + w ** 2) / d2
        # the ray's z stays below |w| * (R + half-diagonal) / D < 30 voxels
        assert np.abs(p3[:, j, :] - scale * p2).max() <= 1e-11 * np.abs(p2).max()


def test_dense_transpose():
    g = C.ConeGeometry(nx=6, ny=5, nz=4, voxel_mm=1.2, n_views=4, n_bins=7, n_rows=3,
                       bin_mm=1.6, row_mm=1.5, sod_mm=25.0, sdd_mm=50.0, det_offset_mm=0.2)
    N, M = g.nx * g.ny * g.nz, g.n_views * g.n_rows * g.n_bins
    A = np.stack([O.project3(g, np.eye(N)[i].reshape(g.nz, g.ny, g.nx)).reshape(-1)
                  for i in range(N)], axis=1)
    AT = np.stack([O.backproject3(g, np.eye(M)[k].reshape(g.n_views, g.n_rows, g.n_bins))
                   .reshape(-1) for k in range(M)], axis=0)
    assert np.abs(AT - A).max() <= 1e-15 * np.abs(A).max()
    assert (A > 0).sum() > 0.05 * A.size


def test_adjoint_identity():
    g = G3
    rng = np.random.default_rng(3)
    x = rng.random((g.nz, g.ny, g.nx))
    y = rng.random((g.n_views, g.n_rows, g.n_bins))
    ax = O.project3(g, x)
    lhs, rhs = float(np.sum(ax * y)), float(np.sum(x * O.backproject3(g, y)))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax) * np.linalg.norm(y)


def test_object_linear_in_z():
    """vol = z (the voxel centre's height, mm), constant in-plane.  Bilinear
    interpolation is exact for it, so on a ray whose in-plane crossings all
    lie between the first and last line centres, each plane contributes its
    path length times the height of the ray at the plane's centre:
    P = L3 * sum_i z(t_i), with z(t) = w t for a source at height 0."""
    g = C.ConeGeometry(nx=30, ny=30, nz=41, voxel_mm=1.0, n_views=10, n_bins=61, n_rows=7,
                       bin_mm=0.9, row_mm=2.0, sod_mm=120.0, sdd_mm=240.0)
    z = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.voxel_mm
    vol = np.broadcast_to(z[:, None, None], (g.nz, g.ny, g.nx)).copy()
    p3 = O.project3(g, vol)
    src, det = P.ray_endpoints(g.central_plane())
    centres = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.voxel_mm
    lim = (g.nx - 1) / 2.0 * g.voxel_mm
    checked = 0
    for v in range(g.n_views):
        for b in range(g.n_bins):
            s, e = src[v, b], det[v, b]
            d = e - s
            xm = abs(d[0]) >= abs(d[1])
            k0, k1 = (0, 1) if xm else (1, 0)
            t = (centres - s[k0]) / d[k0]           # plane centres along the driving axis
            other = s[k1] + t * d[k1]
            if np.any(np.abs(other) > lim):
                continue
            for j in range(g.n_rows):
                w = (j - (g.n_rows - 1) / 2.0) * g.row_mm
                L3 = g.voxel_mm * math.sqrt(d[0] ** 2 + d[1] ** 2 + w ** 2) / abs(d[k0])
                want = L3 * np.sum(w * t)
                assert abs(p3[v, j, b] - want) <= 1e-10 * (1.0 + abs(want))
            checked += 1
    assert checked > 50
