"""Pins of the oracle's Siddon projector pair (exact pixel intersection
lengths, the ray model of Sec. 2.1) against geometry it must reproduce.

Siddon's matrix entry A[(v,b),(r,c)] is the length of the source-to-bin
segment inside pixel (r,c).  Every entry is checked against that length
computed another way: the line is intersected with the four edges of the
pixel square and the chord is the distance between the extreme intersection
points (no parametric clipping, no sorted crossing lists).  The row sums are
checked the same way against the whole grid rectangle, a few rays against a
brute-force supersampling of the segment, and the transpose, adjoint
identity, an axis-aligned closed form and the convergence to the analytic
line integrals of an ellipse as for the Joseph pair.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

G16 = C.Geometry(nx=16, ny=13, pixel_mm=1.1, n_views=9, n_bins=25, bin_mm=1.5, sod_mm=60.0,
                 sdd_mm=130.0, det_offset_mm=0.3, model=1)
RAGGED = C.Geometry(nx=67, ny=45, pixel_mm=1.0, n_views=37, n_bins=101, bin_mm=1.3,
                    sod_mm=300.0, sdd_mm=600.0, det_offset_mm=0.7, model=1)
TINY_S = C.Geometry(**{**C.TINY.__dict__, "model": 1})


def _edge_chord(src, det, x0, x1, y0, y1):
    """Length of the part of segment src->det inside [x0,x1] x [y0,y1]: the
    points where the line meets the rectangle's edges, clipped to the
    segment, and the distance between the two farthest apart."""
    d = det - src
    pts = []
    for xe in (x0, x1):
        if d[0] != 0.0:
            t = (xe - src[0]) / d[0]
            y = src[1] + t * d[1]
            if y0 <= y <= y1:
                pts.append(t)
    for ye in (y0, y1):
        if d[1] != 0.0:
            t = (ye - src[1]) / d[1]
            x = src[0] + t * d[0]
            if x0 <= x <= x1:
                pts.append(t)
    if len(pts) < 2:
        return 0.0
    ta, tb = max(min(pts), 0.0), min(max(pts), 1.0)
    return max(0.0, tb - ta) * float(np.hypot(d[0], d[1]))


def _pixel_box(g, r, c):
    x0 = (c - g.nx / 2.0) * g.pixel_mm
    y0 = (r - g.ny / 2.0) * g.pixel_mm
    return x0, x0 + g.pixel_mm, y0, y0 + g.pixel_mm


def _dense(g):
    N = g.nx * g.ny
    return np.stack([O.project(g, np.eye(N)[i].reshape(g.ny, g.nx)).reshape(-1)
                     for i in range(N)], axis=1)


def test_every_entry_is_the_pixel_chord():
    """A[(v,b),(r,c)] equals the chord of the ray through pixel (r,c)."""
    g = G16
    A = _dense(g)
    src, det = P.ray_endpoints(g)
    ref = np.zeros_like(A)
    for v in range(g.n_views):
        for b in range(g.n_bins):
            for r in range(g.ny):
                for c in range(g.nx):
                    ref[v * g.n_bins + b, r * g.nx + c] = _edge_chord(
                        src[v, b], det[v, b], *_pixel_box(g, r, c))
    assert np.abs(A - ref).max() <= 1e-12 * g.pixel_mm
    assert (ref > 0).sum() > 1000


@pytest.mark.parametrize("geom", [G16, RAGGED], ids=["g16", "ragged"])
def test_row_sums_are_grid_chords(geom):
    """A 1 is the length of each ray inside the whole grid rectangle."""
    g = geom
    S = O.project(g, np.ones((g.ny, g.nx)))
    src, det = P.ray_endpoints(g)
    hx, hy = 0.5 * g.nx * g.pixel_mm, 0.5 * g.ny * g.pixel_mm
    ref = np.array([[_edge_chord(src[v, b], det[v, b], -hx, hx, -hy, hy)
                     for b in range(g.n_bins)] for v in range(g.n_views)])
    assert np.abs(S - ref).max() <= 1e-11 * max(hx, hy)
    assert (ref > 0).mean() > 0.5


def test_brute_force_supersampling():
    """Per-pixel lengths of a few rays against counting 2e6 evenly spaced
    points of the segment by pixel."""
    g = C.Geometry(nx=6, ny=5, pixel_mm=1.3, n_views=3, n_bins=7, bin_mm=1.2, sod_mm=20.0,
                   sdd_mm=45.0, model=1, angles_rad=[0.3, 1.9, 4.0])
    A = _dense(g)
    src, det = P.ray_endpoints(g)
    K = 2_000_000
    t = (np.arange(K) + 0.5) / K
    for v in range(g.n_views):
        for b in (1, 3, 5):
            s, e = src[v, b], det[v, b]
            pts = s[None, :] + t[:, None] * (e - s)[None, :]
            c = np.floor(pts[:, 0] / g.pixel_mm + g.nx / 2.0).astype(np.int64)
            r = np.floor(pts[:, 1] / g.pixel_mm + g.ny / 2.0).astype(np.int64)
            inside = (c >= 0) & (c < g.nx) & (r >= 0) & (r < g.ny)
            counts = np.bincount(r[inside] * g.nx + c[inside], minlength=g.nx * g.ny)
            seg = float(np.linalg.norm(e - s))
            approx = counts * seg / K
            assert np.abs(A[v * g.n_bins + b] - approx).max() <= 4.0 * seg / K
            assert approx.sum() > 0


def test_dense_transpose():
    """matrix(A^T) from unit sinograms equals matrix(A)^T."""
    g = G16
    M = g.n_views * g.n_bins
    A = _dense(g)
    AT = np.stack([O.backproject(g, np.eye(M)[j].reshape(g.n_views, g.n_bins)).reshape(-1)
                   for j in range(M)], axis=0)
    assert np.abs(AT - A).max() <= 1e-15 * np.abs(A).max()


@pytest.mark.parametrize("geom", [TINY_S, RAGGED, G16], ids=["tiny", "ragged", "g16"])
def test_adjoint_identity(geom):
    x = P.random_image(geom, 1)
    y = P.random_sino(geom, 2)
    ax = O.project(geom, x)
    lhs = float(np.sum(ax * y))
    rhs = float(np.sum(x * O.backproject(geom, y)))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax) * np.linalg.norm(y)


def test_axis_aligned_ray_closed_form():
    """The central ray at theta = 0 runs through the middle row's centres:
    every pixel of that row is crossed over its full width."""
    g = C.Geometry(nx=15, ny=15, pixel_mm=0.7, n_views=2, n_bins=17, bin_mm=1.1, sod_mm=40.0,
                   sdd_mm=90.0, angles_rad=[0.0, math.pi / 2], model=1)
    X = P.random_image(g, 3) + 2.0
    S = O.project(g, X)
    assert abs(S[0, 8] - 0.7 * X[7, :].sum()) <= 1e-12 * abs(S[0, 8])
    assert abs(S[1, 8] - 0.7 * X[:, 7].sum()) <= 1e-12 * abs(S[1, 8])


def test_ellipse_line_integrals_converge():
    """The projection of the pixelised ellipse approaches the analytic chord
    integrals as the pixels shrink."""
    el = [P.Ellipse(3.0, -2.0, 17.0, 9.0, 0.6, 0.02, 0.03, 1)]
    errs = []
    for n in (32, 64, 128, 256):
        g = C.Geometry(nx=n, ny=n, pixel_mm=64.0 / n, n_views=24, n_bins=80, bin_mm=1.6,
                       sod_mm=150.0, sdd_mm=300.0, model=1)
        img = P.rasterize(el, g, 0, supersample=8)
        ref = P.analytic_sinogram(el, g, 0)
        errs.append(np.linalg.norm(O.project(g, img) - ref) / np.linalg.norm(ref))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-2


def test_adm_fixed_point():
    """ADM with the Siddon model: consistent data of a constant image, started
    from that image, stays put (G = 0 up to rounding)."""
    g = C.Geometry(nx=24, ny=20, pixel_mm=1.0, n_views=16, n_bins=40, bin_mm=1.2, sod_mm=80.0,
                   sdd_mm=160.0, model=1)
    x0 = np.full((g.ny, g.nx), 0.02)
    m = O.project(g, x0)
    r = O.adm(g, m, 0.9, 1.0, 64.0, 64.0, 8, x0=x0)
    assert np.abs(r.x - x0).max() <= 1e-12


def test_linearity_and_half_turn_symmetry():
    """A(ax + by) = aAx + bAy; rotating the image by 180 degrees shifts the
    sinogram by half the views (full-circle scan, even view count)."""
    g = C.Geometry(nx=48, ny=48, pixel_mm=1.0, n_views=20, n_bins=70, bin_mm=1.4, sod_mm=120.0,
                   sdd_mm=240.0, model=1)
    x, y = P.random_image(g, 5), P.random_image(g, 6)
    lhs = O.project(g, 2.5 * x - 0.75 * y)
    rhs = 2.5 * O.project(g, x) - 0.75 * O.project(g, y)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()
    Sx = O.project(g, x)
    Sr = O.project(g, x[::-1, ::-1].copy())
    V = g.n_views
    shifted = np.concatenate([Sx[V // 2:], Sx[: V // 2]])
    assert np.abs(Sr - shifted).max() <= 1e-12 * np.abs(Sx).max()
