"""Pins of the oracle's fan-beam filtered back-projection (the analytic
reconstruction the paper compares with, Sec. 3) against what any correct
FBP must reproduce from exact line integrals:

* the attenuation of uniform disks, centred and far off-centre (a wrong ramp
  scale, a missing half for the full turn or a wrong distance weight moves
  these values);
* zero outside the object;
* a quarter turn of the views rotates the image by 90 degrees exactly;
* the error in the object's interior falls as views and bins are refined.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P


def _geom(n=128, views=360, bins=300, bin_mm=1.0, sod=300.0, sdd=600.0):
    return C.Geometry(nx=n, ny=n, pixel_mm=1.0, n_views=views, n_bins=bins, bin_mm=bin_mm,
                      sod_mm=sod, sdd_mm=sdd)


def _pix(g, x, y):
    """(row, col) of the pixel whose centre is nearest to (x, y) mm."""
    return (int(round(y / g.pixel_mm + (g.ny - 1) / 2.0)),
            int(round(x / g.pixel_mm + (g.nx - 1) / 2.0)))


@pytest.mark.parametrize("cx,cy", [(0.0, 0.0), (38.0, -27.0), (-44.0, 30.0)],
                         ids=["centre", "off1", "off2"])
def test_uniform_disk_value(cx, cy):
    g = _geom()
    mu = 0.02
    el = [P.Ellipse(cx, cy, 12.0, 12.0, 0.0, mu, 0.03, 1)]
    img = O.fbp(g, P.analytic_sinogram(el, g, 0))
    r, c = _pix(g, cx, cy)
    core = img[r - 5:r + 6, c - 5:c + 6]
    assert np.abs(core - mu).max() <= 2e-3 * mu
    # far from the disk the image is empty, up to the streaks of its edge
    far = img[_pix(g, -cx, -cy)[0] - 3:_pix(g, -cx, -cy)[0] + 4,
              _pix(g, -cx, -cy)[1] - 3:_pix(g, -cx, -cy)[1] + 4]
    if (cx, cy) != (0.0, 0.0):
        assert np.abs(far).max() <= 3e-2 * mu  # only the edge's aliasing streaks


def test_quarter_turn_rotates_the_image():
    """Views shifted by V/4 (a quarter turn of the source) reconstruct the
    image turned by 90 degrees counter-clockwise, to rounding."""
    g = _geom(n=64, views=120, bins=160)
    el = [P.Ellipse(9.0, -4.0, 14.0, 7.0, 0.4, 0.02, 0.03, 1),
          P.Ellipse(-12.0, 10.0, 5.0, 3.0, 0.0, 0.04, 0.08, 2)]
    s = P.analytic_sinogram(el, g, 0)
    a = O.fbp(g, s)
    # the views shifted by a quarter turn are the views of g(p) = f(Rp), R the
    # rotation by +90 degrees: b at (x, y) is a at (-y, x), i.e. b[r, c] =
    # a[c, n - 1 - r] (rows index y, columns x)
    b = O.fbp(g, np.roll(s, -g.n_views // 4, axis=0))
    assert np.abs(b - np.rot90(a, k=1)).max() <= 1e-12 * np.abs(a).max()
    assert np.abs(b - a).max() > 0.1 * np.abs(a).max()  # the test object is not symmetric


def test_interior_error_falls_with_sampling():
    """Inside an off-centre, rotated uniform ellipse (3 px from its edge) the
    mean error falls about fourfold per doubling of views and bins.  (A
    small high-contrast object leaves slowly decaying errors of ~1% of its
    contrast around it in any sampled FBP, so the pin uses one large one.)"""
    el = [P.Ellipse(6.0, -3.0, 40.0, 28.0, 0.3, 0.02, 0.03, 1)]
    errs = []
    for views, bins, bin_mm in ((90, 150, 2.0), (180, 300, 1.0), (360, 600, 0.5)):
        g = _geom(views=views, bins=bins, bin_mm=bin_mm)
        img = O.fbp(g, P.analytic_sinogram(el, g, 0))
        truth = P.rasterize(el, g, 0, supersample=8)
        # pixels inside the object, at least 3 px from every edge of the phantom
        edge = np.zeros_like(truth, dtype=bool)
        for sh in [(i, j) for i in range(-3, 4) for j in range(-3, 4)]:
            edge |= np.roll(truth, sh, axis=(0, 1)) != truth
        inner = ~edge & (truth > 0)
        errs.append(np.abs(img - truth)[inner].mean())
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5, errs
    assert errs[-1] < 5e-5 * 0.02
