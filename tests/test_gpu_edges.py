"""Edge and degenerate cases of the GPU path against the FP64 oracle.

* ADM on a ragged geometry (67 x 45 image, 37 views, offset detector): partial
  tiles and back-projection strips at the right and bottom edges, views split
  unevenly into groups;
* ADM on zero sinograms: the iterate stays exactly zero and J = 0 (the step
  size of a zero gradient is defined as 0 on both sides);
* a single view: projector parity and the adjoint identity;
* an image smaller than one back-projection strip (9 x 5 pixels);
* detector bins so fine that a strip sees hundreds of bins per view;
* PLS on a ragged image;
* a batch of one slice reproduces the single-slice path bit for bit.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

RAGGED = C.Geometry(nx=67, ny=45, pixel_mm=1.0, n_views=37, n_bins=101, bin_mm=1.3,
                    sod_mm=300.0, sdd_mm=600.0, det_offset_mm=0.7)
ONE_VIEW = C.Geometry(nx=40, ny=40, pixel_mm=1.0, n_views=1, n_bins=70, bin_mm=1.2,
                      sod_mm=200.0, sdd_mm=400.0)
SMALL = C.Geometry(nx=9, ny=5, pixel_mm=1.0, n_views=7, n_bins=15, bin_mm=1.1,
                   sod_mm=40.0, sdd_mm=80.0)
# detector bins of 0.06 px at the isocentre: a back-projection strip is hit by
# hundreds of bins per view (more than the per-lane range table holds)
FINE_BINS = C.Geometry(nx=64, ny=64, pixel_mm=1.0, n_views=12, n_bins=1200, bin_mm=0.12,
                       sod_mm=200.0, sdd_mm=400.0)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _dect():
    from paper_1607_01650_amd import dect
    return dect


def _params(g, iters):
    return C.AdmParams(mu=1.0, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79,
                       max_iter=iters)


def test_adm_ragged_parity(torch):
    dect = _dect()
    g = RAGGED
    s = P.make_slice(g, 21, n_inserts=3, r_obj=18.0)
    p = _params(g, 40)
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, 40)
        err = rel_l2(to_np(xe), ref.x)
        jerr = np.max(np.abs(r.J[:, e] - ref.J) / np.abs(ref.J))
        print(f"ragged ADM energy {e}: image rel-L2 {err:.2e}, max J rel err {jerr:.2e}",
              flush=True)
        assert err <= 1e-4
        assert jerr <= 1e-5


def test_adm_zero_data_stays_zero(torch):
    dect = _dect()
    g = C.TINY
    z = torch.zeros((g.n_views, g.n_bins), device="cuda")
    r = dect.adm_tv(z, z, g, _params(g, 6), want_log=True)
    assert not torch.any(r.x_high).item() and not torch.any(r.x_low).item()
    assert np.all(r.J == 0.0)
    ref = O.adm(g, np.zeros((g.n_views, g.n_bins)), 1.0, 1.0, 1024.0, 256.0, 6)
    assert np.all(ref.x == 0.0) and np.all(ref.J == 0.0)


@pytest.mark.parametrize("geom", [ONE_VIEW, SMALL, FINE_BINS], ids=["one_view", "9x5", "fine_bins"])
def test_projectors_degenerate_geometries(torch, geom):
    dect = _dect()
    g = geom
    x = f32(P.random_image(g, 3))
    y = f32(P.random_sino(g, 4))
    ax = to_np(dect.project(to_dev(torch, x), g))
    aty = to_np(dect.backproject(to_dev(torch, y), g))
    assert rel_l2(ax, O.project(g, x)) <= 1e-5
    assert rel_l2(aty, O.backproject(g, y)) <= 1e-5
    lhs, rhs = float(np.sum(ax * y)), float(np.sum(x * aty))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


def test_pls_ragged(torch):
    dect = _dect()
    g = RAGGED
    s = P.make_slice(g, 22, n_inserts=3, r_obj=18.0)
    rng = np.random.default_rng(11)
    xh = f32(s.x_true[0] + 0.0005 * rng.standard_normal(s.x_true[0].shape))
    xl = f32(s.x_true[1] + 0.0005 * rng.standard_normal(s.x_true[1].shape))
    p = dataclasses.replace(C.PlsParams(), gamma=1.0, tol=1e-7)
    u1, u2, _ = dect.pls_decompose(to_dev(torch, xh), to_dev(torch, xl), p)
    r1, r2, _, _ = O.pls(xh, xl, p, tol=1e-12)
    assert rel_l2(to_np(u1), r1) <= 1e-5 and rel_l2(to_np(u2), r2) <= 1e-5


def test_batch_of_one_equals_single(torch):
    dect = _dect()
    g = RAGGED
    s = P.make_slice(g, 23, n_inserts=3, r_obj=18.0)
    p = _params(g, 12)
    mh, ml = to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1])
    single = dect.adm_tv(mh, ml, g, p)
    b = dect.AdmBatch([g], [p])
    xh, xl, _ = b.run([mh], [ml], 12)
    b.close()
    assert np.array_equal(to_np(xh[0]), to_np(single.x_high))
    assert np.array_equal(to_np(xl[0]), to_np(single.x_low))
