"""GPU parity of the Siddon ray model (exact pixel intersection lengths,
Sec. 2.1) against the FP64 oracle's Siddon walk.

* projection and back-projection per call: rel-L2 <= 1e-5, on the tiny and
  ragged geometries, a geometry with views exactly on the axes and the
  diagonals (slopes 0 and 1, the two ends of the weight formula), fine
  detector bins, and the full 512 x 512 x 360-view workload;
* the GPU matrices of A and A^T, built column by column on a 16 x 13 image,
  are transposes of each other to FP32 rounding and match the oracle's exact
  chord lengths entry by entry;
* a batch of three (a pair and a single instance) equals single calls bit
  for bit;
* ADM-TV of both energies on the Siddon model, 50 iterations on the tiny
  workload: image rel-L2 <= 1e-4, objective within 1e-5; 200 iterations at
  512 x 512 x 360 views against the stored oracle run;
* an unknown model value is refused (the batched ADM takes Siddon slices:
  test_gpu_batch.py).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


def _sid(g):
    return C.Geometry(**{**g.__dict__, "model": 1})


TINY_S = _sid(C.TINY)
RAGGED_S = C.Geometry(nx=67, ny=45, pixel_mm=1.0, n_views=37, n_bins=101, bin_mm=1.3,
                      sod_mm=300.0, sdd_mm=600.0, det_offset_mm=0.7, model=1)
# odd sizes: the rays through the isocentre on the axis views run along row
# or column centres, not along pixel boundaries (where the pixel a ray on the
# boundary is assigned to is a matter of rounding)
AXES_S = C.Geometry(nx=41, ny=41, pixel_mm=1.0, n_views=8, n_bins=71, bin_mm=1.0, sod_mm=150.0,
                    sdd_mm=300.0, angles_rad=[k * math.pi / 4 for k in range(8)], model=1)
FINE_S = C.Geometry(nx=64, ny=64, pixel_mm=1.0, n_views=12, n_bins=1200, bin_mm=0.12,
                    sod_mm=200.0, sdd_mm=400.0, model=1)
G16_S = C.Geometry(nx=16, ny=13, pixel_mm=1.1, n_views=9, n_bins=25, bin_mm=1.5, sod_mm=60.0,
                   sdd_mm=130.0, det_offset_mm=0.3, model=1)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _dect():
    from paper_1607_01650_amd import dect
    return dect


@pytest.mark.parametrize("geom", [TINY_S, RAGGED_S, AXES_S, FINE_S],
                         ids=["tiny", "ragged", "axes", "fine_bins"])
def test_projector_parity(torch, geom):
    dect = _dect()
    g = geom
    x = f32(P.random_image(g, 3))
    y = f32(P.random_sino(g, 4))
    ax = to_np(dect.project(to_dev(torch, x), g))
    aty = to_np(dect.backproject(to_dev(torch, y), g))
    e1, e2 = rel_l2(ax, O.project(g, x)), rel_l2(aty, O.backproject(g, y))
    print(f"siddon {g.nx}x{g.ny} V={g.n_views} B={g.n_bins}: A {e1:.2e}, A^T {e2:.2e}", flush=True)
    assert e1 <= 1e-5 and e2 <= 1e-5
    lhs, rhs = float(np.sum(ax * y)), float(np.sum(x * aty))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


def test_projector_parity_metric(torch):
    """The full 512 x 512, 360-view, 736-bin workload on the Siddon model."""
    dect = _dect()
    g = _sid(C.METRIC)
    s = P.make_slice(C.METRIC, 7)
    x = f32(s.x_true[1])
    y = f32(P.random_sino(g, 8))
    ax = to_np(dect.project(to_dev(torch, x), g))
    aty = to_np(dect.backproject(to_dev(torch, y), g))
    e1, e2 = rel_l2(ax, O.project(g, x)), rel_l2(aty, O.backproject(g, y))
    print(f"siddon metric: A {e1:.2e}, A^T {e2:.2e}", flush=True)
    assert e1 <= 1e-5 and e2 <= 1e-5


def test_dense_matrices(torch):
    """GPU A (unit images) and GPU A^T (unit sinograms) on 16 x 13: transposes
    of each other, and every entry the oracle's chord length."""
    dect = _dect()
    g = G16_S
    N, M = g.nx * g.ny, g.n_views * g.n_bins
    eye_n = torch.eye(N, device="cuda").reshape(N, g.ny, g.nx)
    A = to_np(dect.project(eye_n, g)).reshape(N, M).T
    eye_m = torch.eye(M, device="cuda").reshape(M, g.n_views, g.n_bins)
    AT = to_np(dect.backproject(eye_m, g)).reshape(M, N)
    ref = np.stack([O.project(g, np.eye(N)[i].reshape(g.ny, g.nx)).reshape(-1)
                    for i in range(N)], axis=1)
    scale = np.abs(ref).max()
    assert np.abs(AT - A).max() <= 2e-6 * scale
    # the split of a line's path length at a pixel boundary moves by dq / |k|
    # for a position error dq (~1e-9 pixel in 32.32 fixed point over 16 lines)
    assert np.abs(A - ref).max() <= 1e-5 * scale
    assert ((ref > 0) == (A > 1e-6 * scale)).mean() > 0.999


def test_batch_pairs_equal_single_calls(torch):
    dect = _dect()
    g = RAGGED_S
    xs = np.stack([f32(P.random_image(g, 10 + i)) for i in range(3)])
    ys = np.stack([f32(P.random_sino(g, 20 + i)) for i in range(3)])
    pb = to_np(dect.project(to_dev(torch, xs), g))
    bb = to_np(dect.backproject(to_dev(torch, ys), g))
    for i in range(3):
        assert np.array_equal(pb[i], to_np(dect.project(to_dev(torch, xs[i]), g)))
        assert np.array_equal(bb[i], to_np(dect.backproject(to_dev(torch, ys[i]), g)))


def test_adm_tiny_parity(torch):
    dect = _dect()
    s = P.make_slice(C.TINY, 0)
    g = TINY_S
    p = C.default_adm_params(C.TINY, 50)
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, 50)
        err = rel_l2(to_np(xe), ref.x)
        jerr = np.max(np.abs(r.J[:, e] - ref.J) / np.abs(ref.J))
        print(f"siddon tiny ADM energy {e}: image rel-L2 {err:.2e}, max J rel err {jerr:.2e}",
              flush=True)
        assert err <= 1e-4
        assert jerr <= 1e-5


def test_refusals(torch):
    dect = _dect()
    bad = C.Geometry(**{**C.TINY.__dict__, "model": 2})
    with pytest.raises(dect.DectError):
        dect.project(torch.zeros((C.TINY.ny, C.TINY.nx), device="cuda"), bad)


def test_adm_paper_scale_parity_200(torch):
    """512x512, 360 views, 736 bins, both energies, 200 iterations on the
    Siddon model vs the stored FP64 oracle run (tests/golden/make_golden.py
    360 siddon): the same bounds as the Joseph model at 360 views (image
    rel-L2 <= 1e-4 per energy, J(f^200) within 1e-4, J(f^k) for k <= 10
    within 1e-5), whose FP32 rounding floor is derived there."""
    import dataclasses
    import os
    dect = _dect()
    path = os.path.join(os.path.dirname(__file__), "golden", "adm512_v360_k200_siddon.npz")
    gold = np.load(path)
    g = dataclasses.replace(C.paper_geometry(512, 360), model=1)
    s = P.make_slice(g, 0)
    p = C.default_adm_params(g, 200)
    assert float(gold["mu"]) == p.mu and float(gold["xi"]) == p.xi
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    for e, xe in enumerate((r.x_high, r.x_low)):
        err = rel_l2(to_np(xe), gold["x"][e])
        jrel = np.abs(r.J[:, e] - gold["J"][e]) / gold["J"][e]
        print(f"siddon V=360 energy {e}: image rel-L2 {err:.3e}  J200 rel err {jrel[200]:.2e}  "
              f"max J rel err k<=10 {jrel[:11].max():.2e}", flush=True)
        assert err <= 1e-4
        assert jrel[200] <= 1e-4
        assert jrel[:11].max() <= 1e-5
