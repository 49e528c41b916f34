"""GPU parity of the non-negative ADM variant (DECT_NONNEG: every f-step
projected onto f >= 0, BB1 step from the projected step) against the FP64
oracle's projected run.

* tiny workload, 50 iterations, and the ragged geometry, 40 iterations:
  image rel-L2 <= 1e-4, logged objective within 1e-5, images non-negative
  with the constraint active (pixels at exactly zero);
* 512 x 512 x 360 views, 200 iterations, against the stored oracle run
  (tests/golden/make_golden.py 360 nonneg), with the bounds of the
  unconstrained run at 360 views;
* resuming through a state is bitwise equal to one call; a state started
  without the flag refuses to continue with it; the tolerance stop agrees
  with the oracle's iteration count; the batched ADM takes the flag but
  not with the BB2 step.
"""
import dataclasses
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

RAGGED = C.Geometry(nx=67, ny=45, pixel_mm=1.0, n_views=37, n_bins=101, bin_mm=1.3,
                    sod_mm=300.0, sdd_mm=600.0, det_offset_mm=0.7)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _dect():
    from paper_1607_01650_amd import dect
    return dect


def _check(r, g, s, p, iters, tag):
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, iters, nonneg=True)
        x = to_np(xe)
        err = rel_l2(x, ref.x)
        jerr = np.max(np.abs(r.J[:, e] - ref.J) / np.abs(ref.J))
        print(f"{tag} non-negative ADM energy {e}: image rel-L2 {err:.2e}, max J rel err "
              f"{jerr:.2e}, zero pixels {(x == 0).sum()}", flush=True)
        assert err <= 1e-4
        assert jerr <= 1e-5
        assert x.min() >= 0.0 and (x == 0).sum() > 0


def test_tiny_parity(torch):
    dect = _dect()
    s = P.make_slice(C.TINY, 0)
    p = dataclasses.replace(C.default_adm_params(C.TINY, 50), nonneg=True)
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), C.TINY, p,
                    want_log=True)
    _check(r, C.TINY, s, p, 50, "tiny")


def test_ragged_parity(torch):
    dect = _dect()
    g = RAGGED
    s = P.make_slice(g, 21, n_inserts=3, r_obj=18.0)
    p = C.AdmParams(mu=1.0, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79, max_iter=40,
                    nonneg=True)
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    _check(r, g, s, p, 40, "ragged")


def test_paper_scale_parity_200(torch):
    dect = _dect()
    path = os.path.join(os.path.dirname(__file__), "golden", "adm512_v360_k200_nonneg.npz")
    gold = np.load(path)
    g = C.paper_geometry(512, 360)
    s = P.make_slice(g, 0)
    p = dataclasses.replace(C.default_adm_params(g, 200), nonneg=True)
    assert float(gold["mu"]) == p.mu and float(gold["xi"]) == p.xi
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    for e, xe in enumerate((r.x_high, r.x_low)):
        x = to_np(xe)
        err = rel_l2(x, gold["x"][e])
        jrel = np.abs(r.J[:, e] - gold["J"][e]) / gold["J"][e]
        print(f"non-negative V=360 energy {e}: image rel-L2 {err:.3e}  J200 rel err "
              f"{jrel[200]:.2e}  max J rel err k<=10 {jrel[:11].max():.2e}", flush=True)
        assert err <= 1e-4
        assert jrel[200] <= 1e-4
        assert jrel[:11].max() <= 1e-5
        assert x.min() >= 0.0


def test_resume_bitwise_and_flag_mismatch(torch):
    dect = _dect()
    g = C.TINY
    s = P.make_slice(g, 0)
    mh, ml = to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1])
    p = dataclasses.replace(C.default_adm_params(g, 12), nonneg=True)
    one = dect.adm_tv(mh, ml, g, p)
    st = dect.AdmState(g)
    dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=5), state=st)
    two = dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=7), state=st)
    assert np.array_equal(to_np(one.x_high), to_np(two.x_high))
    assert np.array_equal(to_np(one.x_low), to_np(two.x_low))
    with pytest.raises(dect.DectError):
        dect.adm_tv(mh, ml, g, dataclasses.replace(p, nonneg=False), state=st)
    st.close()


def test_tol_stop(torch):
    dect = _dect()
    g = C.TINY
    s = P.make_slice(g, 0)
    p = dataclasses.replace(C.default_adm_params(g, 300), tol=2e-3, nonneg=True)
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    its = []
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, 300, tol=p.tol, nonneg=True)
        assert rel_l2(to_np(xe), ref.x) <= 1e-4
        its.append(ref.iters)
    assert r.report.iters == max(its) < 300


def test_batch_refuses(torch):
    """The batch takes the projection, but not with the BB2 step (as the
    single-slice path)."""
    dect = _dect()
    with pytest.raises(dect.DectError):
        dect.AdmBatch([C.TINY], [dataclasses.replace(C.default_adm_params(C.TINY, 5),
                                                     nonneg=True, step="bb2")])
