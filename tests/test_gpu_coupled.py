"""GPU parity of ADM-TV with the TV coupled across the two energies
(DECT_COUPLED_TV: one joint z-step over both energies' gradients) against
the FP64 oracle's coupled run: tiny workload (50 iterations), ragged
geometry (40), and coupled together with the non-negativity projection
(30): images rel-L2 <= 1e-4; both logged objective columns within 1e-5 over
the first 10 iterations, where a systematic error (a wrong term or scale)
would show, and within 1e-4 over the whole run.  The ragged problem reaches
its minimum within ~25 iterations; from there the BB step is formed from
differences of nearly equal iterates and amplifies rounding (measured: J
within 1.4e-5 and alpha within 2e-4 late in the run, while the final images
agree to 8e-8).  Resuming through a state is bitwise equal to one call; a
tolerance stop is refused, in the batched ADM too (which otherwise takes the
coupled TV).
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


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _dect():
    from paper_1607_01650_amd import dect
    return dect


def _parity(torch, g, s, p, iters, tag):
    dect = _dect()
    r = dect.adm_tv(to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1]), g, p, want_log=True)
    x, J, _ = O.adm_coupled(g, f32(s.sino[0]), f32(s.sino[1]), p.beta_high, p.beta_low, p.mu,
                            p.rho, p.xi, iters, nonneg=p.nonneg)
    for e, xe in enumerate((r.x_high, r.x_low)):
        err = rel_l2(to_np(xe), x[e])
        jrel = np.abs(r.J[:, e] - J[:, e]) / np.abs(J[:, e])
        print(f"{tag} coupled-TV energy {e}: image rel-L2 {err:.2e}, max J rel err "
              f"k<=10 {jrel[:11].max():.2e}, all {jrel.max():.2e}", flush=True)
        assert err <= 1e-4
        assert jrel[:11].max() <= 1e-5
        assert jrel.max() <= 1e-4
        if p.nonneg:
            assert to_np(xe).min() >= 0.0


def test_tiny_parity(torch):
    s = P.make_slice(C.TINY, 0)
    p = dataclasses.replace(C.default_adm_params(C.TINY, 50), coupled_tv=True)
    _parity(torch, C.TINY, s, p, 50, "tiny")


def test_ragged_parity(torch):
    g = RAGGED
    s = P.make_slice(g, 21, n_inserts=3, r_obj=18.0)
    p = C.AdmParams(mu=1.0, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79, max_iter=40,
                    coupled_tv=True)
    _parity(torch, g, s, p, 40, "ragged")


def test_coupled_and_nonneg(torch):
    s = P.make_slice(C.TINY, 1)
    p = dataclasses.replace(C.default_adm_params(C.TINY, 30), coupled_tv=True, nonneg=True)
    _parity(torch, C.TINY, s, p, 30, "tiny non-negative")


def test_resume_and_refusals(torch):
    dect = _dect()
    g = C.TINY
    s = P.make_slice(g, 0)
    mh, ml = to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1])
    p = dataclasses.replace(C.default_adm_params(g, 11), coupled_tv=True)
    one = dect.adm_tv(mh, ml, g, p)
    st = dect.AdmState(g)
    dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=4), state=st)
    two = dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=7), state=st)
    assert np.array_equal(to_np(one.x_high), to_np(two.x_high))
    assert np.array_equal(to_np(one.x_low), to_np(two.x_low))
    with pytest.raises(dect.DectError):
        dect.adm_tv(mh, ml, g, dataclasses.replace(p, coupled_tv=False), state=st)
    st.close()
    with pytest.raises(dect.DectError):
        dect.adm_tv(mh, ml, g, dataclasses.replace(p, tol=1e-3))
    with pytest.raises(dect.DectError):  # the batch takes the coupled TV at tol 0 only
        dect.AdmBatch([g], [dataclasses.replace(p, tol=1e-3)])
