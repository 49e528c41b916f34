"""GPU parity of the BB2 and adaptive Barzilai-Borwein step rules
(DECT_STEP_BB2, DECT_STEP_ABB) against the FP64 oracle's runs with the same
rule: tiny workload, 50 iterations, and the ragged geometry, 40: images
rel-L2 <= 1e-4, the logged objective and step within 1e-5 over the first 10
iterations (where a wrong term or scale would show) and the objective within
1e-4 over the run.  The flags exclude each other and the non-negative
variant, in the batched ADM too (which takes each of them alone).
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
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, iters, step=p.step)
        err = rel_l2(to_np(xe), ref.x)
        jrel = np.abs(r.J[:, e] - ref.J) / np.abs(ref.J)
        arel = np.abs(r.alpha[:11, e] - ref.alpha[:11]) / np.abs(ref.alpha[:11])
        print(f"{tag} {p.step} energy {e}: image rel-L2 {err:.2e}, J rel err k<=10 "
              f"{jrel[:11].max():.2e} all {jrel.max():.2e}, alpha k<=10 {arel.max():.2e}",
              flush=True)
        assert err <= 1e-4
        assert jrel[:11].max() <= 1e-5 and arel.max() <= 1e-5
        assert jrel.max() <= 1e-4


@pytest.mark.parametrize("step", ["bb2", "abb"])
def test_tiny_parity(torch, step):
    s = P.make_slice(C.TINY, 0)
    p = dataclasses.replace(C.default_adm_params(C.TINY, 50), step=step)
    _parity(torch, C.TINY, s, p, 50, "tiny")


@pytest.mark.parametrize("step", ["bb2", "abb"])
def test_ragged_parity(torch, step):
    s = P.make_slice(RAGGED, 21, n_inserts=3, r_obj=18.0)
    p = C.AdmParams(mu=1.0, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79, max_iter=40,
                    step=step)
    _parity(torch, RAGGED, s, p, 40, "ragged")


def test_refusals(torch):
    dect = _dect()
    g = C.TINY
    s = P.make_slice(g, 0)
    mh, ml = to_dev(torch, s.sino[0]), to_dev(torch, s.sino[1])
    p = dataclasses.replace(C.default_adm_params(g, 3), step="bb2", nonneg=True)
    with pytest.raises(dect.DectError):
        dect.adm_tv(mh, ml, g, p)
    prm = dect.dect_adm_params(p.mu, p.rho, p.xi, p.beta_high, p.beta_low, 3, 0.0,
                               dect.DECT_STEP_BB2 | dect.DECT_STEP_ABB, None)
    xh = torch.empty((g.ny, g.nx), device="cuda")
    xl = torch.empty_like(xh)
    st = dect.lib().dect_adm_tv(dect.GeomArg(g).ref, dect.ct.c_void_p(mh.data_ptr()),
                                dect.ct.c_void_p(ml.data_ptr()), dect.ct.byref(prm),
                                dect.ct.c_void_p(xh.data_ptr()), dect.ct.c_void_p(xl.data_ptr()),
                                None, None, None)
    assert st == 1  # DECT_ERR_INVALID_ARG
    with pytest.raises(dect.DectError):  # the batch refuses what the single path does
        dect.AdmBatch([g], [p])
