"""GPU parity of the 3-D ADM-TV (dect_adm_tv3: Eq. 10 on a volume with the
3-D TV and the cone-beam pair) against the FP64 oracle's run (or_adm3) of
each energy on the same FP32 inputs: a 32 x 28 x 12 volume (30 views, 10 x 48
panel, 30 iterations), a ragged one (37 x 29 x 9, detector offset, 25
iterations) and a 128 x 128 x 16 one (90 views, 16 x 192 panel, 40
iterations); a warm start; the relative-change stop rule; the projection
onto f >= 0 and the BB2 / adaptive steps; the TV coupled across the two
energies (or_adm3_coupled).

* Images: rel-L2 <= 1e-4.
* The logged objective of Eq. 4: within 1e-5 over the first 10 iterations,
  where a wrong term or scale would show, and within 1e-4 over the whole
  run.  The iterate and the residual r = A f - beta m are carried as pairs
  of FP32 values updated in FP64, r by the recurrence r -= alpha A G with A G
  from the projector's FP64 ray sums, so |r|^2 keeps its accuracy relative
  to |r| even when r is a small difference of A f and beta m.
* The BB step: within 1e-4 over the first 10 iterations and 1e-3 over the
  run.  It is a ratio of differences of nearly equal iterates (the change
  of the FP32 h = mu A^T r between iterations), which amplifies FP32
  rounding as the run converges; a wrong term would be O(1) from the start.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

VOL = C.ConeGeometry(nx=32, ny=28, nz=12, voxel_mm=1.0, n_views=30, n_bins=48, n_rows=10,
                     bin_mm=1.5, row_mm=1.5, sod_mm=100.0, sdd_mm=200.0)
RAGGED = C.ConeGeometry(nx=37, ny=29, nz=9, voxel_mm=1.0, n_views=23, n_bins=53, n_rows=7,
                        bin_mm=1.4, row_mm=1.7, sod_mm=90.0, sdd_mm=170.0, det_offset_mm=0.6)
MID = C.ConeGeometry(nx=128, ny=128, nz=16, voxel_mm=1.0, n_views=90, n_bins=192, n_rows=16,
                     bin_mm=1.2, row_mm=1.2, sod_mm=500.0, sdd_mm=1000.0)
PARAMS = C.AdmParams(mu=1.0, rho=64.0, xi=16.0, beta_high=1.0, beta_low=0.79, max_iter=30)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _data(g, seed):
    """Two energies' projections of the extruded phantom (low energy 1.3x
    the attenuation) with 0.5%-of-max Gaussian noise, rounded to FP32."""
    vol = P.cone_volume(g, seed, supersample=2) * 10.0
    rng = np.random.default_rng(100 + seed)
    out = []
    for e, scale in enumerate((1.0, 1.3)):
        p = O.project3(g, scale * vol)
        out.append(f32(p + rng.normal(0.0, 0.005 * p.max(), size=p.shape)))
    return out


@pytest.mark.parametrize("geom,iters,seed", [(VOL, 30, 0), (RAGGED, 25, 1), (MID, 40, 2)],
                         ids=["volume", "ragged", "128x128x16"])
def test_parity(torch, geom, iters, seed):
    from paper_1607_01650_amd import dect
    m = _data(geom, seed)
    p = dataclasses.replace(PARAMS, max_iter=iters)
    r = dect.adm_tv3(to_dev(torch, m[0]), to_dev(torch, m[1]), geom, p, want_log=True)
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        x, log = O.adm3(geom, m[e], beta, p.mu, p.rho, p.xi, iters)
        err = rel_l2(to_np(xe), x)
        jrel = np.abs(r.log[:, e] - log[:, 0]) / np.abs(log[:, 0])
        arel = np.abs(r.log[1:, 2 + e] - log[1:, 1]) / np.abs(log[1:, 1])
        print(f"3-D ADM {geom.nx}x{geom.ny}x{geom.nz} energy {e}: image rel-L2 {err:.2e}, "
              f"J rel err k<=10 {jrel[:11].max():.2e}, all {jrel.max():.2e}, "
              f"alpha k<=10 {arel[:10].max():.2e}, all {arel.max():.2e}", flush=True)
        assert err <= 1e-4
        assert jrel[:11].max() <= 1e-5
        assert jrel.max() <= 1e-4
        assert arel[:10].max() <= 1e-4
        assert arel.max() <= 1e-3
        # auxiliary log: |grad f - z| (rows 1.., zero at the zero start) and |G|
        pres = np.abs(r.log_aux[1:iters, e] - log[1:iters, 2]) / log[1:iters, 2]
        gerr = np.abs(r.log_aux[:iters, 2 + e] - log[:iters, 4]) / log[:iters, 4]
        assert pres.max() <= 1e-3 and gerr.max() <= 1e-4, (pres.max(), gerr.max())
    assert r.report.iters == iters


def _start_volume(g, seed):
    """A start image near the solution: the phantom, smoothed along x and
    perturbed by 2% noise, rounded to FP32."""
    vol = P.cone_volume(g, seed, supersample=2) * 10.0
    vol = 0.5 * vol + 0.25 * (np.roll(vol, 1, axis=2) + np.roll(vol, -1, axis=2))
    rng = np.random.default_rng(300 + seed)
    return f32(vol * (1.0 + 0.02 * rng.standard_normal(vol.shape)))


def test_warm_start_parity(torch):
    """DECT_WARM_START: f^0 = beta x0 for each energy (x0 high for the
    high energy, 1.3 x0 for the low), the run then as from zero."""
    from paper_1607_01650_amd import dect
    g, iters = VOL, 20
    m = _data(g, 3)
    x0 = _start_volume(g, 3)
    x0s = (x0, f32(1.3 * x0))
    p = dataclasses.replace(PARAMS, max_iter=iters)
    r = dect.adm_tv3(to_dev(torch, m[0]), to_dev(torch, m[1]), g, p, want_log=True,
                     x0=(to_dev(torch, x0s[0]), to_dev(torch, x0s[1])))
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        x, log = O.adm3(g, m[e], beta, p.mu, p.rho, p.xi, iters, x0=x0s[e])
        _, log_zero = O.adm3(g, m[e], beta, p.mu, p.rho, p.xi, 1)
        err = rel_l2(to_np(xe), x)
        jrel = np.abs(r.log[:, e] - log[:, 0]) / np.abs(log[:, 0])
        arel = np.abs(r.log[1:, 2 + e] - log[1:, 1]) / np.abs(log[1:, 1])
        print(f"3-D ADM warm start energy {e}: image rel-L2 {err:.2e}, J rel err "
              f"{jrel.max():.2e}, alpha rel err {arel.max():.2e}, J0 warm/zero "
              f"{log[0, 0] / log_zero[0, 0]:.3f}", flush=True)
        assert log[0, 0] < 0.5 * log_zero[0, 0]  # the start is used, and it helps
        assert err <= 1e-4
        assert jrel.max() <= 1e-4
        assert arel.max() <= 1e-3


def _tol_between(relchg, first):
    """A tolerance that the run first meets at log row j >= first (the
    relative change of the step that ends before row j), with a margin of
    at least 1% on both sides: the geometric mean of that change and the
    smallest earlier one."""
    for j in range(first, len(relchg)):
        lo = relchg[1:j].min()
        if relchg[j] < 0.99 * lo:
            return float(np.sqrt(relchg[j] * lo)), j
    raise AssertionError("no clear new minimum of the relative change")


def test_tolerance_stop_parity(torch):
    """tol > 0: each energy stops after the first iteration whose relative
    change is below tol, as the oracle does; the report counts the longer
    run and an energy's log rows after its stop are zeros."""
    from paper_1607_01650_amd import dect
    g, kmax = VOL, 60
    m = _data(g, 4)
    p = dataclasses.replace(PARAMS, max_iter=kmax)
    _, probe = O.adm3(g, m[0], p.beta_high, p.mu, p.rho, p.xi, 40)
    tol, _ = _tol_between(probe[:, 3], 12)
    p = dataclasses.replace(p, tol=tol)
    r = dect.adm_tv3(to_dev(torch, m[0]), to_dev(torch, m[1]), g, p, want_log=True)
    its = []
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        x, log, k = O.adm3(g, m[e], beta, p.mu, p.rho, p.xi, kmax, tol=tol, with_iters=True)
        its.append(k)
        near = np.abs(log[1:k + 1, 3] / tol - 1.0).min()
        err = rel_l2(to_np(xe), x)
        jrel = np.abs(r.log[:k + 1, e] - log[:k + 1, 0]) / np.abs(log[:k + 1, 0])
        print(f"3-D ADM tol {tol:.3e} energy {e}: oracle stops after {k} iterations (closest "
              f"relative change {near:.1e} from tol), image rel-L2 {err:.2e}, J rel err "
              f"{jrel.max():.2e}", flush=True)
        assert 1 < k < kmax
        assert near > 1e-3  # no relative change within rounding of the tolerance
        assert err <= 1e-4
        assert jrel.max() <= 1e-4
        assert not np.any(r.log[k + 1:, e]) and not np.any(r.log[k + 1:, 2 + e])
    assert r.report.iters == max(its)


@pytest.mark.parametrize("nonneg,step", [(True, "bb1"), (False, "bb2"), (False, "abb"),
                                         (True, "abb")],
                         ids=["nonneg", "bb2", "abb", "nonneg-abb"])
def test_variant_parity(torch, nonneg, step):
    """DECT_NONNEG (the projected step, the residual following A s) and the
    BB2 / adaptive steps against the oracle's same variants; with noise
    strong enough that f >= 0 binds at many voxels."""
    from paper_1607_01650_amd import dect
    g, iters = VOL, 20
    m = _data(g, 9)
    rng = np.random.default_rng(9)
    m = [f32(a + 0.05 * a.max() * rng.standard_normal(a.shape)) for a in m]
    p = dataclasses.replace(PARAMS, max_iter=iters, nonneg=nonneg, step=step)
    r = dect.adm_tv3(to_dev(torch, m[0]), to_dev(torch, m[1]), g, p, want_log=True)
    for e, (xe, beta) in enumerate(((r.x_high, p.beta_high), (r.x_low, p.beta_low))):
        x, log = O.adm3(g, m[e], beta, p.mu, p.rho, p.xi, iters, nonneg=nonneg, step=step)
        err = rel_l2(to_np(xe), x)
        jrel = np.abs(r.log[:, e] - log[:, 0]) / np.abs(log[:, 0])
        arel = np.abs(r.log[1:, 2 + e] - log[1:, 1]) / np.abs(log[1:, 1])
        zeros = int((x == 0.0).sum())
        print(f"3-D ADM {step}{' nonneg' if nonneg else ''} energy {e}: image rel-L2 {err:.2e}, "
              f"J rel err {jrel.max():.2e}, step rel err k<=10 {arel[:10].max():.2e}, "
              f"all {arel.max():.2e}, oracle zero voxels {zeros}", flush=True)
        assert err <= 1e-4 and jrel.max() <= 1e-4
        assert arel[:10].max() <= 1e-4 and arel.max() <= 1e-3
        if nonneg:
            assert to_np(xe).min() >= 0.0 and zeros > 100


def test_refusals(torch):
    from paper_1607_01650_amd import dect
    g = VOL
    z = torch.zeros((g.n_views, g.n_rows, g.n_bins), device="cuda")
    for change in ({"coupled_tv": True, "tol": 1e-3}, {"coupled_tv": True, "step": "bb2"},
                   {"tol": -1e-3}, {"tol": float("nan")}):
        with pytest.raises(dect.DectError):
            dect.adm_tv3(z, z, g, dataclasses.replace(PARAMS, max_iter=2, **change))


def test_full_size_first_iteration(torch):
    """512 x 512 x 64, 360 views, 64 x 736 panel (the bench configuration):
    from f = 0 (lambda = z = 0, so W = 0) the first gradient is
    G = -mu beta A^T m and the first step the exact line search along it, so
    x^1 = alpha0 mu A^T m with alpha0 = |G|^2 / (mu |A G|^2 + rho |grad G|^2);
    and J^0 = mu/2 |beta m|^2.  A, A^T are the GPU pair (its own parity tests
    hold it to the oracle); the rest is formed on the host in FP64."""
    from paper_1607_01650_amd import dect
    g = C.CONE
    vol = to_dev(torch, P.cone_volume(g, 0, supersample=2))
    mh = dect.cone_project(vol, g)
    ml = dect.cone_project(vol * 1.3, g)
    p = C.AdmParams(mu=45.0 / g.n_views, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79,
                    max_iter=1)
    r = dect.adm_tv3(mh, ml, g, p, want_log=True)
    for e, (m, beta, xe) in enumerate(((mh, p.beta_high, r.x_high), (ml, p.beta_low, r.x_low))):
        atm = to_np(dect.cone_backproject(m, g))
        G = -p.mu * beta * atm
        ag = to_np(dect.cone_project(to_dev(torch, G), g))
        gd = O.grad3(G)
        alpha0 = np.sum(G * G) / (p.mu * np.sum(ag * ag) + p.rho * np.sum(gd * gd))
        want = alpha0 * p.mu * atm
        err = rel_l2(to_np(xe), want)
        gs = beta * to_np(m)  # beta m in FP64, as the residual is formed
        j0 = 0.5 * p.mu * np.sum(gs ** 2)
        print(f"3-D ADM 512x512x64 energy {e}: first iterate rel-L2 {err:.2e}, J0 rel err "
              f"{abs(r.log[0, e] - j0) / j0:.2e}, alpha0 rel err "
              f"{abs(r.log[0, 2 + e] - alpha0) / alpha0:.2e}", flush=True)
        assert err <= 1e-5
        assert abs(r.log[0, e] - j0) <= 1e-9 * j0
        assert abs(r.log[0, 2 + e] - alpha0) <= 1e-5 * alpha0


@pytest.mark.parametrize("geom,seed,nonneg,warm", [(VOL, 5, False, False), (RAGGED, 6, False, False),
                                                   (VOL, 7, True, False), (RAGGED, 8, False, True)],
                         ids=["volume", "ragged", "nonneg", "warm-start"])
def test_coupled_parity(torch, geom, seed, nonneg, warm):
    """DECT_COUPLED_TV: one joint z-step over the 6-vector of both energies'
    gradients, each energy keeping its own f-step and BB1 step; the high
    energy's J column holds the joint TV, the low one's none."""
    from paper_1607_01650_amd import dect
    iters = 25
    m = _data(geom, seed)
    if nonneg:
        rng = np.random.default_rng(seed)
        m = [f32(a + 0.05 * a.max() * rng.standard_normal(a.shape)) for a in m]
    x0s = None
    if warm:
        x0 = _start_volume(geom, seed)
        x0s = (x0, f32(1.3 * x0))
    p = dataclasses.replace(PARAMS, max_iter=iters, coupled_tv=True, nonneg=nonneg)
    r = dect.adm_tv3(to_dev(torch, m[0]), to_dev(torch, m[1]), geom, p, want_log=True,
                     x0=None if x0s is None else (to_dev(torch, x0s[0]), to_dev(torch, x0s[1])))
    x, J, a = O.adm3_coupled(geom, m[0], m[1], p.beta_high, p.beta_low, p.mu, p.rho, p.xi, iters,
                             x0=x0s, nonneg=nonneg)
    for e, xe in enumerate((r.x_high, r.x_low)):
        err = rel_l2(to_np(xe), x[e])
        jrel = np.abs(r.log[:, e] - J[:, e]) / np.abs(J[:, e])
        arel = np.abs(r.log[1:, 2 + e] - a[1:, e]) / np.abs(a[1:, e])
        print(f"3-D coupled ADM {geom.nx}x{geom.ny}x{geom.nz}{' nonneg' if nonneg else ''}"
              f"{' warm' if warm else ''} energy {e}: image rel-L2 {err:.2e}, J rel err "
              f"{jrel.max():.2e}, alpha rel err k<=10 {arel[:10].max():.2e}, all "
              f"{arel.max():.2e}", flush=True)
        assert err <= 1e-4 and jrel.max() <= 1e-4
        assert arel[:10].max() <= 1e-4 and arel.max() <= 1e-3
        if nonneg:
            assert to_np(xe).min() >= 0.0
    # the coupling matters here: the per-energy run ends elsewhere
    xs, _ = O.adm3(geom, m[0], p.beta_high, p.mu, p.rho, p.xi, iters, nonneg=nonneg,
                   x0=None if x0s is None else x0s[0])
    assert rel_l2(xs, x[0]) > 1e-3
    assert r.report.iters == iters
