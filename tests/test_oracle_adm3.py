"""Pins of the oracle's 3-D ADM-TV (Eq. 10 on a volume: Eq. 2's TV with
backward differences along x, y and z, the isotropic shrinkage of Eq. 8 on
the 3-vector, the cone-beam projector pair):

* the 3-D differences equal numpy's first differences (zero on the first
  column, row and slice) and their adjoint satisfies the adjoint identity;
* a one-slice volume seen by a one-row panel is the fan-beam problem: the
  run equals the pinned 2-D ADM of the central plane (the z-differences
  vanish and the central row is the fan-beam projector), also with the
  projection onto f >= 0, the BB2 and adaptive steps, a start image and the
  stop rule;
* zero data keeps the volume exactly zero;
* on a dense 6 x 6 x 4 problem the objective reaches the minimum of Eq. 4
  with the 3-D TV found by an independent algorithm (Chambolle-Pock).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C

SMALL3 = C.ConeGeometry(nx=6, ny=6, nz=4, voxel_mm=1.0, n_views=8, n_bins=12, n_rows=5,
                        bin_mm=1.4, row_mm=1.3, sod_mm=30.0, sdd_mm=60.0)


def test_differences_and_adjoint():
    rng = np.random.default_rng(0)
    x = rng.random((5, 7, 9))
    g = O.grad3(x)
    want = np.zeros((3,) + x.shape)
    want[0][:, :, 1:] = np.diff(x, axis=2)
    want[1][:, 1:, :] = np.diff(x, axis=1)
    want[2][1:, :, :] = np.diff(x, axis=0)
    assert np.array_equal(g, want)
    p = rng.random((3,) + x.shape)
    assert abs(np.sum(g * p) - np.sum(x * O.gradT3(p))) <= 1e-12 * np.sum(np.abs(g * p))


def test_single_slice_is_the_fan_beam_run():
    g3 = C.ConeGeometry(nx=20, ny=18, nz=1, voxel_mm=1.0, n_views=16, n_bins=30, n_rows=1,
                        bin_mm=1.5, row_mm=1.0, sod_mm=80.0, sdd_mm=160.0, det_offset_mm=0.3)
    g2 = g3.central_plane()
    rng = np.random.default_rng(1)
    m = rng.random((g3.n_views, 1, g3.n_bins)) * 5.0
    x3, log3 = O.adm3(g3, m, 0.9, 0.7, 16.0, 4.0, 40)
    r2 = O.adm(g2, m[:, 0, :], 0.9, 0.7, 16.0, 4.0, 40)
    assert np.abs(x3[0] - r2.x).max() <= 1e-9 * np.abs(r2.x).max()
    assert np.allclose(log3[:, 0], r2.log[:41, 0], rtol=1e-9, atol=0)
    assert np.allclose(log3[:, 1], r2.log[:41, 1], rtol=1e-9, atol=0)


@pytest.mark.parametrize("nonneg,step", [(True, "bb1"), (False, "bb2"), (False, "abb"),
                                         (True, "abb")])
def test_single_slice_variants_are_the_fan_beam_runs(nonneg, step):
    """The projection onto f >= 0 and the BB2 / adaptive steps: a one-slice
    volume seen by a one-row panel runs exactly the pinned 2-D variant."""
    g3 = C.ConeGeometry(nx=20, ny=18, nz=1, voxel_mm=1.0, n_views=16, n_bins=30, n_rows=1,
                        bin_mm=1.5, row_mm=1.0, sod_mm=80.0, sdd_mm=160.0, det_offset_mm=0.3)
    g2 = g3.central_plane()
    rng = np.random.default_rng(11)
    m = rng.random((g3.n_views, 1, g3.n_bins)) * 5.0 - 1.0  # inconsistent: f >= 0 binds
    x3, log3 = O.adm3(g3, m, 0.9, 0.7, 16.0, 4.0, 40, nonneg=nonneg, step=step)
    r2 = O.adm(g2, m[:, 0, :], 0.9, 0.7, 16.0, 4.0, 40, nonneg=nonneg, step=step)
    assert np.abs(x3[0] - r2.x).max() <= 1e-9 * np.abs(r2.x).max()
    assert np.allclose(log3[:, 0], r2.log[:41, 0], rtol=1e-9, atol=0)
    assert np.allclose(log3[:, 1], r2.log[:41, 1], rtol=1e-9, atol=0)
    if nonneg:
        assert x3.min() >= 0.0 and (x3 == 0.0).sum() > 0


def test_single_slice_warm_start_and_stop_rule_match_the_fan_beam_run():
    """With a start image and a tolerance the one-slice run still equals the
    pinned 2-D ADM: same start f = beta x0, same stopping iteration."""
    g3 = C.ConeGeometry(nx=16, ny=16, nz=1, voxel_mm=1.0, n_views=20, n_bins=26, n_rows=1,
                        bin_mm=1.4, row_mm=1.0, sod_mm=70.0, sdd_mm=140.0)
    g2 = g3.central_plane()
    rng = np.random.default_rng(3)
    m = rng.random((g3.n_views, 1, g3.n_bins)) * 4.0
    x0 = rng.random((1, 16, 16))
    x3, log3, k3 = O.adm3(g3, m, 1.1, 0.6, 16.0, 4.0, 400, tol=1e-3, x0=x0, with_iters=True)
    r2 = O.adm(g2, m[:, 0, :], 1.1, 0.6, 16.0, 4.0, 400, tol=1e-3, x0=x0[0])
    assert 1 < k3 < 400 and k3 == r2.iters
    assert np.abs(x3[0] - r2.x).max() <= 1e-9 * np.abs(r2.x).max()
    assert np.allclose(log3[:k3 + 1, 0], r2.log[:k3 + 1, 0], rtol=1e-9, atol=0)
    # the stop is the first iteration whose relative change (column 3, the
    # change of the step that ends before the row) falls below tol
    assert log3[k3, 3] < 1e-3 and np.all(log3[1:k3, 3] >= 1e-3)


def test_warm_start_from_a_constant_consistent_volume_is_a_fixed_point():
    """A constant volume has zero TV; with data that volume projects to, the
    start is a minimiser of Eq. 4, so the first step changes nothing (the
    gradient of Eq. 10 vanishes there with lambda = 0 and z = grad f = 0)."""
    g = SMALL3
    x0 = np.full((g.nz, g.ny, g.nx), 0.37)
    m = O.project3(g, x0)
    x, log, k = O.adm3(g, m, 1.0, 0.8, 16.0, 4.0, 3, tol=1e-12, x0=x0, with_iters=True)
    assert np.abs(x - x0).max() <= 1e-12
    assert log[0, 0] <= 1e-20 and log[1, 3] <= 1e-14 and k == 1


def test_zero_data_stays_zero():
    x, log = O.adm3(SMALL3, np.zeros((8, 5, 12)), 1.0, 1.0, 16.0, 4.0, 5)
    assert not np.any(x) and not np.any(log[:, 0])


def _dense_diffs(nx, ny, nz):
    N = nx * ny * nz
    D = [np.zeros((N, N)) for _ in range(3)]
    for z in range(nz):
        for r in range(ny):
            for c in range(nx):
                i = (z * ny + r) * nx + c
                if c >= 1:
                    D[0][i, i], D[0][i, i - 1] = 1.0, -1.0
                if r >= 1:
                    D[1][i, i], D[1][i, i - nx] = 1.0, -1.0
                if z >= 1:
                    D[2][i, i], D[2][i, i - nx * ny] = 1.0, -1.0
    return D


def _cp3(A, m, mu, D, iters):
    """Chambolle-Pock on min sum_i |(D_x f, D_y f, D_z f)_i| + mu/2 |A f - m|^2."""
    N = A.shape[1]
    K = np.vstack(D)
    tau = sig = 0.99 / np.linalg.norm(K, 2)
    Minv = np.linalg.inv(np.eye(N) + tau * mu * A.T @ A)
    Atm = A.T @ m
    f = np.zeros(N)
    fb = f.copy()
    p = np.zeros(3 * N)
    for _ in range(iters):
        p = p + sig * (K @ fb)
        q = p.reshape(3, N)
        nrm = np.maximum(1.0, np.sqrt((q * q).sum(0)))
        p = (q / nrm).reshape(-1)
        fo = f
        f = Minv @ (f - tau * (K.T @ p) + tau * mu * Atm)
        fb = 2 * f - fo
    gd = np.stack([Dk @ f for Dk in D])
    return np.sum(np.sqrt((gd * gd).sum(0))) + 0.5 * mu * np.sum((A @ f - m) ** 2)


@pytest.mark.slow
def test_reaches_the_minimum_of_eq4_in_3d():
    g = SMALL3
    N = g.nx * g.ny * g.nz
    A = np.stack([O.project3(g, np.eye(N)[i].reshape(g.nz, g.ny, g.nx)).reshape(-1)
                  for i in range(N)], axis=1)
    rng = np.random.default_rng(2)
    xt = np.zeros((g.nz, g.ny, g.nx))
    xt[1:3, 1:5, 2:5] = 1.0
    xt[2, 2:4, 3] = 2.0
    m = A @ xt.reshape(-1) + 0.05 * rng.standard_normal(A.shape[0])
    mu = 0.5
    Jstar = _cp3(A, m, mu, _dense_diffs(g.nx, g.ny, g.nz), 60000)
    _, log = O.adm3(g, m.reshape(g.n_views, g.n_rows, g.n_bins), 1.0, mu, 16.0, 4.0, 6000)
    assert abs(log[-1, 0] - Jstar) <= 1e-6 * Jstar, (log[-1, 0], Jstar)


def test_coupled_single_slice_is_the_fan_beam_coupled_run():
    g3 = C.ConeGeometry(nx=20, ny=18, nz=1, voxel_mm=1.0, n_views=16, n_bins=30, n_rows=1,
                        bin_mm=1.5, row_mm=1.0, sod_mm=80.0, sdd_mm=160.0, det_offset_mm=0.3)
    g2 = g3.central_plane()
    rng = np.random.default_rng(12)
    mh = rng.random((g3.n_views, 1, g3.n_bins)) * 5.0
    ml = rng.random((g3.n_views, 1, g3.n_bins)) * 6.0
    for nonneg in (False, True):
        x3, J3, a3 = O.adm3_coupled(g3, mh, ml, 1.0, 0.8, 0.7, 16.0, 4.0, 30, nonneg=nonneg)
        x2, J2, a2 = O.adm_coupled(g2, mh[:, 0], ml[:, 0], 1.0, 0.8, 0.7, 16.0, 4.0, 30,
                                   nonneg=nonneg)
        assert np.abs(x3[:, 0] - x2).max() <= 1e-9 * np.abs(x2).max()
        assert np.allclose(J3, J2, rtol=1e-9, atol=0) and np.allclose(a3, a2, rtol=1e-9, atol=0)


def test_coupled_with_an_empty_second_energy_is_the_single_energy_run():
    """With no data in the low energy its volume stays zero, the joint norm is
    the high energy's own, and the run is or_adm3's bit for bit."""
    g = SMALL3
    rng = np.random.default_rng(13)
    mh = rng.random((g.n_views, g.n_rows, g.n_bins)) * 4.0
    x, J, a = O.adm3_coupled(g, mh, np.zeros_like(mh), 1.0, 0.8, 0.7, 16.0, 4.0, 25)
    x1, log1 = O.adm3(g, mh, 1.0, 0.7, 16.0, 4.0, 25)
    assert not np.any(x[1]) and np.array_equal(x[0], x1)
    assert np.array_equal(J[:, 0], log1[:, 0]) and np.array_equal(a[:, 0], log1[:, 1])


def _cp3_coupled(A, m, mu, D, iters):
    """Chambolle-Pock on min sum_i |(D f_h, D f_l)_i| + mu/2 sum_e |A f_e - m_e|^2,
    the norm over the 6-vector of both energies' differences at voxel i."""
    N = A.shape[1]
    K1 = np.vstack(D)  # [3N, N]
    tau = sig = 0.99 / np.linalg.norm(K1, 2)
    Minv = np.linalg.inv(np.eye(N) + tau * mu * A.T @ A)
    f = [np.zeros(N), np.zeros(N)]
    fb = [a.copy() for a in f]
    p = [np.zeros(3 * N), np.zeros(3 * N)]
    for _ in range(iters):
        q = [p[e] + sig * (K1 @ fb[e]) for e in range(2)]
        qq = [a.reshape(3, N) for a in q]
        nrm = np.maximum(1.0, np.sqrt((qq[0] ** 2).sum(0) + (qq[1] ** 2).sum(0)))
        p = [(a / nrm).reshape(-1) for a in qq]
        for e in range(2):
            fo = f[e]
            f[e] = Minv @ (f[e] - tau * (K1.T @ p[e]) + tau * mu * (A.T @ m[e]))
            fb[e] = 2 * f[e] - fo
    gd = [np.stack([Dk @ f[e] for Dk in D]) for e in range(2)]
    tv = np.sum(np.sqrt((gd[0] ** 2).sum(0) + (gd[1] ** 2).sum(0)))
    return tv + 0.5 * mu * sum(np.sum((A @ f[e] - m[e]) ** 2) for e in range(2))


@pytest.mark.slow
def test_coupled_reaches_the_vectorial_tv_minimum():
    g = SMALL3
    N = g.nx * g.ny * g.nz
    A = np.stack([O.project3(g, np.eye(N)[i].reshape(g.nz, g.ny, g.nx)).reshape(-1)
                  for i in range(N)], axis=1)
    rng = np.random.default_rng(14)
    xt = np.zeros((g.nz, g.ny, g.nx))
    xt[1:3, 1:5, 2:5] = 1.0
    xt[2, 2:4, 3] = 2.0
    m = [A @ xt.reshape(-1) + 0.05 * rng.standard_normal(A.shape[0]),
         A @ (1.3 * xt).reshape(-1) + 0.05 * rng.standard_normal(A.shape[0])]
    mu = 0.5
    Jstar = _cp3_coupled(A, m, mu, _dense_diffs(g.nx, g.ny, g.nz), 60000)
    shp = (g.n_views, g.n_rows, g.n_bins)
    _, J, _ = O.adm3_coupled(g, m[0].reshape(shp), m[1].reshape(shp), 1.0, 1.0, mu, 16.0, 4.0,
                             6000)
    assert abs(J[-1].sum() - Jstar) <= 1e-6 * Jstar, (J[-1].sum(), Jstar)
