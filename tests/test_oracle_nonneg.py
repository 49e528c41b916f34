"""Pins of the oracle's non-negative ADM variant (every f-step projected onto
f >= 0; the images are attenuation maps):

* on a dense 16 x 16 problem whose unconstrained minimiser has negative
  pixels, the objective reaches the minimum of Eq. 4 over the non-negative
  images found by an independent algorithm (Chambolle-Pock with the data
  term in the dual and the projection as the primal step), within 1e-6;
* every returned image is non-negative where the unconstrained one is not;
* when the constraint never binds (a positive object started at itself), the
  run equals the unconstrained one bit for bit.
"""
import numpy as np
import pytest

from oracle import oracle as O

from test_oracle_adm import _dense_problem


def _chambolle_pock_nonneg(A, m, mu, n, iters):
    """min |grad f|_{2,1} + mu/2 |A f - m|^2 over f >= 0: K = [Dx; Dy; A],
    F = |.|_{2,1} (+) mu/2 |. - m|^2 handled through its conjugate, G the
    indicator of f >= 0 (prox = projection); the finite differences of Eq. 2
    built densely."""
    N = n * n
    Dx, Dy = np.zeros((N, N)), np.zeros((N, N))
    for r in range(n):
        for c in range(n):
            i = r * n + c
            if c >= 1:
                Dx[i, i], Dx[i, i - 1] = 1.0, -1.0
            if r >= 1:
                Dy[i, i], Dy[i, i - n] = 1.0, -1.0
    K = np.vstack([Dx, Dy, A])
    tau = sig = 0.99 / np.linalg.norm(K, 2)
    f = np.zeros(N)
    fb = f.copy()
    p = np.zeros(2 * N)
    q = np.zeros(A.shape[0])
    for _ in range(iters):
        y = K @ fb
        p = p + sig * y[:2 * N]
        px, py = p[:N], p[N:]
        nrm = np.maximum(1.0, np.sqrt(px * px + py * py))
        p = np.concatenate([px / nrm, py / nrm])
        q = (q + sig * y[2 * N:] - sig * m) / (1.0 + sig / mu)
        fo = f
        f = np.maximum(f - tau * (K.T @ np.concatenate([p, q])), 0.0)
        fb = 2 * f - fo
    gx, gy = Dx @ f, Dy @ f
    return np.sum(np.sqrt(gx * gx + gy * gy)) + 0.5 * mu * np.sum((A @ f - m) ** 2)


def _binding_problem():
    g, A, m = _dense_problem()
    bump = np.zeros((16, 16))
    bump[1:5, 1:5] = 1.0
    return g, A, m - 0.6 * (A @ bump.reshape(-1))


@pytest.mark.slow
def test_reaches_the_constrained_minimum():
    g, A, m = _binding_problem()
    mu = 0.5
    Jstar = _chambolle_pock_nonneg(A, m, mu, 16, 100000)
    r = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, mu, 16.0, 4.0, 2000, nonneg=True)
    assert abs(r.J[-1] - Jstar) <= 1e-6 * Jstar, (r.J[-1], Jstar)


def test_images_stay_non_negative():
    g, A, m = _binding_problem()
    r = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, 0.5, 16.0, 4.0, 300, nonneg=True)
    plain = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, 0.5, 16.0, 4.0, 300)
    assert r.x.min() >= 0.0
    assert plain.x.min() < -0.1  # the constraint binds
    assert (r.x == 0.0).sum() > 5


def test_inactive_constraint_changes_nothing():
    g, A, _ = _dense_problem()
    xt = np.full((16, 16), 1.0)
    xt[4:12, 5:11] = 2.0
    m = A @ xt.reshape(-1) + 0.01 * np.random.default_rng(3).standard_normal(A.shape[0])
    a = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, 0.5, 16.0, 4.0, 100, x0=xt, nonneg=True)
    b = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, 0.5, 16.0, 4.0, 100, x0=xt)
    assert b.x.min() > 0.5
    assert np.array_equal(a.x, b.x) and np.array_equal(a.J, b.J)
