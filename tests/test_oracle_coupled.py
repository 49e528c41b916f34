"""Pins of the oracle's coupled-TV ADM (the norm of Eq. 2 over the 4-vector of
both energies' gradients, one joint z-step):

* with the second energy's data and image zero, the coupled run is the
  single-energy run of or_adm, bit for bit (the joint norm reduces to the
  2-vector one);
* on a dense 16 x 16 two-energy problem the objective reaches the minimum
  of the coupled Eq. 4 found by an independent algorithm (Chambolle-Pock on
  the vectorial TV), within 1e-6, and that minimum differs from the
  separable one (so the pin sees the coupling).
"""
import numpy as np
import pytest

from oracle import oracle as O

from test_oracle_adm import G16, _dense_problem


def test_zero_second_energy_is_single_energy_run():
    g, A, m = _dense_problem()
    mh = m.reshape(g.n_views, g.n_bins)
    ml = np.zeros_like(mh)
    x, J, al = O.adm_coupled(g, mh, ml, 1.0, 0.8, 0.5, 16.0, 4.0, 60)
    ref = O.adm(g, mh, 1.0, 0.5, 16.0, 4.0, 60)
    assert np.array_equal(x[0], ref.x)
    assert np.array_equal(J[:, 0], ref.log[:61, 0])
    assert np.array_equal(al[:, 0], ref.log[:61, 1])
    assert not np.any(x[1])


def _cp_vectorial(A, m2, mu, n, iters):
    """min sum_i |(grad f_h, grad f_l)_i| + mu/2 sum_e |A f_e - m_e|^2 by
    Chambolle-Pock, finite differences of Eq. 2 built densely."""
    N = n * n
    Dx, Dy = np.zeros((N, N)), np.zeros((N, N))
    for r in range(n):
        for c in range(n):
            i = r * n + c
            if c >= 1:
                Dx[i, i], Dx[i, i - 1] = 1.0, -1.0
            if r >= 1:
                Dy[i, i], Dy[i, i - n] = 1.0, -1.0
    K1 = np.vstack([Dx, Dy])
    tau = sig = 0.99 / np.linalg.norm(K1, 2)
    Minv = np.linalg.inv(np.eye(N) + tau * mu * A.T @ A)
    Atm = [A.T @ m2[e] for e in (0, 1)]
    f = [np.zeros(N), np.zeros(N)]
    fb = [f[0].copy(), f[1].copy()]
    p = [np.zeros(2 * N), np.zeros(2 * N)]
    for _ in range(iters):
        q = [p[e] + sig * (K1 @ fb[e]) for e in (0, 1)]
        nrm = np.maximum(1.0, np.sqrt(q[0][:N] ** 2 + q[0][N:] ** 2 + q[1][:N] ** 2 + q[1][N:] ** 2))
        p = [np.concatenate([q[e][:N] / nrm, q[e][N:] / nrm]) for e in (0, 1)]
        for e in (0, 1):
            fo = f[e]
            f[e] = Minv @ (f[e] - tau * (K1.T @ p[e]) + tau * mu * Atm[e])
            fb[e] = 2 * f[e] - fo
    gx = [Dx @ f[e] for e in (0, 1)]
    gy = [Dy @ f[e] for e in (0, 1)]
    tv = np.sum(np.sqrt(gx[0] ** 2 + gy[0] ** 2 + gx[1] ** 2 + gy[1] ** 2))
    return tv + 0.5 * mu * sum(np.sum((A @ f[e] - m2[e]) ** 2) for e in (0, 1))


@pytest.mark.slow
def test_reaches_the_coupled_minimum():
    g, A, m = _dense_problem()
    rng = np.random.default_rng(8)
    xl = np.zeros((16, 16))
    xl[3:10, 6:13] = 1.5
    ml = A @ xl.reshape(-1) + 0.05 * rng.standard_normal(A.shape[0])
    mu = 0.5
    Jstar = _cp_vectorial(A, [m, ml], mu, 16, 100000)
    x, J, _ = O.adm_coupled(g, m.reshape(g.n_views, g.n_bins), ml.reshape(g.n_views, g.n_bins),
                            1.0, 1.0, mu, 16.0, 4.0, 3000)
    Jc = J[-1].sum()
    assert abs(Jc - Jstar) <= 1e-6 * Jstar, (Jc, Jstar)
    sep = (O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, mu, 16.0, 4.0, 3000).J[-1] +
           O.adm(g, ml.reshape(g.n_views, g.n_bins), 1.0, mu, 16.0, 4.0, 3000).J[-1])
    assert sep > Jstar * (1 + 1e-3)  # the separable minimum is a different problem's
