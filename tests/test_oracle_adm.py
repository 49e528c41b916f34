"""Pins of the oracle's TV operators and ADM iteration (Eqs. 2-10).

The pins come from outside the oracle: adjoint identities and closed forms
of the finite differences, a brute-force minimisation for the shrinkage, a
consistent-data fixed point, the exact line-search identity of the BB step,
and an independent solver (Chambolle-Pock primal-dual, dense NumPy) that
reaches the minimum of Eq. 4 on a 16x16 problem.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

G16 = C.Geometry(nx=16, ny=16, pixel_mm=1.0, n_views=8, n_bins=24, bin_mm=1.5, sod_mm=60.0,
                 sdd_mm=120.0)


def test_grad_adjoint_and_closed_forms():
    """Pi6: <grad x, p> = <x, grad^T p>; TV(const) = 0; TV of a vertical step of
    height h over ny rows is ny*h; grad^T grad 1 = 0."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((23, 31))
    px, py = rng.standard_normal((2, 23, 31))
    gx, gy = O.grad(x)
    lhs = np.sum(gx * px) + np.sum(gy * py)
    rhs = np.sum(x * O.gradT(px, py))
    assert abs(lhs - rhs) <= 1e-14 * max(abs(lhs), 1.0) * 100
    assert O.tv(np.full((9, 11), 3.7)) == 0.0
    step = np.zeros((13, 20))
    step[:, 8:] = 0.25
    assert O.tv(step) == 13 * 0.25
    one = np.ones((7, 9))
    assert np.abs(O.gradT(*O.grad(one))).max() == 0.0
    # backward differences: first column/row have zero difference
    gx, gy = O.grad(x)
    assert np.all(gx[:, 0] == 0) and np.all(gy[0, :] == 0)
    assert np.allclose(gx[:, 1:], x[:, 1:] - x[:, :-1], rtol=0, atol=0)


def _brute_min(v, rho):
    """argmin |z| + rho/2 |z - v|^2 by nested grid refinement."""
    obj = lambda zx, zy: np.sqrt(zx * zx + zy * zy) + 0.5 * rho * ((zx - v[0]) ** 2 + (zy - v[1]) ** 2)
    cx, cy, half = 0.0, 0.0, 2.0 * (abs(v[0]) + abs(v[1]) + 1.0)
    for _ in range(12):
        xs = np.linspace(cx - half, cx + half, 81)
        ys = np.linspace(cy - half, cy + half, 81)
        X, Y = np.meshgrid(xs, ys)
        k = np.argmin(obj(X, Y))
        cx, cy = X.flat[k], Y.flat[k]
        half /= 8.0
    return np.array([cx, cy])


def test_shrink_is_the_exact_minimiser():
    """Pi7/Pi9: the closed form of Eq. 8 matches brute-force minimisation, is
    zero inside the ball |v| <= 1/rho, and no perturbation lowers the
    z-subproblem objective."""
    rng = np.random.default_rng(1)
    for rho in (0.7, 4.0, 64.0):
        for _ in range(6):
            v = rng.standard_normal(2) * rng.choice([0.01, 0.3, 2.0])
            zx, zy = O.shrink(np.array([v[0]]), np.array([v[1]]), 1.0 / rho)
            z = np.array([zx[0], zy[0]])
            zb = _brute_min(v, rho)
            assert np.abs(z - zb).max() <= 1e-7 * (1.0 + np.abs(v).max())  # flat minimum: sqrt(eps)
            f = lambda q: np.linalg.norm(q) + 0.5 * rho * np.sum((q - v) ** 2)
            for _ in range(20):
                assert f(z) <= f(z + 1e-3 * rng.standard_normal(2)) + 1e-15
    zx, zy = O.shrink(np.array([0.1, 0.0]), np.array([0.05, 0.0]), 0.2)
    assert zx[0] == 0 and zy[0] == 0 and zx[1] == 0 and zy[1] == 0


def test_fixed_point_on_consistent_data():
    """Pi8: with g = A(c 1) and f0 = c 1 the gradient of Eq. 9 vanishes and the
    iteration does not move."""
    g = G16
    c = 0.3
    x0 = np.full((g.ny, g.nx), c)
    m = O.project(g, x0)
    r = O.adm(g, m, 1.0, 2.0, 8.0, 8.0, 30, x0=x0)
    assert np.abs(r.x - x0).max() <= 1e-13
    assert np.all(r.log[:30, 4] <= 1e-10)  # |G^k|


def _tiny_run(e=1, iters=200):
    s = P.make_slice(C.TINY, 0)
    p = C.default_adm_params(C.TINY, iters)
    beta = p.beta_high if e == 0 else p.beta_low
    return s, p, O.adm(C.TINY, s.sino[e], beta, p.mu, p.rho, p.xi, iters)


@pytest.mark.parametrize("energy", [0, 1])
def test_objective_decreases_by_blocks_and_residual_vanishes(energy):
    """Pi10/Pi12: BB steps are not monotone step by step, but the smallest
    J(f^k) of each block of 20 iterations falls strictly from block to block;
    the primal residual |grad f - z| falls by orders of magnitude and the image
    approaches the phantom."""
    s, p, r = _tiny_run(energy, 200)
    J = r.J
    block_min = np.array([J[i:i + 20].min() for i in range(0, 200, 20)])
    assert np.all(np.diff(block_min) < 0), block_min
    assert J[-1] < 1e-2 * J[0]
    pres = r.log[:200, 2]
    assert pres[-1] < 1e-2 * pres[1:10].max()
    err = np.linalg.norm(r.x - s.x_true[energy]) / np.linalg.norm(s.x_true[energy])
    assert err < 0.06


def test_bb_step_equals_delayed_cauchy_step():
    """Pi13: the BB1 step <s,s>/<s,y> after step k equals the exact line-search
    step along G^k, |G|^2 / (mu |A G|^2 + rho |grad G|^2).  G^k is rebuilt here
    from the oracle's primitives and the state after k iterations."""
    g = C.TINY
    s = P.make_slice(g, 0)
    p = C.default_adm_params(g, 1)
    beta = p.beta_low
    m = s.sino[1]
    for k in (0, 3, 17):
        run_k = O.adm(g, m, beta, p.mu, p.rho, p.xi, k) if k > 0 else None
        run_next = O.adm(g, m, beta, p.mu, p.rho, p.xi, k + 2)
        if k == 0:
            f = np.zeros((g.ny, g.nx))
            lam = np.zeros((2, g.ny, g.nx))
        else:
            f = beta * run_k.x
            # the multiplier after k steps, as the oracle returns it
            lam = run_k.lam
        d = O.grad(f)
        zx, zy = O.shrink(d[0] - lam[0] / p.rho, d[1] - lam[1] / p.rho, 1.0 / p.rho)
        h = p.mu * O.backproject(g, O.project(g, f) - beta * m)
        G = h + O.gradT(p.rho * (d[0] - zx) - lam[0], p.rho * (d[1] - zy) - lam[1])
        AG = O.project(g, G)
        gx, gy = O.grad(G)
        cauchy = np.sum(G * G) / (p.mu * np.sum(AG * AG) + p.rho * (np.sum(gx * gx) + np.sum(gy * gy)))
        alpha_next = run_next.log[k + 1, 1]
        assert abs(alpha_next - cauchy) <= 1e-9 * cauchy, (k, alpha_next, cauchy)
        if k == 0:
            assert abs(run_next.log[0, 1] - cauchy) <= 1e-12 * cauchy


def _dense_problem():
    g = G16
    n, N = 16, 256
    A = np.stack([O.project(g, np.eye(N)[i].reshape(n, n)).reshape(-1) for i in range(N)], axis=1)
    rng = np.random.default_rng(0)
    xt = np.zeros((n, n))
    xt[4:12, 5:11] = 1.0
    xt[7:9, 7:9] = 2.0
    m = A @ xt.reshape(-1) + 0.05 * rng.standard_normal(A.shape[0])
    return g, A, m


def _chambolle_pock(A, m, mu, n, iters):
    """Primal-dual solver of min |grad f|_{2,1} + mu/2 |A f - m|^2 with the
    finite differences of Eq. 2 built densely (independent of the oracle)."""
    N = n * n
    Dx, Dy = np.zeros((N, N)), np.zeros((N, N))
    for r in range(n):
        for c in range(n):
            i = r * n + c
            if c >= 1:
                Dx[i, i], Dx[i, i - 1] = 1.0, -1.0
            if r >= 1:
                Dy[i, i], Dy[i, i - n] = 1.0, -1.0
    K = np.vstack([Dx, Dy])
    tau = sig = 0.99 / np.linalg.norm(K, 2)
    Minv = np.linalg.inv(np.eye(N) + tau * mu * A.T @ A)
    Atm = A.T @ m
    f = np.zeros(N)
    fb = f.copy()
    p = np.zeros(2 * N)
    for _ in range(iters):
        p = p + sig * (K @ fb)
        px, py = p[:N], p[N:]
        nrm = np.maximum(1.0, np.sqrt(px * px + py * py))
        p = np.concatenate([px / nrm, py / nrm])
        fo = f
        f = Minv @ (f - tau * (K.T @ p) + tau * mu * Atm)
        fb = 2 * f - fo
    gx, gy = Dx @ f, Dy @ f
    return np.sum(np.sqrt(gx * gx + gy * gy)) + 0.5 * mu * np.sum((A @ f - m) ** 2)


@pytest.mark.slow
def test_adm_reaches_the_minimum_of_eq4():
    """Pi11: ADM's objective converges to the minimum J* of Eq. 4 found by an
    independent algorithm (Chambolle-Pock, 10^5 iterations), within 1e-6."""
    g, A, m = _dense_problem()
    mu = 0.5
    Jstar = _chambolle_pock(A, m, mu, 16, 100000)
    r = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, mu, 16.0, 4.0, 20000)
    assert abs(r.J[-1] - Jstar) <= 1e-6 * Jstar, (r.J[-1], Jstar)


def test_beta_scaling_identity():
    """Eq. 3: with f = beta x and g = beta m, shrink(beta v, t) = beta shrink(v,
    t/beta) gives z_f = beta z_x, the same G, alpha_f = beta alpha_x and the
    same multiplier, so a run with weight beta and (mu, rho, xi) equals the
    beta = 1 run with (beta mu, beta rho, beta xi); J scales by beta."""
    g = G16
    _, A, m = _dense_problem()
    m = m.reshape(g.n_views, g.n_bins)
    beta = 0.5
    r1 = O.adm(g, m, beta, 2.0, 8.0, 8.0, 40)
    r2 = O.adm(g, m, 1.0, 2.0 * beta, 8.0 * beta, 8.0 * beta, 40)
    assert np.abs(r1.x - r2.x).max() <= 1e-10 * np.abs(r2.x).max()
    assert np.allclose(r1.J, beta * r2.J, rtol=1e-10, atol=0)


def _g_and_parts(g, m, beta, p, k):
    """G^k rebuilt from the oracle's primitives and its state after k
    iterations, with A G and grad G."""
    if k == 0:
        f = np.zeros((g.ny, g.nx))
        lam = np.zeros((2, g.ny, g.nx))
    else:
        run_k = O.adm(g, m, beta, p.mu, p.rho, p.xi, k)
        f, lam = beta * run_k.x, run_k.lam
    d = O.grad(f)
    zx, zy = O.shrink(d[0] - lam[0] / p.rho, d[1] - lam[1] / p.rho, 1.0 / p.rho)
    h = p.mu * O.backproject(g, O.project(g, f) - beta * m)
    G = h + O.gradT(p.rho * (d[0] - zx) - lam[0], p.rho * (d[1] - zy) - lam[1])
    AG = O.project(g, G)
    gx, gy = O.grad(G)
    return G, AG, gx, gy


def test_bb2_and_adaptive_steps():
    """The BB2 step <s,y>/<y,y> after step k, for s = -alpha G^k and y = (mu
    A^T A + rho grad^T grad) s, equals (mu |A G|^2 + rho |grad G|^2) / |mu A^T
    A G + rho grad^T grad G|^2; the adaptive rule takes it where it is below
    half the BB1 (Cauchy) step and the BB1 step otherwise."""
    g = C.TINY
    s = P.make_slice(g, 0)
    p = C.default_adm_params(g, 1)
    beta = p.beta_low
    m = s.sino[1]
    for k in (0, 3, 17):
        G, AG, gx, gy = _g_and_parts(g, m, beta, p, k)
        den = p.mu * np.sum(AG * AG) + p.rho * (np.sum(gx * gx) + np.sum(gy * gy))
        ytil = p.mu * O.backproject(g, AG) + p.rho * O.gradT(gx, gy)
        bb1, bb2 = np.sum(G * G) / den, den / np.sum(ytil * ytil)
        assert bb2 <= bb1 * (1 + 1e-12)  # Cauchy-Schwarz
        for step, want in (("bb2", bb2), ("abb", bb2 if bb2 / bb1 < 0.5 else bb1)):
            run_k = O.adm(g, m, beta, p.mu, p.rho, p.xi, k, step=step) if k > 0 else None
            if k > 0:
                # the state after k steps of this rule differs from the BB1 one:
                # rebuild G^k from the rule's own run
                f, lam = beta * run_k.x, run_k.lam
                d = O.grad(f)
                zx, zy = O.shrink(d[0] - lam[0] / p.rho, d[1] - lam[1] / p.rho, 1.0 / p.rho)
                h = p.mu * O.backproject(g, O.project(g, f) - beta * m)
                G = h + O.gradT(p.rho * (d[0] - zx) - lam[0], p.rho * (d[1] - zy) - lam[1])
                AG = O.project(g, G)
                gx, gy = O.grad(G)
                den = p.mu * np.sum(AG * AG) + p.rho * (np.sum(gx * gx) + np.sum(gy * gy))
                ytil = p.mu * O.backproject(g, AG) + p.rho * O.gradT(gx, gy)
                b1, b2 = np.sum(G * G) / den, den / np.sum(ytil * ytil)
                want = b2 if step == "bb2" else (b2 if b2 / b1 < 0.5 else b1)
            run_next = O.adm(g, m, beta, p.mu, p.rho, p.xi, k + 2, step=step)
            assert abs(run_next.log[k + 1, 1] - want) <= 1e-9 * want, (step, k)


@pytest.mark.slow
@pytest.mark.parametrize("step", ["bb2", "abb"])
def test_bb2_and_adaptive_reach_the_minimum(step):
    """With either step rule ADM still reaches the minimum J* of Eq. 4 found
    by Chambolle-Pock, within 1e-6."""
    g, A, m = _dense_problem()
    mu = 0.5
    Jstar = _chambolle_pock(A, m, mu, 16, 100000)
    r = O.adm(g, m.reshape(g.n_views, g.n_bins), 1.0, mu, 16.0, 4.0, 20000, step=step)
    assert abs(r.J[-1] - Jstar) <= 1e-6 * Jstar, (r.J[-1], Jstar)
