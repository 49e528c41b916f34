"""Pins of the oracle's decomposition (Eqs. 11-15).

D^{-1} is checked against D itself and pure materials; the Laplacian of Eq. 14
against a dense graph Laplacian assembled pair by pair; PCG against a direct
dense solve; the Prewitt edge map against a hand-drawn step.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C

PP = C.PlsParams()
ETA = (PP.eta_water_high, PP.eta_bone_high, PP.eta_water_low, PP.eta_bone_low)


def test_dinv_inverts_d():
    """Pi14: D u reproduces x for u = D^{-1} x (Eq. 12), pure materials map to
    the unit vectors."""
    rng = np.random.default_rng(0)
    xh, xl = rng.uniform(0.0, 0.1, (2, 9, 7))
    u1, u2 = O.dinv(xh, xl, *ETA)
    e1h, e2h, e1l, e2l = ETA
    assert np.abs(e1h * u1 + e2h * u2 - xh).max() <= 1e-15
    assert np.abs(e1l * u1 + e2l * u2 - xl).max() <= 1e-15
    for (a, b) in ((1.0, 0.0), (0.0, 1.0), (0.3, 0.7)):
        w1, w2 = O.dinv(np.array([e1h * a + e2h * b]), np.array([e1l * a + e2l * b]), *ETA)
        assert abs(w1[0] - a) <= 1e-12 and abs(w2[0] - b) <= 1e-12


def _dense_laplacian(er, ed):
    ny, nx = er.shape
    N = nx * ny
    L = np.zeros((N, N))
    for r in range(ny):
        for c in range(nx):
            i = r * nx + c
            for (k, w) in (((r * nx + c + 1), er[r, c]) if c + 1 < nx else (None, 0.0),
                           ((r + 1) * nx + c, ed[r, c]) if r + 1 < ny else (None, 0.0)):
                if k is None:
                    continue
                L[i, i] += w
                L[k, k] += w
                L[i, k] -= w
                L[k, i] -= w
    return L


def _weights(rng, ny, nx):
    er = rng.choice([0.1, 1.0], size=(ny, nx))
    ed = rng.choice([0.1, 1.0], size=(ny, nx))
    er[:, -1] = 0.0
    ed[-1, :] = 0.0
    return er, ed


def test_laplacian_is_the_hessian_of_r():
    """The oracle's L equals the graph Laplacian sum_pairs e (e_i - e_k)(e_i - e_k)^T
    (so R(u) = u^T L u with each pair counted twice in Eq. 14, grad R = 2 L u):
    symmetric, zero row sums, and R computed from Eq. 14 directly matches."""
    rng = np.random.default_rng(1)
    ny, nx = 6, 7
    er, ed = _weights(rng, ny, nx)
    L = _dense_laplacian(er, ed)
    N = nx * ny
    cols = np.stack([O.laplacian(er, ed, np.eye(N)[j].reshape(ny, nx)).reshape(-1)
                     for j in range(N)], axis=1)
    assert np.abs(cols - L).max() <= 1e-15
    assert np.abs(L - L.T).max() == 0.0
    assert np.abs(L.sum(axis=1)).max() <= 1e-14
    u = rng.standard_normal((ny, nx))
    R = 0.0  # Eq. 14: (1/2) sum_i sum_{k in N_i} e_ik (u_i - u_k)^2
    for r in range(ny):
        for c in range(nx):
            for (rr, cc, w) in ((r, c + 1, er[r, c] if c + 1 < nx else 0),
                                (r, c - 1, er[r, c - 1] if c >= 1 else 0),
                                (r + 1, c, ed[r, c] if r + 1 < ny else 0),
                                (r - 1, c, ed[r - 1, c] if r >= 1 else 0)):
                if w:
                    R += 0.5 * w * (u[r, c] - u[rr, cc]) ** 2
    assert abs(R - u.reshape(-1) @ L @ u.reshape(-1)) <= 1e-12 * R


@pytest.mark.parametrize("gamma", [1e-3, 1.0, 30.0])
def test_pcg_solves_eq15(gamma):
    """Pi15: PCG reaches the dense direct solution of (I + gamma L) u = b."""
    rng = np.random.default_rng(2)
    ny, nx = 16, 16
    er, ed = _weights(rng, ny, nx)
    b = rng.standard_normal((ny, nx))
    u, it, rr = O.pcg(er, ed, gamma, b, max_iter=500, tol=1e-13)
    ref = np.linalg.solve(np.eye(nx * ny) + gamma * _dense_laplacian(er, ed), b.reshape(-1))
    assert np.abs(u.reshape(-1) - ref).max() <= 1e-10 * np.abs(ref).max()
    assert rr <= 1e-13 and it > 0


def test_pls_special_cases():
    """Pi14: gamma = 0 gives the direct decomposition; a constant image gives a
    constant decomposition for any gamma (L 1 = 0)."""
    rng = np.random.default_rng(3)
    xh, xl = rng.uniform(0.01, 0.05, (2, 12, 10))
    p0 = C.PlsParams(gamma=0.0)
    u1, u2, its, _ = O.pls(xh, xl, p0)
    d1, d2 = O.dinv(xh, xl, *ETA)
    assert np.array_equal(u1, d1) and np.array_equal(u2, d2) and its == (0, 0)
    ch, cl = np.full((12, 10), 0.02), np.full((12, 10), 0.03)
    v1, v2, _, _ = O.pls(ch, cl, C.PlsParams(gamma=5.0))
    e1, e2 = O.dinv(ch, cl, *ETA)
    assert np.abs(v1 - e1).max() <= 1e-12 and np.abs(v2 - e2).max() <= 1e-12


def test_prewitt_edges_of_a_step():
    """Pi16: a vertical step marks exactly the two columns beside it; the weights
    take eps on every pair that touches them and 1 elsewhere."""
    ny, nx, c0 = 9, 12, 5
    x = np.zeros((ny, nx))
    x[:, c0:] = 1.0
    em = O.edges(x, 0.25, 0.1)
    er, ed = em.weights
    e = em.edge
    expect = np.zeros((ny, nx), dtype=bool)
    expect[:, c0 - 1] = expect[:, c0] = True
    assert np.array_equal(e.astype(bool), expect)
    eps = 0.1
    for r in range(ny):
        for c in range(nx - 1):
            touch = expect[r, c] or expect[r, c + 1]
            assert er[r, c] == (eps if touch else 1.0)
        assert er[r, nx - 1] == 0.0
    for r in range(ny - 1):
        for c in range(nx):
            assert ed[r, c] == (eps if expect[r, c] else 1.0)
    assert np.all(ed[ny - 1] == 0.0)


def test_pls_smooths_noise_inside_materials():
    """Eq. 13: raising gamma lowers the noise of the decomposed maps inside a
    flat region (the purpose of the penalty), while gamma -> 0 keeps D^{-1} x."""
    rng = np.random.default_rng(4)
    ny = nx = 32
    xh = np.full((ny, nx), PP.eta_water_high) + 0.0005 * rng.standard_normal((ny, nx))
    xl = np.full((ny, nx), PP.eta_water_low) + 0.0005 * rng.standard_normal((ny, nx))
    sds = []
    for gamma in (0.0, 1.0, 10.0):
        u1, u2, _, _ = O.pls(xh, xl, C.PlsParams(gamma=gamma, edge_tau=2.0))
        sds.append(u2.std())
    assert sds[0] > sds[1] > sds[2]


def test_prewitt_magnitude_is_scipys():
    """The squared gradient magnitude that decides the edges is the Prewitt
    operator of scipy.ndimage with replicated borders ('nearest'), and the
    threshold is tau^2 times its maximum."""
    from scipy import ndimage
    rng = np.random.default_rng(12)
    x = rng.standard_normal((13, 17))
    em = O.edges(x, 0.3, 0.1)
    gx = ndimage.prewitt(x, axis=1, mode="nearest")
    gy = ndimage.prewitt(x, axis=0, mode="nearest")
    m2 = gx * gx + gy * gy
    assert np.abs(em.m2 - m2).max() <= 1e-12 * m2.max()
    assert abs(em.thr - 0.09 * m2.max()) <= 1e-12 * m2.max()
    assert np.array_equal(em.edge.astype(bool), em.m2 > em.thr)
