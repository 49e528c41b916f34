"""Pins of the oracle's attenuation-space decomposition (|x - Du|^2 +
gamma R(u), both materials coupled through D^T D) against what fixes it
independently of the oracle's code:

* the exact solution of its linear system (D^T D (x) I + gamma I (x) L) u =
  D^T x, assembled here from the definitions (the 2 x 2 matrix D of Eq. 12 and
  the edge-weighted 4-neighbour Laplacian of Eq. 14) and solved with a sparse
  direct solver, on random images and weights;
* gamma = 0 gives the direct decomposition D^{-1} x;
* an image of one pure material gives that material's unit map for any gamma.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1607_01650_amd import configs as C

ETA = (C.PlsParams().eta_water_high, C.PlsParams().eta_bone_high,
       C.PlsParams().eta_water_low, C.PlsParams().eta_bone_low)


def _laplacian(er, ed):
    """Sparse L with (L u)_i = sum over the 4-neighbours k of e_ik (u_i - u_k)."""
    ny, nx = er.shape
    N = nx * ny
    rows, cols, vals = [], [], []
    for r in range(ny):
        for c in range(nx):
            i = r * nx + c
            for (rr, cc, w) in ((r, c + 1, er[r, c] if c + 1 < nx else 0.0),
                                (r + 1, c, ed[r, c] if r + 1 < ny else 0.0)):
                if w == 0.0:
                    continue
                k = rr * nx + cc
                rows += [i, k, i, k]
                cols += [i, k, k, i]
                vals += [w, w, -w, -w]
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def _exact(er, ed, gamma, xh, xl):
    e1h, e2h, e1l, e2l = ETA
    D = np.array([[e1h, e2h], [e1l, e2l]])
    G = D.T @ D
    N = xh.size
    A = sp.kron(sp.csr_matrix(G), sp.identity(N)) + gamma * sp.kron(sp.identity(2),
                                                                     _laplacian(er, ed))
    rhs = np.concatenate([D[0, 0] * xh.ravel() + D[1, 0] * xl.ravel(),
                          D[0, 1] * xh.ravel() + D[1, 1] * xl.ravel()])
    u = spla.spsolve(A.tocsc(), rhs)
    return u[:N].reshape(xh.shape), u[N:].reshape(xh.shape)


def _weights(rng, ny, nx, eps=0.1):
    er = np.where(rng.random((ny, nx)) < 0.2, eps, 1.0)
    ed = np.where(rng.random((ny, nx)) < 0.2, eps, 1.0)
    er[:, -1] = 0.0
    ed[-1, :] = 0.0
    return er, ed


@pytest.mark.parametrize("gamma", [1e-4, 1e-3, 0.05])
@pytest.mark.parametrize("shape", [(10, 12), (48, 40)], ids=["10x12", "48x40"])
def test_matches_direct_solve(gamma, shape):
    rng = np.random.default_rng(5)
    ny, nx = shape
    er, ed = _weights(rng, ny, nx)
    xh = 0.02 + 0.01 * rng.standard_normal((ny, nx))
    xl = 0.025 + 0.015 * rng.standard_normal((ny, nx))
    u1, u2, it, rel = O.pcg_att(er, ed, ETA, gamma, xh, xl, max_iter=2000, tol=1e-13)
    r1, r2 = _exact(er, ed, gamma, xh, xl)
    scale = max(np.abs(r1).max(), np.abs(r2).max())
    assert np.abs(u1 - r1).max() <= 1e-9 * scale
    assert np.abs(u2 - r2).max() <= 1e-9 * scale
    assert it > 0


def test_gamma_zero_is_direct():
    rng = np.random.default_rng(6)
    er, ed = _weights(rng, 20, 17)
    xh, xl = rng.random((20, 17)) * 0.05, rng.random((20, 17)) * 0.08
    u1, u2, _, _ = O.pcg_att(er, ed, ETA, 0.0, xh, xl)
    d1, d2 = O.dinv(xh, xl, *ETA)
    assert np.abs(u1 - d1).max() <= 1e-12 * np.abs(d1).max()
    assert np.abs(u2 - d2).max() <= 1e-12 * np.abs(d2).max()


@pytest.mark.parametrize("material", [0, 1])
def test_pure_material(material):
    rng = np.random.default_rng(7)
    er, ed = _weights(rng, 16, 16)
    e1h, e2h, e1l, e2l = ETA
    xh = np.full((16, 16), e1h if material == 0 else e2h)
    xl = np.full((16, 16), e1l if material == 0 else e2l)
    u1, u2, _, _ = O.pcg_att(er, ed, ETA, 0.3, xh, xl)
    assert np.abs(u1 - (1.0 if material == 0 else 0.0)).max() <= 1e-10
    assert np.abs(u2 - (0.0 if material == 0 else 1.0)).max() <= 1e-10
