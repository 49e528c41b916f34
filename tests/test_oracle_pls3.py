"""Pins of the oracle's 3-D PLS pieces (Eqs. 13-15 on a volume, R of Eq. 14
over the six face neighbours, edges from the 3-D Prewitt operator):

* a step along z (constant in-plane) marks exactly the two slices beside the
  step; a step along x marks exactly the two columns beside it in every row
  and slice; a constant volume has no edges;
* the six-neighbour Laplacian's quadratic form equals R(u) of Eq. 14 summed
  pair by pair over the face neighbours; L 1 = 0; on a one-slice volume it is
  the 2-D Laplacian, bit for bit;
* PCG solves (I + gamma L) u = b as numpy.linalg.solve does on the dense
  matrix assembled pair by pair;
* the attenuation-space system on a volume, (D^T D (x) I + gamma I (x) L) u
  = D^T x, is solved as numpy.linalg.solve does on that matrix assembled from
  the 2 x 2 D of Eq. 12 and the pairwise L; gamma = 0 gives D^{-1} x; a
  one-slice volume gives the 2-D solver's result bit for bit.
"""
import numpy as np

from oracle import oracle as O
from paper_1607_01650_amd import configs as C

ETA = (C.PlsParams().eta_water_high, C.PlsParams().eta_bone_high,
       C.PlsParams().eta_water_low, C.PlsParams().eta_bone_low)


def test_z_step_marks_two_slices():
    x = np.zeros((9, 7, 8))
    x[4:] = 1.0
    em = O.edges3(x, 0.25, 0.1)
    ex, ey, ez = em.weights
    e = em.edge
    want = np.zeros_like(e)
    want[3:5] = 1
    assert np.array_equal(e, want)
    assert np.all(ez[2:5] == 0.1) and np.all(ez[5:8] == 1.0) and np.all(ez[8] == 0.0)
    assert np.all(ez[:2] == 1.0)


def test_x_step_marks_two_columns():
    x = np.zeros((5, 6, 10))
    x[:, :, 6:] = 2.0
    e = O.edges3(x, 0.25, 0.1).edge
    want = np.zeros_like(e)
    want[:, :, 5:7] = 1
    assert np.array_equal(e, want)
    e0 = O.edges3(np.full((4, 5, 6), 3.0), 0.25, 0.1).edge
    assert not e0.any()


def test_prewitt3_magnitude_is_scipys():
    """Each axis's derivative is scipy.ndimage's Prewitt operator along it
    (the difference of the neighbouring faces, each face summed over the
    other two axes), with replicated borders."""
    from scipy import ndimage
    rng = np.random.default_rng(13)
    x = rng.standard_normal((6, 7, 9))
    em = O.edges3(x, 0.3, 0.1)
    m2 = sum(ndimage.prewitt(x, axis=a, mode="nearest") ** 2 for a in range(3))
    assert np.abs(em.m2 - m2).max() <= 1e-12 * m2.max()
    assert np.array_equal(em.edge.astype(bool), em.m2 > em.thr)


def _pairs(nx, ny, nz):
    P = nx * ny
    for z in range(nz):
        for r in range(ny):
            for c in range(nx):
                i = z * P + r * nx + c
                if c + 1 < nx:
                    yield 0, i, i + 1
                if r + 1 < ny:
                    yield 1, i, i + nx
                if z + 1 < nz:
                    yield 2, i, i + P


def test_laplacian_is_eq14_pairwise():
    rng = np.random.default_rng(0)
    nz, ny, nx = 4, 5, 6
    w = [rng.random((nz, ny, nx)) for _ in range(3)]
    for a, idx in ((0, np.s_[:, :, -1]), (1, np.s_[:, -1, :]), (2, np.s_[-1, :, :])):
        w[a][idx] = 0.0
    u = rng.random((nz, ny, nx))
    Lu = O.laplacian3(w[0], w[1], w[2], u)
    uf, wf = u.reshape(-1), [a.reshape(-1) for a in w]
    R = sum(wf[a][i] * (uf[i] - uf[k]) ** 2 for a, i, k in _pairs(nx, ny, nz))
    assert abs(np.sum(u * Lu) - R) <= 1e-12 * R
    assert np.abs(O.laplacian3(w[0], w[1], w[2], np.ones_like(u))).max() <= 1e-14
    one = [a[:1] for a in w]
    assert np.array_equal(O.laplacian3(one[0], one[1], np.zeros_like(one[2]), u[:1])[0],
                          O.laplacian(one[0][0], one[1][0], u[0]))


def test_pcg3_matches_dense_solve():
    rng = np.random.default_rng(1)
    nz, ny, nx = 4, 5, 6
    N = nx * ny * nz
    w = [np.where(rng.random((nz, ny, nx)) < 0.2, 0.1, 1.0) for _ in range(3)]
    w[0][:, :, -1] = 0.0
    w[1][:, -1, :] = 0.0
    w[2][-1] = 0.0
    gamma = 0.7
    A = np.eye(N)
    wf = [a.reshape(-1) for a in w]
    for a, i, k in _pairs(nx, ny, nz):
        A[i, i] += gamma * wf[a][i]
        A[k, k] += gamma * wf[a][i]
        A[i, k] -= gamma * wf[a][i]
        A[k, i] -= gamma * wf[a][i]
    b = rng.standard_normal((nz, ny, nx))
    u, it, rr = O.pcg3(w[0], w[1], w[2], gamma, b, 500, 1e-13)
    ref = np.linalg.solve(A, b.reshape(-1)).reshape(nz, ny, nx)
    assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max() and rr <= 1e-13 and it < 500


def _vol_weights(rng, nz, ny, nx):
    w = [np.where(rng.random((nz, ny, nx)) < 0.2, 0.1, 1.0) for _ in range(3)]
    w[0][:, :, -1] = 0.0
    w[1][:, -1, :] = 0.0
    w[2][-1] = 0.0
    return w


def test_attenuation_solver_matches_dense_solve():
    rng = np.random.default_rng(3)
    nz, ny, nx = 3, 5, 4
    N = nx * ny * nz
    w = _vol_weights(rng, nz, ny, nx)
    gamma = 2e-3
    L = np.zeros((N, N))
    wf = [a.reshape(-1) for a in w]
    for a, i, k in _pairs(nx, ny, nz):
        L[i, i] += wf[a][i]
        L[k, k] += wf[a][i]
        L[i, k] -= wf[a][i]
        L[k, i] -= wf[a][i]
    e1h, e2h, e1l, e2l = ETA
    D = np.array([[e1h, e2h], [e1l, e2l]])
    A = np.kron(D.T @ D, np.eye(N)) + gamma * np.kron(np.eye(2), L)
    xh = 0.02 + 0.01 * rng.random((nz, ny, nx))
    xl = 0.025 + 0.02 * rng.random((nz, ny, nx))
    rhs = np.concatenate([D[0, 0] * xh.ravel() + D[1, 0] * xl.ravel(),
                          D[0, 1] * xh.ravel() + D[1, 1] * xl.ravel()])
    ref = np.linalg.solve(A, rhs)
    u1, u2, it, rr = O.pcg_att3(w[0], w[1], w[2], ETA, gamma, xh, xl, 2000, 1e-14)
    got = np.concatenate([u1.ravel(), u2.ravel()])
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max() and rr <= 1e-14 and it < 2000
    # gamma = 0: the direct decomposition
    d1, d2 = O.dinv(xh, xl, *ETA)
    z1, z2, _, _ = O.pcg_att3(w[0], w[1], w[2], ETA, 0.0, xh, xl, 50, 1e-14)
    assert np.abs(z1 - d1).max() <= 1e-12 * np.abs(d1).max()
    assert np.abs(z2 - d2).max() <= 1e-12 * np.abs(d2).max()


def test_attenuation_solver_one_slice_is_2d():
    rng = np.random.default_rng(4)
    ny, nx = 9, 11
    w = _vol_weights(rng, 1, ny, nx)
    w[2][:] = 0.0
    xh = 0.02 + 0.01 * rng.random((1, ny, nx))
    xl = 0.025 + 0.02 * rng.random((1, ny, nx))
    a1, a2, ia, ra = O.pcg_att3(w[0], w[1], w[2], ETA, 1e-3, xh, xl, 200, 1e-12)
    b1, b2, ib, rb = O.pcg_att(w[0][0], w[1][0], ETA, 1e-3, xh[0], xl[0], 200, 1e-12)
    assert ia == ib and np.array_equal(a1[0], b1) and np.array_equal(a2[0], b2)
