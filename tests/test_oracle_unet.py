"""Pins of the network oracle (oracle/unet_ref.py) on the CPU, in FP64.

The oracle's functions are held to facts that do not depend on the oracle:
* conv is 'same'-padded cross-correlation: scipy.signal.correlate2d per
  channel pair, and a brute-force loop with explicit zero padding;
* conv_dx and conv_dw are conv's adjoint and weight gradient:
  <conv(x, w), dz> = <x, conv_dx(dz, w)> = <w, conv_dw(dz, x)>, and the bias
  gradient is the sum of dz;
* pool is the 2x2 maximum (first maximum on ties); pool_dx is its adjoint at
  the fixed argmax pattern and puts each gradient on that maximum only;
* shuffle is the depth-to-space permutation (brute force) and unshuffle its
  inverse and adjoint;
* unet_backward is the gradient of unet_forward: central differences of a
  tiny U-Net's loss <y, dy> per layer, with the bfloat16 rounding switched off;
* adam follows the bias-corrected closed form: a constant gradient g moves
  every weight by exactly lr * g / (|g| + eps) on every step;
* the unrolled ADM oracle with the BB steps logged by or_adm reproduces
  or_adm's iterates (the same Eq. 10 sequence, assembled from other code).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_ref as U


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- conv
@pytest.mark.parametrize("k", [1, 3])
def test_conv_is_same_padded_cross_correlation(k):
    rng = _rng(1)
    N, H, W, Ci, Co, CoP = 2, 5, 7, 3, 4, 16
    x = rng.standard_normal((N, H, W, Ci))
    w = np.zeros((k * k, CoP, Ci))
    w[:, :Co] = rng.standard_normal((k * k, Co, Ci))
    w[:, Co:] = 99.0  # padding rows beyond cout must never be read
    b = np.zeros(CoP)
    b[:Co] = rng.standard_normal(Co)
    y = U.conv(x, w, b, Co, k)
    ref = np.zeros((N, H, W, Co))
    for n in range(N):
        for co in range(Co):
            ref[n, :, :, co] = b[co]
            for ci in range(Ci):
                ker = w[:, co, ci].reshape(k, k)
                ref[n, :, :, co] += correlate2d(x[n, :, :, ci], ker, mode="same")
    assert np.abs(y - ref).max() <= 1e-12
    # brute force with explicit zero padding
    p = k // 2
    bf = np.zeros((N, H, W, Co))
    for n in range(N):
        for h in range(H):
            for ww in range(W):
                for co in range(Co):
                    acc = b[co]
                    for dy in range(k):
                        for dx in range(k):
                            yy, xx = h + dy - p, ww + dx - p
                            if 0 <= yy < H and 0 <= xx < W:
                                acc += float(np.dot(x[n, yy, xx, :], w[dy * k + dx, co, :]))
                    bf[n, h, ww, co] = acc
    assert np.abs(y - bf).max() <= 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_conv_gradients_are_adjoints(k):
    rng = _rng(2)
    N, H, W, Ci, Co, CoP = 2, 6, 5, 5, 3, 16
    x = rng.standard_normal((N, H, W, Ci))
    dz = rng.standard_normal((N, H, W, Co))
    w = np.zeros((k * k, CoP, Ci))
    w[:, :Co] = rng.standard_normal((k * k, Co, Ci))
    y = U.conv(x, w, None, Co, k)
    lhs = float(np.sum(y * dz))
    dx = U.conv_dx(dz, w, Ci, k)
    dw, db = U.conv_dw(dz, x, k, CoP)
    assert dx.shape == x.shape and dw.shape == w.shape
    assert abs(lhs - float(np.sum(x * dx))) <= 1e-12 * abs(lhs) + 1e-12
    assert abs(lhs - float(np.sum(w * dw))) <= 1e-12 * abs(lhs) + 1e-12
    assert np.all(dw[:, Co:] == 0)
    assert np.allclose(db[:Co], dz.sum(axis=(0, 1, 2)), rtol=0, atol=1e-12)
    assert np.all(db[Co:] == 0)


def test_conv_gradient_of_bias_by_difference():
    """y = conv(x, w, b): dL/db[co] of L = <y, dz> is sum dz[..., co]; checked by a
    difference of two forward passes (L is linear in b, so it is exact)."""
    rng = _rng(3)
    x = rng.standard_normal((1, 4, 4, 2))
    w = np.zeros((9, 16, 2))
    w[:, :3] = rng.standard_normal((9, 3, 2))
    dz = rng.standard_normal((1, 4, 4, 3))
    _, db = U.conv_dw(dz, x, 3, 16)
    b0 = np.zeros(16)
    for co in range(3):
        b1 = b0.copy()
        b1[co] = 1.0
        d = np.sum(U.conv(x, w, b1, 3, 3) * dz) - np.sum(U.conv(x, w, b0, 3, 3) * dz)
        assert abs(d - db[co]) <= 1e-12


# ---------------------------------------------------------------- pool / shuffle
def test_pool_is_blockwise_max_first_wins():
    rng = _rng(4)
    x = rng.integers(0, 3, (2, 6, 8, 3)).astype(np.float64)  # many ties
    y, idx = U.pool(x)
    for n in range(2):
        for i in range(3):
            for j in range(4):
                for c in range(3):
                    blk = [x[n, 2 * i, 2 * j, c], x[n, 2 * i, 2 * j + 1, c],
                           x[n, 2 * i + 1, 2 * j, c], x[n, 2 * i + 1, 2 * j + 1, c]]
                    m = max(blk)
                    assert y[n, i, j, c] == m
                    assert idx[n, i, j, c] == blk.index(m)  # raster order, first wins


def test_pool_dx_routes_to_the_maximum_and_is_adjoint():
    rng = _rng(5)
    x = rng.standard_normal((2, 6, 4, 3))
    y, idx = U.pool(x)
    dy = rng.standard_normal(y.shape)
    dx = U.pool_dx(dy, idx)
    assert dx.shape == x.shape
    for n in range(2):
        for i in range(3):
            for j in range(2):
                for c in range(3):
                    blk = x[n, 2 * i:2 * i + 2, 2 * j:2 * j + 2, c]
                    r, s = np.unravel_index(np.argmax(blk), (2, 2))
                    g = dx[n, 2 * i:2 * i + 2, 2 * j:2 * j + 2, c]
                    assert g[r, s] == dy[n, i, j, c]
                    assert np.count_nonzero(g) == (1 if dy[n, i, j, c] != 0 else 0)
    # adjoint of the linear map x -> x[argmax] at the fixed pattern
    sel = U.pool_dx(np.ones_like(y), idx)  # 1 at every selected position
    v = rng.standard_normal(x.shape)
    picked = U.pool_dx(np.ones_like(y), idx) * v
    yv = picked.reshape(2, 3, 2, 2, 2, 3).transpose(0, 1, 3, 2, 4, 5).reshape(2, 3, 2, 4, 3).sum(3)
    assert abs(np.sum(yv * dy) - np.sum(v * dx)) <= 1e-12
    assert sel.sum() == y.size


def test_shuffle_is_depth_to_space_and_unshuffle_inverts_it():
    rng = _rng(6)
    N, H, W, C = 2, 3, 4, 5
    t = rng.standard_normal((N, H, W, 4 * C))
    s = U.shuffle(t, C)
    for n in range(N):
        for h in range(H):
            for w in range(W):
                for i in range(2):
                    for j in range(2):
                        for c in range(C):
                            assert s[n, 2 * h + i, 2 * w + j, c] == t[n, h, w, (2 * i + j) * C + c]
    assert np.array_equal(U.unshuffle(s, C), t)
    y = rng.standard_normal(s.shape)
    assert abs(np.sum(s * y) - np.sum(t * U.unshuffle(y, C))) <= 1e-12


# ---------------------------------------------------------------- whole network
def _tiny_unet(rng, cin=2, ch=(2, 3, 4, 5), cout=2):
    c0, c1, c2, c3 = ch
    spec = [(cin, c0, 3, True), (c0, c0, 3, True), (c0, c1, 3, True), (c1, c1, 3, True),
            (c1, c2, 3, True), (c2, c2, 3, True), (c2, c3, 3, True), (c3, c3, 3, True),
            (c3, 4 * c2, 1, False), (c2, 4 * c1, 1, False), (c1, 4 * c0, 1, False),
            (2 * c2, c2, 3, True), (c2, c2, 3, True), (2 * c1, c1, 3, True), (c1, c1, 3, True),
            (2 * c0, c0, 3, True), (c0, c0, 3, True), (c0, cout, 1, False)]
    layers = []
    for ci, co, k, relu in spec:
        cop = ((co + 15) // 16) * 16
        w = np.zeros((k * k, cop, ci))
        w[:, :co] = rng.standard_normal((k * k, co, ci)) * np.sqrt(2.0 / (ci * k * k))
        b = np.zeros(cop)
        b[:co] = 0.1 * rng.standard_normal(co)
        layers.append((w, b, ci, co, k, relu))
    return layers


def test_unet_backward_matches_central_differences(monkeypatch):
    """FP64 central differences of L = <unet_forward(x), dy> along a random
    direction of each layer's weights and of its bias, against the same
    directional derivative from unet_backward.  Rounding to bfloat16 is off, so
    both sides are the exact network; a gradient routed to the wrong sub-pixel,
    a skip added to the wrong level or a missing ReLU mask fails a layer."""
    monkeypatch.setattr(U, "bf16", lambda a: np.asarray(a, dtype=np.float64))
    rng = _rng(7)
    ch = (2, 3, 4, 5)
    layers = _tiny_unet(rng, ch=ch)
    x = rng.standard_normal((2, 8, 16, 2))
    y, tape = U.unet_forward(layers, x, ch)
    dy = rng.standard_normal(y.shape)
    grads = U.unet_backward(layers, tape, dy, ch)
    eps = 1e-6

    def loss(ls):
        return float(np.sum(U.unet_forward(ls, x, ch)[0] * dy))

    for i, (w, b, ci, co, k, relu) in enumerate(layers):
        dw, db = grads[i]
        for which in ("w", "b"):
            d = np.zeros_like(w if which == "w" else b)
            if which == "w":
                d[:, :co] = rng.standard_normal((k * k, co, ci))
            else:
                d[:co] = rng.standard_normal(co)
            plus, minus = list(layers), list(layers)
            if which == "w":
                plus[i] = (w + eps * d, b, ci, co, k, relu)
                minus[i] = (w - eps * d, b, ci, co, k, relu)
                an = float(np.sum(dw * d))
            else:
                plus[i] = (w, b + eps * d, ci, co, k, relu)
                minus[i] = (w, b - eps * d, ci, co, k, relu)
                an = float(np.sum(db * d))
            fd = (loss(plus) - loss(minus)) / (2 * eps)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, which, fd, an)


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0, 3e38])
    out = U.bf16(vals)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    assert out[0] == 1.0 and out[1] == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert out[2] == 1.0 + 2 ** -6
    assert out[3] == 1.0 and out[4] == -2.5 and out[5] == 0.0
    mant = (out.astype(np.float32).view(np.uint32) & 0xFFFF)
    assert np.all(mant == 0)


# ---------------------------------------------------------------- Adam
def test_adam_constant_gradient_closed_form():
    """With the bias corrections 1 - b1^t and 1 - b2^t, a constant gradient g
    gives m_hat = g and v_hat = g^2 at every step t, so each step moves the
    weight by exactly lr * g / (|g| + eps)."""
    rng = _rng(8)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        w, m, v = U.adam(w, m, v, g, lr, b1, b2, eps, t)
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=0, atol=1e-14)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=0, atol=1e-14)


def test_adam_weight_decay_enters_the_gradient():
    w = np.array([2.0, -1.0])
    g = np.array([0.0, 0.0])
    wd, lr = 0.5, 1e-3
    w1, _, _ = U.adam(w, np.zeros(2), np.zeros(2), g, lr, 0.9, 0.999, 0.0, 1, wd=wd)
    # the effective gradient is wd * w, so the first step is lr * sign(w)
    assert np.allclose(w1, w - lr * np.sign(w), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- unrolled ADM
def test_unrolled_oracle_reproduces_adm_with_its_logged_steps():
    """K unrolled steps with (mu, rho, xi) fixed and alpha_k the step or_adm
    logged at iteration k give or_adm's iterate f^K = beta x^K: the unrolled
    oracle assembles Eq. 10 from the projector and difference primitives, or_adm
    is the C loop, so a step out of order or a wrong multiplier sign fails."""
    from oracle import oracle as O
    from paper_1607_01650_amd import configs as C
    from paper_1607_01650_amd import phantom as P
    from oracle import unrolled as OU

    g = C.Geometry(nx=24, ny=20, pixel_mm=1.0, n_views=18, n_bins=40, bin_mm=1.2, sod_mm=100.0,
                   sdd_mm=200.0)
    s = P.make_slice(g, 3, n_inserts=2, r_obj=8.0)
    beta, mu, rho, xi = 0.79, 1.0, 16.0, 4.0
    m = np.asarray(s.sino[1], dtype=np.float64)
    for K in (1, 2, 7):
        ref = O.adm(g, m, beta, mu, rho, xi, K)
        params = [(mu, rho, xi, float(ref.log[k, 1])) for k in range(K)]
        f = OU.unrolled(g, beta * m, params)
        err = np.linalg.norm(f - beta * ref.x) / np.linalg.norm(beta * ref.x)
        assert err <= 1e-12, (K, err)
