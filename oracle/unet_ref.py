"""FP64 NumPy oracle of the U-Net operations (TEST INFRASTRUCTURE ONLY).

Direct definitions: 'same'-padded cross-correlation over NHWC tensors with
weights [taps][Cout(P)][Cin] (taps in row-major (dy, dx) order), its input
and weight gradients, 2x2 max pooling (first maximum wins), depth-to-space,
channel concat, MSE and Adam.  unet_forward/unet_backward mirror the network
layer by layer and round to bfloat16 (nearest even) where the GPU path stores
bfloat16, so the two differ only by the order of FP32 accumulation.
"""
import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad(x, k):
    p = k // 2
    return np.pad(x, ((0, 0), (p, p), (p, p), (0, 0))) if p else x


def conv(x, w, b, cout, k):
    """y[n,h,w,co] = b[co] + sum_{dy,dx,ci} x[n,h+dy-k//2,w+dx-k//2,ci] w[tap,co,ci]."""
    N, H, W, Ci = x.shape
    xp = _pad(x, k)
    y = np.zeros((N, H, W, cout))
    for t in range(k * k):
        dy, dx = t // k, t % k
        y += np.einsum("nhwc,oc->nhwo", xp[:, dy:dy + H, dx:dx + W, :], w[t, :cout, :])
    if b is not None:
        y += b[:cout]
    return y


def conv_dx(dz, w, cin, k):
    """Input gradient of conv: dx = sum_tap shift^T(dz) w[tap]."""
    N, H, W, Co = dz.shape
    p = k // 2
    dxp = np.zeros((N, H + 2 * p, W + 2 * p, cin))
    for t in range(k * k):
        dy, dx = t // k, t % k
        dxp[:, dy:dy + H, dx:dx + W, :] += np.einsum("nhwo,oc->nhwc", dz, w[t, :Co, :cin])
    return dxp[:, p:p + H, p:p + W, :] if p else dxp


def conv_dw(dz, x, k, coutp):
    N, H, W, Co = dz.shape
    Ci = x.shape[-1]
    xp = _pad(x, k)
    dw = np.zeros((k * k, coutp, Ci))
    for t in range(k * k):
        dy, dx = t // k, t % k
        dw[t, :Co] = np.einsum("nhwo,nhwc->oc", dz, xp[:, dy:dy + H, dx:dx + W, :])
    db = np.zeros(coutp)
    db[:Co] = dz.sum(axis=(0, 1, 2))
    return dw, db


def pool(x):
    N, H, W, C = x.shape
    v = x.reshape(N, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(N, H // 2, W // 2, 4, C)
    idx = np.argmax(v, axis=3)  # first maximum
    return np.take_along_axis(v, idx[:, :, :, None, :], axis=3)[:, :, :, 0, :], idx


def pool_dx(dy, idx):
    N, Ho, Wo, C = dy.shape
    d = np.zeros((N, Ho, Wo, 4, C))
    np.put_along_axis(d, idx[:, :, :, None, :], dy[:, :, :, None, :], axis=3)
    return d.reshape(N, Ho, Wo, 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(N, 2 * Ho, 2 * Wo, C)


def shuffle(t, c):
    N, H, W, _ = t.shape
    return t.reshape(N, H, W, 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(N, 2 * H, 2 * W, c)


def unshuffle(y, c):
    N, H2, W2, _ = y.shape
    return y.reshape(N, H2 // 2, 2, W2 // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(
        N, H2 // 2, W2 // 2, 4 * c)


def adam(w, m, v, g, lr, b1, b2, eps, step, wd=0.0):
    g = g + wd * w
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def unet_forward(layers, x, ch):
    """layers: list of (w, b, cin, cout, k, relu) in UNet.layers() order."""
    enc = [layers[0:2], layers[2:4], layers[4:6], layers[6:8]]
    up = layers[8:11]
    dec = [layers[11:13], layers[13:15], layers[15:17]]
    out = layers[17]
    t = {"x": x}

    def run(L, h, keep_f32=False):
        w, b, cin, cout, k, relu = L
        y = conv(h, w, b, cout, k)
        if relu:
            y = np.maximum(y, 0.0)
        return y if keep_f32 else bf16(y)

    h = x
    skips = []
    for lvl in range(4):
        a = run(enc[lvl][0], h)
        bb = run(enc[lvl][1], a)
        t[f"e{lvl}a"], t[f"e{lvl}b"] = a, bb
        if lvl < 3:
            skips.append(bb)
            h, idx = pool(bb)
            t[f"p{lvl}"], t[f"i{lvl}"] = h, idx
        else:
            h = bb
    for j, lvl in enumerate((2, 1, 0)):
        c = ch[lvl]
        u = shuffle(run(up[j], h), c)
        z = np.concatenate([u, skips[lvl]], axis=-1)
        a = run(dec[j][0], z)
        bb = run(dec[j][1], a)
        t[f"uin{j}"], t[f"z{j}"], t[f"d{j}a"], t[f"d{j}b"] = h, z, a, bb
        h = bb
    t["dout_in"] = h
    return run(out, h, keep_f32=True), t


def unet_backward(layers, t, dy, ch):
    """Gradients (dw, db) per layer for the output gradient dy (FP64)."""
    grads = [None] * len(layers)

    def back(i, d, xin, yout):
        w, b, cin, cout, k, relu = layers[i]
        dz = d * (yout > 0) if relu else d
        grads[i] = conv_dw(dz, xin, k, w.shape[1])
        return bf16(conv_dx(dz, w, cin, k))

    dh = back(17, bf16(dy), t["dout_in"], None)
    dskip = [None] * 3
    for j in (2, 1, 0):
        lvl = (2, 1, 0)[j]
        c = ch[lvl]
        da = back(12 + 2 * j, dh, t[f"d{j}a"], t[f"d{j}b"])
        dz = back(11 + 2 * j, da, t[f"z{j}"], t[f"d{j}a"])
        du, dskip[lvl] = dz[..., :c], dz[..., c:]
        dh = back(8 + j, unshuffle(du, c), t[f"uin{j}"], None)
    for lvl in (3, 2, 1, 0):
        if lvl < 3:
            dh = bf16(pool_dx(dh, t[f"i{lvl}"]) + dskip[lvl])
        inp = t["x"] if lvl == 0 else t[f"p{lvl - 1}"]
        da = back(2 * lvl + 1, dh, t[f"e{lvl}a"], t[f"e{lvl}b"])
        dh = back(2 * lvl, da, inp, t[f"e{lvl}a"])
    return grads
