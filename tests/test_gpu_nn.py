"""BF16 MFMA network kernels vs the FP64 oracle on bfloat16-rounded inputs.

Tolerances follow from the arithmetic: inputs and weights are exact bfloat16
values, so FP32 accumulation leaves ~1e-6 relative error (FP32 outputs); a
bfloat16 output may differ from the rounded oracle by one unit in the last
place.  The whole U-Net (forward and every weight gradient) is compared with
an oracle that rounds to bfloat16 at the same points.
"""
import numpy as np
import pytest

from oracle import unet_ref as R

from helpers import need_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _nn():
    from paper_1607_01650_amd import nn
    return nn


def _bf(torch, a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda().to(torch.bfloat16)


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


CASES = [  # N, H, W, Cin, Cout, k
    (2, 8, 72, 8, 32, 3), (1, 16, 64, 32, 48, 3), (1, 4, 130, 96, 64, 3),
    (2, 8, 64, 128, 64, 3), (1, 8, 64, 96, 256, 1), (2, 3, 256, 8, 32, 3),
    (1, 5, 128, 64, 32, 3), (1, 6, 40, 32, 8, 1), (1, 4, 64, 16, 200, 3)]
# the weight gradient on ragged strips and rows, 1x1 and 3x3, one to thirteen
# tile splits, and (last) several four-row steps per block
GRAD_CASES = CASES + [(4, 256, 256, 32, 32, 3)]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_conv_fwd(torch, case):
    nn = _nn()
    N, H, W, Ci, Co, k = case
    rng = np.random.default_rng(hash(case) % 2**32)
    x = R.bf16(rng.standard_normal((N, H, W, Ci)))
    CoP = (Co + 15) // 16 * 16
    w = np.zeros((k * k, CoP, Ci))
    w[:, :Co] = R.bf16(rng.standard_normal((k * k, Co, Ci)) * 0.1)
    b = rng.standard_normal(CoP).astype(np.float32).astype(np.float64)
    ref = R.conv(x, w, b, Co, k)
    xt, wt = _bf(torch, x), _bf(torch, w)
    bt = torch.as_tensor(b, dtype=torch.float32).cuda()
    y32 = _np(nn.conv_fwd(xt, wt, bt, Co, k, False, out_f32=True))
    assert rel_l2(y32, ref) <= 1e-5
    yr = _np(nn.conv_fwd(xt, wt, bt, Co, k, True))
    rr = R.bf16(np.maximum(ref, 0))
    # one bfloat16 ulp, plus the FP32 sum's own error (its order is the
    # kernel's), which can move a value within it of zero across the ReLU
    e = 1e-5 * np.sqrt(np.mean(ref ** 2))
    bound = np.abs(rr) * 2.0 ** -7 + e
    bad = np.abs(yr - rr) - bound
    i = np.unravel_index(np.argmax(bad), bad.shape)
    assert bad[i] <= 0, (i, yr[i], rr[i], ref[i])


@pytest.mark.parametrize("case", GRAD_CASES, ids=[str(c) for c in GRAD_CASES])
def test_conv_input_and_weight_gradients(torch, case):
    nn = _nn()
    N, H, W, Ci, Co, k = case
    if Co % 8:
        pytest.skip("gradients need Cout % 8 == 0")
    rng = np.random.default_rng(7)
    x = R.bf16(rng.standard_normal((N, H, W, Ci)))
    dz = R.bf16(rng.standard_normal((N, H, W, Co)))
    CoP = (Co + 15) // 16 * 16
    w = np.zeros((k * k, CoP, Ci))
    w[:, :Co] = R.bf16(rng.standard_normal((k * k, Co, Ci)) * 0.1)
    wt, dzt, xt = _bf(torch, w), _bf(torch, dz), _bf(torch, x)
    wd = nn.weight_flip(wt, Ci, Co, k)
    dx = _np(nn.conv_fwd(dzt, wd, None, Ci, k, False, out_f32=True))
    assert rel_l2(dx, R.conv_dx(dz, w, Ci, k)) <= 1e-5
    gw = torch.zeros((k * k, CoP, Ci), device="cuda")
    gb = torch.zeros((CoP,), device="cuda")
    nn.conv_wgrad(dzt, xt, Co, k, gw, gb)
    rw, rb = R.conv_dw(dz, x, k, CoP)
    assert rel_l2(_np(gw), rw) <= 1e-5
    assert rel_l2(_np(gb), rb) <= 1e-5


def test_pool_shuffle_concat_exact(torch):
    nn = _nn()
    rng = np.random.default_rng(3)
    x = R.bf16(rng.standard_normal((2, 8, 12, 16)))
    y, idx = nn.pool_fwd(_bf(torch, x))
    ry, ridx = R.pool(x)
    assert np.array_equal(_np(y), ry) and np.array_equal(idx.cpu().numpy(), ridx)
    dy = R.bf16(rng.standard_normal(ry.shape))
    assert np.array_equal(_np(nn.pool_bwd(_bf(torch, dy), idx)), R.pool_dx(dy, ridx))
    t = R.bf16(rng.standard_normal((2, 4, 6, 4 * 24)))
    s = nn.shuffle(_bf(torch, t), 24)
    assert np.array_equal(_np(s), R.shuffle(t, 24))
    assert np.array_equal(_np(nn.unshuffle(s, 24)), t)
    a, b = R.bf16(rng.standard_normal((2, 4, 6, 16))), R.bf16(rng.standard_normal((2, 4, 6, 24)))
    z = nn.concat(_bf(torch, a), _bf(torch, b))
    assert np.array_equal(_np(z), np.concatenate([a, b], -1))
    a2, b2 = nn.split(z, 16)
    assert np.array_equal(_np(a2), a) and np.array_equal(_np(b2), b)
    assert np.array_equal(_np(nn.add(_bf(torch, a), _bf(torch, a))), R.bf16(2 * a))


@pytest.mark.parametrize("c1,c2", [(24, 16), (48, 48), (8, 32)])
def test_shuffle_concat_is_the_two_passes(torch, c1, c2):
    """dect_nn_shuffle_concat equals shuffle then concat, and its inverse split
    then unshuffle, bit for bit (odd image sizes, uneven channel splits)."""
    nn = _nn()
    rng = np.random.default_rng(5)
    t = _bf(torch, R.bf16(rng.standard_normal((2, 3, 5, 4 * c1))))
    s = _bf(torch, R.bf16(rng.standard_normal((2, 6, 10, c2))))
    z = nn.shuffle_concat(t, s, c1)
    ref = nn.concat(nn.shuffle(t, c1), s)
    assert np.array_equal(_np(z), _np(ref))
    t2, s2 = nn.split_unshuffle(z, c1)
    a, b = nn.split(ref, c1)
    assert np.array_equal(_np(t2), _np(nn.unshuffle(a, c1)))
    assert np.array_equal(_np(t2), _np(t)) and np.array_equal(_np(s2), _np(s))
    dect = __import__("paper_1607_01650_amd.dect", fromlist=["DectError"])
    with pytest.raises(dect.DectError):  # channels not a multiple of 8
        nn._ck(nn._lib().dect_nn_shuffle_concat(nn._p(t), nn._p(s), nn._p(z), 2, 3, 5, 12, c2,
                                                0, nn._s()), "shuffle_concat")


def test_adam_and_mse(torch):
    nn = _nn()
    rng = np.random.default_rng(4)
    n = 1000
    w = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = rng.standard_normal(n).astype(np.float32) * 0.1
    v = np.abs(rng.standard_normal(n)).astype(np.float32) * 0.1
    tw, tg, tm, tv = (torch.as_tensor(a).cuda() for a in (w, g, m, v))
    L = nn._lib()
    import ctypes as ct
    L.dect_nn_adam(nn._p(tw), nn._p(tm), nn._p(tv), nn._p(tg), None, n, 1e-3, 0.9, 0.999, 1e-8, 3,
                   0.0, nn._s())
    rw, _, _ = R.adam(w.astype(np.float64), m, v, g, 1e-3, 0.9, 0.999, 1e-8, 3)
    assert np.abs(tw.cpu().numpy() - rw).max() <= 1e-6
    y = rng.standard_normal((5, 7, 8)).astype(np.float32)
    tgt = rng.standard_normal((5, 7, 2)).astype(np.float32)
    dy = torch.empty((5, 7, 8), device="cuda")
    parts = nn.mse(torch.as_tensor(y).cuda(), torch.as_tensor(tgt).cuda(), dy)
    ref = np.mean((y[..., :2].astype(np.float64) - tgt) ** 2)
    # the kernel forms y - t in FP32 (one rounding) and sums squares in FP64
    assert abs(float(parts.sum()) / (35 * 2) - ref) <= 1e-6 * ref
    rdy = np.zeros_like(y, dtype=np.float64)
    rdy[..., :2] = 2 * (y[..., :2] - tgt) / (35 * 2)
    assert np.abs(dy.cpu().numpy() - rdy).max() <= 1e-7


def _layers_np(net):
    out = []
    for c in net.layers():
        out.append((R.bf16(c.w.cpu().numpy()), c.b.cpu().numpy().astype(np.float64), c.cin,
                    c.cout, c.k, c.relu))
    return out


@pytest.mark.parametrize("N,H,W", [(2, 32, 64), (1, 256, 256)], ids=["2x32x64", "1x256x256"])
def test_unet_forward_and_gradients_vs_oracle(torch, N, H, W):
    """The production network (channels 32/48/64/96): small images, and
    256 x 256, where every kernel runs its full-size path (several row and
    column tiles, weight-gradient blocks of several steps, many partial
    chunks); the FP64 oracle takes about 15 s there."""
    nn = _nn()
    net = nn.UNet(seed=1)
    for c in net.layers():  # non-zero biases exercise the bias paths
        c.b.copy_(torch.randn(c.b.shape) * 0.05 * (torch.arange(c.coutp) < c.cout).float())
    assert 480_000 < net.n_params() < 520_000
    rng = np.random.default_rng(5)
    x = np.zeros((N, H, W, 8))
    x[..., :2] = R.bf16(rng.uniform(0, 1.5, (N, H, W, 2)))
    xt = _bf(torch, x)
    y = net.forward(xt, keep=True)
    L = _layers_np(net)
    ry, tape = R.unet_forward(L, x, net.ch)
    err = rel_l2(_np(y), ry)
    print(f"U-Net forward rel-L2 vs oracle {err:.2e}", flush=True)
    assert err <= 1e-2
    dy = np.zeros((N, H, W, 8))
    dy[..., :2] = rng.standard_normal((N, H, W, 2)) * 1e-3
    # the backward pass is checked on the GPU's own forward activations: the
    # ReLU masks and pooling choices are then identical on both sides, and the
    # two differ only by accumulation order (and the bf16 roundings it flips)
    gpu_tape = {k: (v.cpu().numpy() if k.startswith("i") else _np(v))
                for k, v in net._t.items()}
    net.backward(torch.as_tensor(dy, dtype=torch.float32).cuda())
    rg = R.unet_backward(L, gpu_tape, dy, net.ch)
    worst = 0.0
    for i, c in enumerate(net.layers()):
        ew = rel_l2(_np(c.gw), rg[i][0])
        eb = rel_l2(_np(c.gb), rg[i][1])
        print(f"  layer {i}: dW rel-L2 {ew:.2e}  db rel-L2 {eb:.2e}", flush=True)
        worst = max(worst, ew, eb)
    print(f"U-Net worst layer gradient rel-L2 vs oracle {worst:.2e}", flush=True)
    assert worst <= 2e-2


def test_unet_learns(torch):
    """A few Adam steps on a fixed batch reduce the loss."""
    nn = _nn()
    net = nn.UNet(seed=2)
    rng = np.random.default_rng(6)
    xin = np.zeros((4, 64, 64, 8))
    xin[..., :2] = rng.uniform(0, 1, (4, 64, 64, 2))
    tgt = (xin[..., :2] * 0.8 + 0.1).astype(np.float32)
    xt = _bf(torch, xin)
    tt = torch.as_tensor(tgt).cuda()
    losses = []
    for it in range(40):
        r = net.forward(xt, keep=True)
        base = nn.to_f32(xt)
        y = (base[..., :] + r).contiguous()
        dy = torch.empty_like(y)
        parts = nn.mse(y, tt, dy)
        losses.append(float(parts.sum()))
        net.backward(dy)
        net.adam_step(2e-3)
    assert losses[-1] < 0.2 * losses[0], losses[::8]


def test_checkpoint_resumes_training_exactly(torch, tmp_path):
    """Weights saved with the Adam moments and step, loaded into a network of
    other initial weights: one more training step on both gives the same
    weights bit for bit (the checkpoint holds the whole training state)."""
    from paper_1607_01650_amd import nn as NN
    from paper_1607_01650_amd import warmstart as W
    ch = (8, 16, 16, 24)
    rng = np.random.default_rng(21)
    f = torch.as_tensor(rng.uniform(0, 0.05, (2, 2, 32, 64)), dtype=torch.float32).cuda()
    x, base = NN.pack_input(f[:, 0], f[:, 1])
    tgt = (f.permute(0, 2, 3, 1) * NN.SCALE).contiguous()

    def step(net):
        r = net.forward(x, keep=True)
        y = (base + r).contiguous()
        dy = torch.empty_like(y)
        NN.mse(y, tgt, dy)
        net.backward(dy)
        net.adam_step(1e-3)

    a = NN.UNet(seed=3, ch=ch)
    for _ in range(3):
        step(a)
    path = str(tmp_path / "ckpt.npz")
    W.save_weights(a, path)
    b = NN.UNet(seed=4, ch=ch)
    W.load_weights(b, path)
    assert b.step == a.step == 3
    step(a)
    step(b)
    for ca, cb in zip(a.layers(), b.layers()):
        assert torch.equal(ca.w, cb.w) and torch.equal(ca.b, cb.b)
        assert torch.equal(ca.mw, cb.mw) and torch.equal(ca.vw, cb.vw)


def test_fused_relu_backward_is_bitwise_the_unfused_path(torch):
    """dect_nn_conv_fwd_masked and dect_nn_add_relu_bwd equal the ReLU
    backward applied after the plain calls, bit for bit (bf16 and FP32
    outputs, a ragged width, and the element-wise fallback)."""
    nn = _nn()
    rng = np.random.default_rng(11)
    for (N, H, W, Ci, Co, k) in [(2, 8, 72, 32, 48, 3), (1, 5, 40, 16, 24, 1), (1, 4, 33, 8, 12, 3)]:
        dz = _bf(torch, rng.standard_normal((N, H, W, Ci)))
        w = _bf(torch, rng.standard_normal((k * k, (Co + 15) // 16 * 16, Ci)) * 0.1)
        mask = _bf(torch, rng.standard_normal((N, H, W, Co)))
        for f32 in (False, True):
            plain = nn.conv_fwd(dz, w, None, Co, k, False, out_f32=f32)
            fused = nn.conv_fwd(dz, w, None, Co, k, False, out_f32=f32, mask=mask)
            ref = torch.where(mask.float() > 0, plain, torch.zeros_like(plain))
            assert torch.equal(fused, ref)
    a, b, y = (_bf(torch, rng.standard_normal((3, 7, 9, 16))) for _ in range(3))
    assert torch.equal(nn.add_relu_bwd(a, b, y), nn.relu_bwd(nn.add(a, b), y))
    n = 1001  # not a multiple of 8: the element-wise kernel
    a, b, y = (_bf(torch, rng.standard_normal(n)) for _ in range(3))
    assert torch.equal(nn.add_relu_bwd(a, b, y), nn.relu_bwd(nn.add(a, b), y))
