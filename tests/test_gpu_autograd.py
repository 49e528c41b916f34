"""Differentiable projector and unrolled ADM on the GPU.

* autograd projector: backward is dect_backproject; checked by central
  differences (eps = 1e-3, random directions) and the adjoint identity;
* unrolled ADM forward vs the FP64 oracle of the same steps (rel-L2 <= 1e-4);
* gradients w.r.t. the learnable step parameters vs central differences of
  the FP64 oracle;
* checkpointing every 2 steps gives the same gradients as no checkpointing.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import unrolled as OU
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

SMALL = C.Geometry(nx=64, ny=64, pixel_mm=1.0, n_views=30, n_bins=96, bin_mm=1.2, sod_mm=250.0,
                   sdd_mm=500.0)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def test_projector_finite_differences(torch):
    from paper_1607_01650_amd import autograd as AG
    g = C.paper_geometry(512, 180)
    rng = np.random.default_rng(0)
    x = to_dev(torch, rng.uniform(0, 0.05, (2, g.ny, g.nx))).requires_grad_(True)
    y = to_dev(torch, rng.standard_normal((2, g.n_views, g.n_bins)))

    def loss(t):
        r = AG.project(t, g) - y
        return 0.5 * (r.double() ** 2).sum()

    L = loss(x)
    (gx,) = torch.autograd.grad(L, x)
    eps = 1e-3
    for k in range(3):
        d = torch.randn_like(x)  # unit RMS per element: eps * d is 1e-3 per pixel
        with torch.no_grad():
            fd = (loss(x + eps * d) - loss(x - eps * d)) / (2 * eps)
        an = (gx.double() * d.double()).sum()
        assert abs(float(fd - an)) <= 1e-3 * abs(float(an)) + 1e-6


def test_autograd_adjoint_identity(torch):
    from paper_1607_01650_amd import autograd as AG
    g = SMALL
    x = to_dev(torch, P.random_image(g, 1)).requires_grad_(True)
    y = to_dev(torch, P.random_sino(g, 2))
    (aty,) = torch.autograd.grad((AG.project(x, g) * y).sum(), x)
    ref = O.backproject(g, f32(P.random_sino(g, 2)))
    assert rel_l2(to_np(aty), ref) <= 1e-5
    yy = to_dev(torch, P.random_sino(g, 2)).requires_grad_(True)
    (ax,) = torch.autograd.grad((AG.backproject(yy, g) * x.detach()).sum(), yy)
    assert rel_l2(to_np(ax), O.project(g, f32(P.random_image(g, 1)))) <= 1e-5


def _setup(torch, n_steps=10):
    from paper_1607_01650_amd.unrolled import UnrolledADM
    g = SMALL
    s = P.make_slice(g, 3, n_inserts=4, r_obj=25.0)
    gdata = f32(s.sino[1])
    model = UnrolledADM(g, n_steps=n_steps, mu=1.0, rho=1024.0, xi=256.0,
                        alphas=[2e-4 * (1 + 0.1 * k) for k in range(n_steps)]).cuda()
    return g, s, gdata, model


def _params(model):
    out = []
    with torch_no_grad():
        for k in range(model.n_steps):
            out.append(tuple(float(v) for v in model.params_of(k)))
    return out


def torch_no_grad():
    import torch
    return torch.no_grad()


def test_unrolled_forward_parity(torch):
    g, s, gdata, model = _setup(torch)
    with torch.no_grad():
        f = model(to_dev(torch, gdata)[None])[0]
    ref = OU.unrolled(g, gdata, _params(model))
    err = rel_l2(to_np(f), ref)
    print(f"unrolled forward rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_unrolled_parameter_gradients_vs_oracle(torch):
    g, s, gdata, model = _setup(torch, n_steps=6)
    target = s.x_true[1]
    f = model(to_dev(torch, gdata)[None])[0]
    loss = 0.5 * ((f.double() - to_dev(torch, target).double()) ** 2).sum()
    loss.backward()
    grads = {n: p.grad.detach().cpu().numpy() for n, p in model.named_parameters()}
    base = _params(model)

    def oracle_loss(pp):
        fr = OU.unrolled(g, gdata, pp)
        return 0.5 * np.sum((fr - target) ** 2)

    h = 1e-5
    names = ["log_mu", "log_rho", "log_xi", "log_alpha"]
    checked = 0
    for k in (0, 2, 5):
        for j, name in enumerate(names):
            up = [list(t) for t in base]
            dn = [list(t) for t in base]
            up[k][j] *= np.exp(h)
            dn[k][j] *= np.exp(-h)
            fd = (oracle_loss(up) - oracle_loss(dn)) / (2 * h)
            an = grads[name][k]
            scale = max(abs(fd), 1e-3 * max(abs(grads['log_alpha']).max(), 1e-12))
            assert abs(an - fd) <= 3e-3 * scale + 1e-9, (name, k, an, fd)
            checked += 1
    assert checked == 12


def test_checkpointing_matches_plain_backward(torch):
    g, s, gdata, model = _setup(torch)
    gd = to_dev(torch, gdata)[None]
    out = []
    for use_ckpt in (True, False):
        model.zero_grad()
        f = model(gd, use_checkpoint=use_ckpt)
        (f.double() ** 2).sum().backward()
        out.append(np.concatenate([p.grad.cpu().numpy() for p in model.parameters()]))
    assert np.array_equal(out[0], out[1])
