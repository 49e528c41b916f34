"""Differentiable projector and unrolled ADM on the GPU.

* autograd projector: backward is dect_backproject; checked by central
  differences (eps = 1e-3, random directions) and the adjoint identity;
* unrolled ADM forward vs the FP64 oracle of the same steps (rel-L2 <= 1e-4);
* gradients w.r.t. the learnable step parameters vs central differences of
  the FP64 oracle;
* checkpointing every 2 steps gives the same gradients as no checkpointing;
* one step (dect_unrolled_step) from a nonzero (f, lambda) vs the oracle
  step, and its vector-Jacobian product (dect_unrolled_step_backward and the
  projector pair) vs central differences of the oracle step along random
  directions and along each parameter.
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


def _step_inputs(g, seed):
    """f: a phantom image; lambda: random multipliers of the size rho times
    the image's gradients, so that the shrinkage is active at some pixels
    and not at others; g: the phantom's data plus noise.  All FP32."""
    s = P.make_slice(g, seed, n_inserts=4, r_obj=25.0)
    rng = np.random.default_rng(50 + seed)
    f = f32(s.x_true[1] * (1.0 + 0.05 * rng.standard_normal(s.x_true[1].shape)))
    lx = f32(0.02 * rng.standard_normal(f.shape))
    ly = f32(0.02 * rng.standard_normal(f.shape))
    return f, lx, ly, f32(s.sino[1])


def test_unrolled_step_forward_parity(torch):
    """One step from a nonzero (f, lambda): f' and lambda' vs the FP64
    oracle step on the same FP32 inputs."""
    from paper_1607_01650_amd import unrolled as U
    g = SMALL
    f, lx, ly, gd = _step_inputs(g, 5)
    prm = (0.8, 512.0, 128.0, 3e-4)
    t = [to_dev(torch, a)[None] for a in (f, lx, ly, gd)]
    p = [torch.tensor(v, dtype=torch.float32, device="cuda") for v in prm]
    with torch.no_grad():
        fo, lxo, lyo = U.adm_step(t[0], t[1], t[2], t[3], g, *p)
    ref = OU.step(g, gd, f, lx, ly, *[float(np.float32(v)) for v in prm])
    errs = [rel_l2(to_np(a[0]), b) for a, b in zip((fo, lxo, lyo), ref)]
    print(f"unrolled step: f' {errs[0]:.2e}, lambda_x' {errs[1]:.2e}, lambda_y' {errs[2]:.2e}",
          flush=True)
    assert max(errs) <= 1e-5


def test_unrolled_step_vjp_vs_oracle_differences(torch):
    """dect_unrolled_step_backward (with the projector pair's autograd):
    <grad L, d> for L = <c, (f', lambda')> with random cotangents c, along
    random directions d in (f, lambda_x, lambda_y) and along each of the
    four parameters, against central differences of the FP64 oracle step."""
    from paper_1607_01650_amd import unrolled as U
    g = SMALL
    f, lx, ly, gd = _step_inputs(g, 6)
    prm = np.array([0.8, 512.0, 128.0, 3e-4], dtype=np.float32).astype(np.float64)
    rng = np.random.default_rng(7)
    cot = [rng.standard_normal(f.shape) for _ in range(3)]
    t = [to_dev(torch, a)[None].requires_grad_(True) for a in (f, lx, ly)]
    p = [torch.tensor(v, dtype=torch.float32, device="cuda", requires_grad=True) for v in prm]
    out = U.adm_step(t[0], t[1], t[2], to_dev(torch, gd)[None], g, *p)
    L = sum((o[0].double() * to_dev(torch, c).double()).sum() for o, c in zip(out, cot))
    grads = torch.autograd.grad(L, t + p)
    gx = [to_np(q[0]) for q in grads[:3]]
    gp = [float(q) for q in grads[3:]]

    def oracle_L(ff, xx, yy, pp):
        return sum(np.sum(a * c) for a, c in zip(OU.step(g, gd, ff, xx, yy, *pp), cot))

    base = [f, lx, ly]
    for k in range(3):
        d = [rng.standard_normal(f.shape) for _ in range(3)]
        # small enough that no pixel's shrinkage crosses its kink |v| = 1/rho
        # (the oracle's quotient is then stable to ~1e-8 as eps varies 10x)
        eps = 1e-7 * max(np.abs(a).max() for a in base)
        up = [b + eps * e for b, e in zip(base, d)]
        dn = [b - eps * e for b, e in zip(base, d)]
        fd = (oracle_L(*up, prm) - oracle_L(*dn, prm)) / (2 * eps)
        an = sum(np.sum(a * e) for a, e in zip(gx, d))
        print(f"step VJP direction {k}: analytic {an:.6e}, oracle differences {fd:.6e}",
              flush=True)
        assert abs(an - fd) <= 2e-4 * abs(fd), (k, an, fd)
    for j, name in enumerate(("mu", "rho", "xi", "alpha")):
        h = 1e-6
        up, dn = prm.copy(), prm.copy()
        up[j] *= 1 + h
        dn[j] *= 1 - h
        fd = (oracle_L(f, lx, ly, up) - oracle_L(f, lx, ly, dn)) / (2 * h * prm[j])
        print(f"step VJP {name}: analytic {gp[j]:.6e}, oracle differences {fd:.6e}", flush=True)
        assert abs(gp[j] - fd) <= 1e-3 * abs(fd), (name, gp[j], fd)
