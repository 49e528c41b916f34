"""Learned warm start for ADM-TV: data generation, U-Net training, evaluation.

Data: seeded dual-energy water/bone ellipse phantoms (the same recipe as the
phantom module) rasterised on the device, projected with the Joseph
projector and given 0.5 % Gaussian noise; plain ADM-TV provides the input
(5 iterations) and the target (200 iterations) of each training pair.

Evaluation (time to tolerance): J_ref = J(plain f^200) per phantom, the
objective of Eq. 4 summed over both energies.  Plain time = time of the first
k iterations with J(f^k) <= J_ref.  Learned time = 5 iterations + U-Net
inference + ADM-TV started from the network output until J <= J_ref.  Plain
ADM stays the judge of the network's error: the continuation runs the
unchanged method.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import configs as C
from . import dect
from . import nn as NN
from . import phantom as P

EARLY = 5
LATE = 200


def rasterize_device(ellipses, geom: C.Geometry, supersample: int = 4, device="cuda"):
    """[2, ny, nx] attenuation images (high, low) by supersampled coverage."""
    s = supersample
    off = (torch.arange(s, device=device, dtype=torch.float64) + 0.5) / s - 0.5
    xs = ((torch.arange(geom.nx, device=device, dtype=torch.float64) - (geom.nx - 1) / 2)[:, None]
          + off[None, :]).reshape(-1) * geom.pixel_mm
    ys = ((torch.arange(geom.ny, device=device, dtype=torch.float64) - (geom.ny - 1) / 2)[:, None]
          + off[None, :]).reshape(-1) * geom.pixel_mm
    Y, X = torch.meshgrid(ys, xs, indexing="ij")
    img = torch.zeros((2,) + X.shape, device=device, dtype=torch.float64)
    for el in ellipses:
        cp, sp = math.cos(el.phi), math.sin(el.phi)
        dx, dy = X - el.cx, Y - el.cy
        inside = ((cp * dx + sp * dy) / el.a) ** 2 + ((-sp * dx + cp * dy) / el.b) ** 2 <= 1.0
        img[0] += el.mu_high * inside
        img[1] += el.mu_low * inside
    img = img.reshape(2, geom.ny, s, geom.nx, s).mean(dim=(2, 4))
    return img.float()


def make_case(geom: C.Geometry, seed: int, noise_frac: float = 0.005):
    """Phantom images [2,ny,nx] and noisy sinograms [2,V,B] on the device."""
    els = P.make_phantom(seed, C.object_radius_mm(geom))
    x = rasterize_device(els, geom)
    clean = dect.project(x, geom)
    gen = torch.Generator(device="cuda").manual_seed(10000 + 2 * seed)
    sino = torch.empty_like(clean)
    for e in (0, 1):
        sig = noise_frac * float(clean[e].max())
        sino[e] = clean[e] + sig * torch.randn(clean[e].shape, generator=gen, device="cuda")
    return x, sino


@dataclasses.dataclass
class Pair:
    early: torch.Tensor   # [2, ny, nx] f^5 / beta (attenuation units)
    late: torch.Tensor    # [2, ny, nx] f^200 / beta
    J_late: float         # J(f^200) summed over energies


def make_pairs(geom: C.Geometry, seeds, params: Optional[C.AdmParams] = None,
               log_every: int = 0) -> List[Pair]:
    p = params or C.default_adm_params(geom, LATE)
    out = []
    t0 = time.time()
    for i, sd in enumerate(seeds):
        _, sino = make_case(geom, sd)
        st = dect.AdmState(geom)
        r5 = dect.adm_tv(sino[0], sino[1], geom, dataclasses.replace(p, max_iter=EARLY), state=st)
        early = torch.stack([r5.x_high.clone(), r5.x_low.clone()])
        r = dect.adm_tv(sino[0], sino[1], geom, dataclasses.replace(p, max_iter=LATE - EARLY),
                        state=st, want_log=True)
        late = torch.stack([r.x_high.clone(), r.x_low.clone()])
        st.close()
        out.append(Pair(early, late, float(r.report.objective)))
        if log_every and (i + 1) % log_every == 0:
            print(f"  pairs {i + 1}/{len(seeds)}  {time.time() - t0:.1f}s", flush=True)
    return out


def _batch(pairs: List[Pair], idx) -> Tuple[torch.Tensor, torch.Tensor]:
    e = torch.stack([pairs[i].early for i in idx])   # [B, 2, ny, nx]
    l = torch.stack([pairs[i].late for i in idx])
    x = NN.pack_input(e[:, 0], e[:, 1])
    tgt = (l.permute(0, 2, 3, 1) * NN.SCALE).contiguous()  # [B, ny, nx, 2]
    return x, tgt


def train(net: NN.UNet, pairs: List[Pair], epochs: int = 10, batch: int = 8,
          lr: float = 1e-3, seed: int = 0, log: bool = True) -> List[float]:
    rng = np.random.default_rng(seed)
    losses = []
    n = len(pairs)
    for ep in range(epochs):
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / max(1, epochs)))
        for b0 in range(0, n - batch + 1, batch):
            x, tgt = _batch(pairs, order[b0:b0 + batch])
            r = net.forward(x, keep=True)
            y = (NN.to_f32(x) + r).contiguous()
            dy = torch.empty_like(y)
            parts = NN.mse(y, tgt, dy)
            net.backward(dy)
            net.adam_step(lr_ep)
            tot += float(parts.sum()) / (tgt.numel())
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            print(f"  epoch {ep}: mse {losses[-1]:.4e}", flush=True)
    return losses


def _time_adm(sino, geom, p, iters, x0=None) -> Tuple[float, dect.AdmResult]:
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dect.adm_tv(sino[0], sino[1], geom, dataclasses.replace(p, max_iter=iters), x0=x0,
                    want_log=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def first_reach(J: np.ndarray, target: float) -> int:
    hit = np.nonzero(J <= target * (1 + 1e-12))[0]
    return int(hit[0]) if hit.size else -1


def evaluate(net: NN.UNet, geom: C.Geometry, seeds, max_cont: int = 400) -> Dict:
    """Time to J_ref = J(plain f^200), plain vs learned warm start."""
    p = C.default_adm_params(geom, LATE)
    rows = []
    for sd in seeds:
        _, sino = make_case(geom, sd)
        # plain: the full 200 iterations give J_ref and the iteration count
        _, rp = _time_adm(sino, geom, p, LATE)
        Jp = rp.J.sum(axis=1)
        J_ref = Jp[LATE]
        k_plain = first_reach(Jp, J_ref)
        t_plain, _ = _time_adm(sino, geom, p, k_plain)
        # learned: 5 iterations + network + continuation
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r5 = dect.adm_tv(sino[0], sino[1], geom, dataclasses.replace(p, max_iter=EARLY))
        yh, yl = NN.predict(net, r5.x_high[None], r5.x_low[None])
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t0
        _, rc = _time_adm(sino, geom, p, max_cont, x0=(yh[0], yl[0]))
        Jc = rc.J.sum(axis=1)
        k_cont = first_reach(Jc, J_ref)
        if k_cont < 0:  # the network did not help: fall back to the plain count
            rows.append(dict(seed=sd, J_ref=J_ref, k_plain=k_plain, k_cont=-1, t_plain=t_plain,
                             t_learned=float("nan"), J_net=float(Jc[0])))
            continue
        t_cont, rfin = _time_adm(sino, geom, p, k_cont, x0=(yh[0], yl[0]))
        rows.append(dict(seed=sd, J_ref=J_ref, k_plain=k_plain, k_cont=k_cont, t_plain=t_plain,
                         t_learned=t_net + t_cont, J_net=float(Jc[0])))
    ratios = [r["t_learned"] / r["t_plain"] for r in rows if r["k_cont"] >= 0]
    return {"rows": rows,
            "median_time_ratio": float(np.median(ratios)) if ratios else float("nan"),
            "reached": len(ratios), "n": len(rows),
            "median_k_plain": float(np.median([r["k_plain"] for r in rows])),
            "median_k_cont": float(np.median([r["k_cont"] for r in rows if r["k_cont"] >= 0]))
            if ratios else float("nan")}
