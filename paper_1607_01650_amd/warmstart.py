"""Learned warm start for ADM-TV: data generation, U-Net training, evaluation.

Data: seeded dual-energy water/bone ellipse phantoms (the same recipe as the
phantom module) rasterised on the device, projected with the Joseph
projector and given 0.5 % Gaussian noise; plain ADM-TV provides the input
(5 iterations) and the target (200 iterations) of each training pair.

Evaluation (time to tolerance): J_ref = J(plain f^200) per phantom, the
objective of Eq. 4 summed over both energies.  Plain time = time of the first
k iterations with J(f^k) <= J_ref.  Learned time = 5 iterations + U-Net
inference + the start check + ADM-TV continued until J <= J_ref.  Plain ADM
stays the judge of the network's error and its fallback: the continuation
runs the unchanged method, from the network output when that is finite and
its objective J(x_net) does not exceed J(f^5), and otherwise by resuming the
plain run at f^5 (its multipliers and step kept), so that a failed network
costs only its own time.

Command line (one GPU):
    python -m paper_1607_01650_amd.warmstart --n-train 2000 --n-eval 200 \\
        --weights-out unet.npz --json-out warmstart.json
    python -m paper_1607_01650_amd.warmstart --weights-in unet.npz --n-eval 200
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time
from typing import Callable, Dict, Optional, Tuple

import numpy as np
import torch

from . import configs as C
from . import dect
from . import nn as NN
from . import phantom as P

EARLY = 5
LATE = 200
TRAIN_SEED0 = 0            # training phantoms: seeds 0 .. n_train-1
EVAL_SEED0 = 2000          # held-out phantoms: seeds 2000 .. 2000+n_eval-1


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


class Solver:
    """Plain ADM-TV for one geometry on fixed device buffers: every case is
    copied into the same sinogram buffer, so the library's captured iteration
    graphs are reused from case to case."""

    def __init__(self, geom: C.Geometry, params: Optional[C.AdmParams] = None):
        self.geom = geom
        self.p = params or C.default_adm_params(geom, LATE)
        self.m = torch.empty((2, geom.n_views, geom.n_bins), device="cuda")
        self.x = torch.empty((2, geom.ny, geom.nx), device="cuda")
        # resumable runs: the plain one (kept at f^5 as the fallback) and the
        # one started from the network output
        self.st_plain = dect.AdmState(geom)
        self.st_net = dect.AdmState(geom)

    def load(self, sino: torch.Tensor):
        self.m.copy_(sino)

    def run(self, iters: int, x0=None, log: bool = False,
            state: Optional[dect.AdmState] = None) -> dect.AdmResult:
        """`iters` iterations from zero (or from x0 = (x_high, x_low)), or
        continued on `state`; the result's images are views of this solver's
        output buffer."""
        p = dataclasses.replace(self.p, max_iter=iters)
        return dect.adm_tv(self.m[0], self.m[1], self.geom, p, x0=x0, want_log=log,
                           out=(self.x[0], self.x[1]), state=state)


def warm_start(net: NN.UNet, sol: Solver, corrupt: Optional[Callable] = None):
    """Five plain iterations, the network, and the choice of the start.

    Returns (state, kind): the ADM state to continue and why it was chosen:
    "net" when the network output is finite and J(x_net) <= J(f^5), else
    "nonfinite" or "objective", and then the state is the plain run itself,
    resumed at f^5.  `corrupt(y_high, y_low)`, when given, edits the network
    output in place before the check (a test hook)."""
    st5 = sol.st_plain
    st5.reset()
    J5 = sol.run(EARLY, log=True, state=st5).report.objective
    yh, yl = NN.predict(net, sol.x[0][None], sol.x[1][None])
    if corrupt is not None:
        corrupt(yh, yl)
    if not bool(torch.isfinite(yh).all() & torch.isfinite(yl).all()):
        return st5, "nonfinite"
    stn = sol.st_net
    stn.reset()
    Jn = sol.run(0, x0=(yh[0], yl[0]), log=True, state=stn).report.objective
    if not (math.isfinite(Jn) and Jn <= J5):
        return st5, "objective"
    return stn, "net"


def make_pairs(geom: C.Geometry, seeds, log_every: int = 0):
    """Early (f^5/beta) and late (f^200/beta) images [n,2,ny,nx] for the seeds."""
    sol = Solver(geom)
    n = len(seeds)
    early = torch.empty((n, 2, geom.ny, geom.nx), device="cuda")
    late = torch.empty_like(early)
    t0 = time.time()
    for i, sd in enumerate(seeds):
        _, sino = make_case(geom, sd)
        sol.load(sino)
        sol.run(EARLY)
        early[i].copy_(sol.x)
        sol.run(LATE)
        late[i].copy_(sol.x)
        if log_every and (i + 1) % log_every == 0:
            torch.cuda.synchronize()
            print(f"  pairs {i + 1}/{n}  {time.time() - t0:.1f}s", flush=True)
    torch.cuda.synchronize()
    return early, late


def train(net: NN.UNet, early: torch.Tensor, late: torch.Tensor, epochs: int = 10,
          batch: int = 8, lr: float = 1e-3, seed: int = 0, seconds: float = 0.0,
          log: bool = True) -> Dict:
    """Adam on the MSE between base + network residual and the late image
    (both scaled by NN.SCALE), cosine learning-rate decay over `epochs`;
    stops early after `seconds` of training when that is > 0."""
    rng = np.random.default_rng(seed)
    n = early.shape[0]
    losses = []
    t0 = time.time()
    steps = 0
    for ep in range(epochs):
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / max(1, epochs)))
        for b0 in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(order[b0:b0 + batch], device="cuda")
            e = early.index_select(0, idx)
            x, base = NN.pack_input(e[:, 0], e[:, 1])
            tgt = (late.index_select(0, idx).permute(0, 2, 3, 1) * NN.SCALE).contiguous()
            r = net.forward(x, keep=True)
            y = (base + r).contiguous()
            dy = torch.empty_like(y)
            parts = NN.mse(y, tgt, dy)
            net.backward(dy)
            net.adam_step(lr_ep)
            tot += float(parts.sum()) / tgt.numel()
            cnt += 1
            steps += 1
        losses.append(tot / max(cnt, 1))
        if log:
            print(f"  epoch {ep}: mse {losses[-1]:.4e}  ({time.time() - t0:.1f}s)", flush=True)
        if seconds > 0 and time.time() - t0 > seconds:
            break
    return {"losses": losses, "epochs_run": len(losses), "steps": steps,
            "train_s": time.time() - t0}


def first_reach(J: np.ndarray, target: float) -> int:
    """First index k with J[k] <= target, or -1."""
    hit = np.nonzero(J <= target * (1 + 1e-12))[0]
    return int(hit[0]) if hit.size else -1


def _timed(fn, reps: int = 3) -> float:
    """Median wall time of fn() over reps runs, the device drained around each."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def evaluate_case(net: NN.UNet, sol: Solver, sino: torch.Tensor, max_cont: int = 400,
                  reps: int = 3, corrupt: Optional[Callable] = None) -> Dict:
    """Time to J_ref = J(plain f^200) for one case, plain vs learned (with
    the fallback of warm_start)."""
    sol.load(sino)
    Jp = sol.run(LATE, log=True).J.sum(axis=1)
    J_ref = float(Jp[LATE])
    k_plain = first_reach(Jp, J_ref)
    sol.run(k_plain)
    plain_img = sol.x.clone()

    def learned_start():
        sol.run(EARLY)
        return NN.predict(net, sol.x[0][None], sol.x[1][None])

    # filtered back-projection start (the paper's analytic reconstruction)
    def fbp_start():
        return dect.fbp(sol.m, sol.geom)

    xf = fbp_start()
    Jf = sol.run(max_cont, x0=(xf[0].clone(), xf[1].clone()), log=True).J.sum(axis=1)
    k_fbp = first_reach(Jf, J_ref)

    st, kind = warm_start(net, sol, corrupt)
    Jc = sol.run(max_cont, log=True, state=st).J.sum(axis=1)
    k_cont = first_reach(Jc, J_ref)
    row = dict(J_ref=J_ref, k_plain=k_plain, k_cont=k_cont, start=kind, J_start=float(Jc[0]),
               k_fbp=k_fbp, J_fbp=float(Jf[0]))
    t_plain = _timed(lambda: sol.run(k_plain), reps)
    row["t_plain_ms"] = 1e3 * t_plain
    if k_fbp >= 0:
        def fbp_run():
            a = fbp_start()
            sol.run(k_fbp, x0=(a[0], a[1]))

        row["t_fbp_ms"] = 1e3 * _timed(fbp_run, reps)
    else:
        row["t_fbp_ms"] = float("nan")
    if k_cont < 0:
        row.update(t_learned_ms=float("nan"), learned_img=None, plain_img=plain_img)
        return row

    def learned():
        st2, kind2 = warm_start(net, sol, corrupt)
        assert kind2 == kind
        sol.run(k_cont, state=st2)

    t_learned = _timed(learned, reps)
    t_net = _timed(lambda: learned_start(), reps)
    learned()
    row.update(t_learned_ms=1e3 * t_learned, t_start_ms=1e3 * t_net,
               learned_img=sol.x.clone(), plain_img=plain_img)
    return row


def evaluate(net: NN.UNet, geom: C.Geometry, seeds, max_cont: int = 400, reps: int = 3,
             log_every: int = 0) -> Dict:
    sol = Solver(geom)
    rows = []
    for i, sd in enumerate(seeds):
        _, sino = make_case(geom, sd)
        r = evaluate_case(net, sol, sino, max_cont, reps)
        r.pop("learned_img")
        r.pop("plain_img")
        r["seed"] = int(sd)
        rows.append(r)
        if log_every and (i + 1) % log_every == 0:
            print(f"  eval {i + 1}/{len(seeds)}", flush=True)
    return summarize(rows)


def summarize(rows) -> Dict:
    ok = [r for r in rows if r["k_cont"] >= 0]
    starts = {}
    for r in rows:
        starts[r.get("start", "net")] = starts.get(r.get("start", "net"), 0) + 1
    ratios = np.array([r["t_learned_ms"] / r["t_plain_ms"] for r in ok])
    it_l = np.array([EARLY + r["k_cont"] for r in ok])
    it_p = np.array([r["k_plain"] for r in ok])
    med = lambda a: float(np.median(a)) if len(a) else float("nan")
    fb = [r for r in rows if r.get("k_fbp", -1) >= 0 and np.isfinite(r.get("t_fbp_ms", np.nan))]
    return {
        "fbp": {"reached": len(fb),
                "median_time_ratio": med([r["t_fbp_ms"] / r["t_plain_ms"] for r in fb])},
        "n": len(rows), "reached": len(ok),
        "median_k_plain": med([r["k_plain"] for r in rows]),
        "median_iters_learned": med(it_l),
        "median_t_plain_ms": med([r["t_plain_ms"] for r in ok]),
        "median_t_learned_ms": med([r["t_learned_ms"] for r in ok]),
        "median_t_start_ms": med([r["t_start_ms"] for r in ok]),
        "median_time_ratio": med(ratios),
        "mean_time_ratio": float(ratios.mean()) if len(ratios) else float("nan"),
        "frac_faster": float((ratios < 1).mean()) if len(ratios) else float("nan"),
        "p10_p90_time_ratio": ([float(np.percentile(ratios, 10)), float(np.percentile(ratios, 90))]
                               if len(ratios) else None),
        "iters_saved_median": med(it_p - it_l),
        "starts": starts,
        "fallbacks": len(rows) - starts.get("net", 0),
        "rows": rows,
    }


def save_weights(net: NN.UNet, path: str, optimizer: bool = True):
    """FP32 master weights and biases; with optimizer, also the Adam moments
    and step count, so that training can resume exactly where it stopped."""
    arrs = {}
    for i, c in enumerate(net.layers()):
        arrs[f"l{i}_w"] = c.w.cpu().numpy()
        arrs[f"l{i}_b"] = c.b.cpu().numpy()
        if optimizer:
            arrs[f"l{i}_mw"] = c.mw.cpu().numpy()
            arrs[f"l{i}_vw"] = c.vw.cpu().numpy()
            arrs[f"l{i}_mb"] = c.mb.cpu().numpy()
            arrs[f"l{i}_vb"] = c.vb.cpu().numpy()
    if optimizer:
        arrs["adam_step"] = np.array(net.step, dtype=np.int64)
    np.savez(path, **arrs)


def load_weights(net: NN.UNet, path: str):
    """Weights (and the Adam state when the file holds it) saved by save_weights."""
    z = np.load(path, allow_pickle=False)
    sd = {}
    for i, _ in enumerate(net.layers()):
        sd[f"l{i}"] = (torch.as_tensor(z[f"l{i}_w"]), torch.as_tensor(z[f"l{i}_b"]))
    net.load_state_dict(sd)
    if "adam_step" in z.files:
        for i, c in enumerate(net.layers()):
            c.mw.copy_(torch.as_tensor(z[f"l{i}_mw"]))
            c.vw.copy_(torch.as_tensor(z[f"l{i}_vw"]))
            c.mb.copy_(torch.as_tensor(z[f"l{i}_mb"]))
            c.vb.copy_(torch.as_tensor(z[f"l{i}_vb"]))
        net.step = int(z["adam_step"])


def summary_markdown(out: Dict, command: str) -> str:
    """A short text record of an evaluation: the figures, not the rows."""
    ev = out["eval"]
    lo, hi = ev["p10_p90_time_ratio"] or (float("nan"), float("nan"))
    lines = [
        f"# Learned warm start: time to the plain method's objective, {ev['n']} held-out phantoms",
        "",
        "Command (from the repository root, one MI355X):",
        "",
        f"    {command}",
        "",
        f"Workload: {out['workload']}; held-out phantoms (seeds {EVAL_SEED0} .. "
        f"{EVAL_SEED0 + ev['n'] - 1}, never seen in training); J_ref = J(plain f^{LATE}) per "
        "phantom (Eq. 4, both energies).  Plain: ADM-TV until J <= J_ref.  Learned: "
        f"{EARLY} plain iterations, the U-Net, the start check, then ADM-TV until J <= J_ref; "
        "a start that is not finite or whose objective exceeds J(f^5) falls back to the "
        "plain run resumed at f^5.  Wall times are medians of repeated runs on the GPU.",
        "",
        "| figure | value |",
        "|---|---|",
        f"| cases / reached J_ref | {ev['n']} / {ev['reached']} |",
        f"| starts from the network / fallbacks | {ev['starts'].get('net', 0)} / {ev['fallbacks']} |",
        f"| median plain iterations | {ev['median_k_plain']:.0f} |",
        f"| median learned iterations (5 + continuation) | {ev['median_iters_learned']:.0f} |",
        f"| median plain time | {ev['median_t_plain_ms']:.2f} ms |",
        f"| median learned time (incl. network and check) | {ev['median_t_learned_ms']:.2f} ms |",
        f"| median network start (5 iterations + U-Net) | {ev['median_t_start_ms']:.2f} ms |",
        f"| median time ratio learned / plain | {ev['median_time_ratio']:.3f} |",
        f"| p10 - p90 time ratio | {lo:.3f} - {hi:.3f} |",
        f"| learned faster than plain | {100 * ev['frac_faster']:.1f} % of cases |",
        f"| median iterations saved | {ev['iters_saved_median']:.0f} |",
    ]
    if "fbp" in ev:
        f = ev["fbp"]
        lines.append(f"| FBP start: reached / median time ratio | {f['reached']} / "
                     f"{f['median_time_ratio']:.3f} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--views", type=int, default=90)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-eval", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-seconds", type=float, default=0.0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--weights-in", default=None)
    ap.add_argument("--weights-out", default=None)
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--md-out", default=None, help="short text record of the evaluation")
    a = ap.parse_args(argv)
    geom = C.paper_geometry(a.size, a.views)
    net = NN.UNet(seed=0)
    out = {"workload": f"learned warm start, {a.size}x{a.size}, {a.views} views, "
                       f"{geom.n_bins} bins, 2 energies",
           "early_iters": EARLY, "late_iters": LATE, "n_params": net.n_params()}
    if a.weights_in:
        load_weights(net, a.weights_in)
        out["weights"] = a.weights_in
    else:
        t0 = time.time()
        early, late = make_pairs(geom, list(range(TRAIN_SEED0, TRAIN_SEED0 + a.n_train)),
                                 log_every=100)
        out["datagen_s"] = time.time() - t0
        print(f"pairs: {a.n_train} in {out['datagen_s']:.1f}s", flush=True)
        tr = train(net, early, late, epochs=a.epochs, batch=a.batch, lr=a.lr,
                   seconds=a.train_seconds)
        out.update(n_train=a.n_train, batch=a.batch, lr=a.lr, **tr)
        del early, late
        if a.weights_out:
            save_weights(net, a.weights_out)
    if a.n_eval > 0:
        ev = evaluate(net, geom, list(range(EVAL_SEED0, EVAL_SEED0 + a.n_eval)), reps=a.reps,
                      log_every=20)
        out["eval"] = ev
        print(json.dumps({k: v for k, v in ev.items() if k != "rows"}), flush=True)
    if a.json_out:
        with open(a.json_out, "w") as f:
            json.dump(out, f, indent=1)
    if a.md_out and "eval" in out:
        import sys
        cmd = "python -m paper_1607_01650_amd.warmstart " + " ".join(argv if argv is not None
                                                                     else sys.argv[1:])
        with open(a.md_out, "w") as f:
            f.write(summary_markdown(out, cmd))


if __name__ == "__main__":
    main()
