"""Benchmark: ADM-TV iterations/s at 512^2 x 360 views x 736 bins x 2 energies.

One step = one ADM-TV iteration (Eq. 10) of both energy images: the fused
TV/shrink/gradient stencil, the forward projection of G, the step, the image
and residual update and the back-projection, all on the GPU (replayed as a
hipGraph).  Inputs (seeded water/bone ellipse phantom, analytic sinograms
with 0.5 % Gaussian noise) are resident in HBM before timing starts.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (the gather back-projection, timed with HIP events on the stream it
is launched on, set against the VALU issue peak with its instruction count
from rocprofv3 counters) and the FP64 CPU oracle timed on a bounded sample.

Other modes (for hardware-counter runs under rocprofv3, one GPU):
  --mode projectors   only the back- and forward-projection launches of the
                      roofline entry (same inputs and launch configuration)
  --mode copy         device-to-device copies of --copy-mb MiB: a kernel of
                      known traffic that calibrates FETCH_SIZE / WRITE_SIZE
  --mode counters     reads the counter CSVs of those runs (--pmc-dir) and
                      writes profiles/adm_tv_512x512_360v_counters.json
                      (no GPU needed)
"""
from __future__ import annotations

import argparse
import ctypes as ct
import dataclasses
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


class HipEvents:
    """hipEventRecord/ElapsedTime through the HIP runtime (any stream)."""

    def __init__(self):
        self.h = ct.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ct.POINTER(ct.c_void_p)]
        self.h.hipEventRecord.argtypes = [ct.c_void_p, ct.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ct.c_void_p]
        self.h.hipEventElapsedTime.argtypes = [ct.POINTER(ct.c_float), ct.c_void_p, ct.c_void_p]
        self.h.hipEventDestroy.argtypes = [ct.c_void_p]

    def event(self):
        e = ct.c_void_p()
        assert self.h.hipEventCreate(ct.byref(e)) == 0
        return e

    def record(self, e, stream):
        assert self.h.hipEventRecord(e, stream) == 0

    def ms(self, a, b):
        assert self.h.hipEventSynchronize(b) == 0
        out = ct.c_float()
        assert self.h.hipEventElapsedTime(ct.byref(out), a, b) == 0
        return float(out.value)


def cpu_baseline(geom, sino, p, seconds_hint: float = 15.0):
    """The FP64 oracle's ADM iterations/s (both energies) on a bounded sample:
    t(K2) - t(K1) over K2 - K1 iterations excludes the shared set-up."""
    from oracle import oracle as O
    import numpy as np
    m = [np.asarray(sino[e], dtype=np.float32).astype(np.float64) for e in (0, 1)]
    betas = (p.beta_high, p.beta_low)

    def run(k):
        t0 = time.perf_counter()
        for e in (0, 1):
            O.adm(geom, m[e], betas[e], p.mu, p.rho, p.xi, k)
        return time.perf_counter() - t0

    t1 = run(1)
    per_iter = max(t1 / 3.0, 1e-3)
    k2 = max(3, min(20, int(seconds_hint / per_iter)))
    t2 = run(k2)
    rate = (k2 - 1) / max(t2 - t1, 1e-9)
    return {"value": round(rate, 4), "unit": "iters/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"ADM-TV both energies, 512x512, 360 views, 736 bins, FP64; "
                      f"(t({k2} it) - t(1 it)) / {k2 - 1}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel-launches", type=int, default=50)
    ap.add_argument("--mode", choices=["metric", "projectors", "copy", "counters", "cone"],
                    default="metric")
    ap.add_argument("--copy-mb", type=int, default=512)
    ap.add_argument("--pmc-dir", default="pmc", help="directory of the counter runs (--mode counters)")
    ap.add_argument("--warm-cases", type=int, default=4,
                    help="held-out cases for the learned-warm-start time-to-tol entry")
    ap.add_argument("--batch-slices", type=int, default=64,
                    help="slices of the batched multi-slice entry (0: skip)")
    ap.add_argument("--batch-iters", type=int, default=20)
    ap.add_argument("--unet-steps", type=int, default=5,
                    help="timed training steps / inferences of the U-Net entry (0: skip)")
    ap.add_argument("--unrolled-steps", type=int, default=3,
                    help="timed training steps of the unrolled-ADM entry (0: skip)")
    ap.add_argument("--siddon-steps", type=int, default=100,
                    help="timed ADM iterations of the Siddon-model entry (0: skip)")
    ap.add_argument("--no-fbp", action="store_true",
                    help="skip the filtered back-projection comparator entry")
    ap.add_argument("--nonneg-steps", type=int, default=100,
                    help="timed ADM iterations of the non-negative, coupled-TV and "
                         "adaptive-step variant entries (0: skip)")
    ap.add_argument("--cone-launches", type=int, default=3,
                    help="timed calls of each cone-beam projector (0: skip)")
    ap.add_argument("--adm3-iters", type=int, default=6,
                    help="iterations of the 3-D ADM entry (0: skip; at least 2)")
    ap.add_argument("--prewarm-ms", type=float, default=150.0,
                    help="untimed ADM iterations on a separate state for about this long "
                         "before the warmup steps, so that the timed steps see the GPU at its "
                         "sustained clock (0: none)")
    args = ap.parse_args()
    if args.mode == "counters":
        return counters_summary(args.pmc_dir)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the whole path on a single MI355X "
              "(multi-GPU sharding is described, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.mode == "copy":
        return copy_probe(args.copy_mb, args.kernel_launches)
    if args.mode == "projectors":
        return projector_launches(args.kernel_launches)
    if args.mode == "cone":  # the cone-beam projector pair and the 3-D ADM alone
        print(json.dumps({"cone": cone_extra(max(1, args.cone_launches)),
                          "adm3": adm3_extra(max(2, args.adm3_iters))}), flush=True)
        return
    g = C.METRIC
    s = P.make_slice(g, 0)
    p = C.default_adm_params(g, args.steps)
    mh = torch.as_tensor(s.sino[0], dtype=torch.float32).cuda()
    ml = torch.as_tensor(s.sino[1], dtype=torch.float32).cuda()
    xh = torch.empty((g.ny, g.nx), device="cuda")
    xl = torch.empty_like(xh)
    stream = torch.cuda.current_stream()
    sp = ct.c_void_p(stream.cuda_stream)
    ev = HipEvents()

    # the GPU raises its clock under sustained load: a short timed window
    # right after idle measures the ramp (about 7% lower at 20 steps), so the
    # device first runs untimed iterations of the same workload on its own
    # state; the timed state then gets exactly `warmup` untimed steps
    prewarm_its = 0
    if args.prewarm_ms > 0:
        pre = dect.AdmState(g)
        chunk = dataclasses.replace(p, max_iter=50)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        while (time.perf_counter() - w0) * 1e3 < args.prewarm_ms:
            dect.adm_tv(mh, ml, g, chunk, state=pre, out=(xh, xl))
            torch.cuda.synchronize()
            prewarm_its += chunk.max_iter
        pre.close()
    state = dect.AdmState(g)
    dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=args.warmup), state=state,
                out=(xh, xl))
    timed = dataclasses.replace(p, max_iter=args.steps)
    torch.cuda.synchronize()
    e0, e1 = ev.event(), ev.event()
    t0 = time.perf_counter()
    ev.record(e0, sp)
    dect.adm_tv(mh, ml, g, timed, state=state, out=(xh, xl))
    ev.record(e1, sp)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev.ms(e0, e1)
    iters_per_s = args.steps / (gpu_ms / 1e3)

    # dominant kernel: the gather back-projection of both energies (same
    # launch as inside the iteration), timed with HIP events
    r = torch.randn((2, g.n_views, g.n_bins), device="cuda")
    img = torch.empty((2, g.ny, g.nx), device="cuda")
    for _ in range(3):
        dect.backproject(r, g, out=img)
    a0, a1 = ev.event(), ev.event()
    ev.record(a0, sp)
    for _ in range(args.kernel_launches):
        dect.backproject(r, g, out=img)
    ev.record(a1, sp)
    adj_ms = ev.ms(a0, a1) / args.kernel_launches
    S = dect.count_samples(g)
    M, N = g.n_views * g.n_bins, g.nx * g.ny
    adj_bytes = 2 * (8 * S + 4 * M + 4 * N)

    # forward projection of both energies for context
    x = torch.randn((2, g.ny, g.nx), device="cuda")
    sino = torch.empty((2, g.n_views, g.n_bins), device="cuda")
    for _ in range(3):
        dect.project(x, g, out=sino)
    f0, f1 = ev.event(), ev.event()
    ev.record(f0, sp)
    for _ in range(args.kernel_launches):
        dect.project(x, g, out=sino)
    ev.record(f1, sp)
    fwd_ms = ev.ms(f0, f1) / args.kernel_launches

    # PLS decomposition of the reconstruction (gamma = 1)
    pp = C.PlsParams(gamma=1.0, tol=1e-6)
    dect.pls_decompose(xh, xl, pp)
    torch.cuda.synchronize()
    q0 = time.perf_counter()
    _, _, prep = dect.pls_decompose(xh, xl, pp)
    torch.cuda.synchronize()
    pls_ms = (time.perf_counter() - q0) * 1e3
    # the attenuation-space variant (|x - Du|^2 + gamma R), gamma in the paper's range
    pa = C.PlsParams(gamma=1e-4, tol=1e-6, mode=1)
    dect.pls_decompose(xh, xl, pa)
    torch.cuda.synchronize()
    q0 = time.perf_counter()
    _, _, arep = dect.pls_decompose(xh, xl, pa)
    torch.cuda.synchronize()
    pls_att_ms = (time.perf_counter() - q0) * 1e3

    warm = warm_start_extra(args.warm_cases)
    batched = batched_extra(args.batch_slices, args.batch_iters) if args.batch_slices > 0 else None
    unrolled = unrolled_extra(args.unrolled_steps) if args.unrolled_steps > 0 else None
    unet = unet_extra(args.unet_steps) if args.unet_steps > 0 else None
    siddon = (siddon_extra(args.siddon_steps, args.kernel_launches)
              if args.siddon_steps > 0 else None)
    fbp = None if args.no_fbp else fbp_extra(max(1, args.kernel_launches))
    nonneg = nonneg_extra(args.nonneg_steps) if args.nonneg_steps > 0 else None
    coupled = nonneg_extra(args.nonneg_steps, coupled=True) if args.nonneg_steps > 0 else None
    abb = nonneg_extra(args.nonneg_steps, step="abb") if args.nonneg_steps > 0 else None
    cone = cone_extra(args.cone_launches) if args.cone_launches > 0 else None
    adm3 = adm3_extra(max(2, args.adm3_iters)) if args.adm3_iters > 0 else None

    roofline = adjoint_roofline(adj_ms, adj_bytes)

    out = {
        "metric": "ADM-TV iters/s at 512x512 x 360 views x 2 energies",
        "value": round(iters_per_s, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "adm_tv_512x512_360views_736bins_2energies", "image": 512,
                   "views": 360, "bins": 736, "energies": 2, "sod_mm": g.sod_mm,
                   "sdd_mm": g.sdd_mm, "mu": p.mu, "rho": p.rho, "xi": p.xi},
        "roofline": roofline,
        "extra": {"fwd_projection_us_2energies": round(fwd_ms * 1e3, 2),
                  "samples_per_projection": S,
                  "ray_updates_per_s": round(4 * S * iters_per_s, 1),
                  "wall_s_timed": round(wall, 4),
                  "prewarm_iterations": prewarm_its,
                  "pls_ms": round(pls_ms, 3), "pls_pcg_iters": prep.iters,
                  "pls_attenuation_ms": round(pls_att_ms, 3), "pls_attenuation_iters": arep.iters,
                  "warm_start": warm, "batched": batched, "unrolled": unrolled, "unet": unet,
                  "siddon": siddon, "fbp": fbp, "nonneg": nonneg, "coupled_tv": coupled,
                  "abb_step": abb, "cone": cone, "adm3": adm3},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, s.sino, p)
    print(json.dumps(out), flush=True)


def adjoint_roofline(adj_ms: float, adj_bytes: int):
    """The roofline entry of the dominant kernel, the gather back-projection
    of both energies (k_adj + k_adj_sum, one dect_backproject launch).

    Its operands come from LDS and L2 (HBM carries a few percent of its
    algorithmic bytes), and what binds it is instruction issue: the entry
    sets the wave-level VALU instructions of one launch (counted by rocprofv3,
    profiles/adm_tv_512x512_360v_counters.json, valid while the kernel sources
    hash the same) over the launch time measured here against the VALU issue
    peak (VALU_PEAK_GINST).  The measured HBM bytes of a launch (the same
    counter file) give `traffic` and the HBM fraction; the algorithmic bytes
    (8 B per Joseph sample per image + 4 B per ray + 4 B per pixel) over the
    launch time give the effective gather bandwidth."""
    t = adj_ms / 1e3
    eff = adj_bytes / t / 1e9
    roof = {"bound": "alu", "achieved": None, "peak": round(VALU_PEAK_GINST, 1),
            "unit": "Ginst/s", "frac": None, "traffic": None,
            "kernel": "k_adj + k_adj_sum (gather back-projection, 2 energies)",
            "avg_launch_us": round(adj_ms * 1e3, 2), "algorithmic_bytes": adj_bytes,
            "effective_gbs": round(eff, 1), "effective_over_hbm_peak": round(eff / HBM_PEAK_GBS, 3),
            "counters": None}
    cfile = os.path.join(ROOT, "profiles", "adm_tv_512x512_360v_counters.json")
    try:
        info = json.load(open(cfile))
    except Exception:
        return roof
    if info.get("kernel_hash") != _counter_sources_hash():
        roof["counters"] = "stale (kernel sources changed since the counter runs)"
        return roof
    k = info["kernels"]
    a, s_ = k["k_adj"], k["k_adj_sum"]
    valu = a["SQ_INSTS_VALU"] + s_["SQ_INSTS_VALU"]
    traffic = (a["hbm_read_bytes"] + a["hbm_write_bytes"] + s_["hbm_read_bytes"] +
               s_["hbm_write_bytes"])
    achieved = valu / t / 1e9
    roof.update(achieved=round(achieved, 1), frac=round(achieved / VALU_PEAK_GINST, 4),
                traffic=round(traffic), counters=os.path.relpath(cfile, ROOT),
                valu_instr_per_launch=valu,
                hbm_gbs=round(traffic / t / 1e9, 1),
                hbm_frac=round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                lds_instr_per_launch=a["SQ_INSTS_LDS"] + s_["SQ_INSTS_LDS"])
    return roof


def siddon_extra(steps: int, launches: int):
    """The metric workload on the Siddon ray model (pixel intersection
    lengths): ADM iterations/s and both projectors' launch times."""
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    g = dataclasses.replace(C.METRIC, model=1)
    s = P.make_slice(C.METRIC, 0)
    p = C.default_adm_params(C.METRIC, steps)
    mh = torch.as_tensor(s.sino[0], dtype=torch.float32).cuda()
    ml = torch.as_tensor(s.sino[1], dtype=torch.float32).cuda()
    xh = torch.empty((g.ny, g.nx), device="cuda")
    xl = torch.empty_like(xh)
    sp = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = HipEvents()
    state = dect.AdmState(g)
    dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=5), state=state, out=(xh, xl))
    torch.cuda.synchronize()
    e0, e1 = ev.event(), ev.event()
    ev.record(e0, sp)
    dect.adm_tv(mh, ml, g, p, state=state, out=(xh, xl))
    ev.record(e1, sp)
    torch.cuda.synchronize()
    adm_ms = ev.ms(e0, e1) / steps

    def per_launch(fn):
        for _ in range(3):
            fn()
        a0, a1 = ev.event(), ev.event()
        ev.record(a0, sp)
        for _ in range(launches):
            fn()
        ev.record(a1, sp)
        torch.cuda.synchronize()
        return ev.ms(a0, a1) / launches

    r = torch.randn((2, g.n_views, g.n_bins), device="cuda")
    img = torch.empty((2, g.ny, g.nx), device="cuda")
    x = torch.randn((2, g.ny, g.nx), device="cuda")
    sino = torch.empty((2, g.n_views, g.n_bins), device="cuda")
    adj_ms = per_launch(lambda: dect.backproject(r, g, out=img))
    fwd_ms = per_launch(lambda: dect.project(x, g, out=sino))
    return {"workload": "adm_tv_512x512_360views_736bins_2energies, Siddon model",
            "iters_per_s": round(1e3 / adm_ms, 2), "ms_per_iteration": round(adm_ms, 4),
            "steps": steps, "backprojection_us_2energies": round(adj_ms * 1e3, 2),
            "fwd_projection_us_2energies": round(fwd_ms * 1e3, 2)}


def nonneg_extra(steps: int, coupled: bool = False, step: str = "bb1"):
    """The metric workload with every f-step projected onto f >= 0
    (DECT_NONNEG), with the TV coupled across the energies (DECT_COUPLED_TV),
    or with another BB step rule (DECT_STEP_BB2 / DECT_STEP_ABB): ADM
    iterations/s."""
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    g = C.METRIC
    s = P.make_slice(g, 0)
    plain_step = step == "bb1"
    p = dataclasses.replace(C.default_adm_params(g, steps), nonneg=not coupled and plain_step,
                            coupled_tv=coupled, step=step)
    mh = torch.as_tensor(s.sino[0], dtype=torch.float32).cuda()
    ml = torch.as_tensor(s.sino[1], dtype=torch.float32).cuda()
    xh = torch.empty((g.ny, g.nx), device="cuda")
    xl = torch.empty_like(xh)
    sp = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = HipEvents()
    state = dect.AdmState(g)
    dect.adm_tv(mh, ml, g, dataclasses.replace(p, max_iter=5), state=state, out=(xh, xl))
    torch.cuda.synchronize()
    e0, e1 = ev.event(), ev.event()
    ev.record(e0, sp)
    dect.adm_tv(mh, ml, g, p, state=state, out=(xh, xl))
    ev.record(e1, sp)
    torch.cuda.synchronize()
    ms = ev.ms(e0, e1) / steps
    state.close()
    what = ("TV coupled across energies" if coupled else
            "f >= 0" if plain_step else step + " step")
    out = {"workload": "adm_tv_512x512_360views_736bins_2energies, " + what,
           "iters_per_s": round(1e3 / ms, 2), "ms_per_iteration": round(ms, 4), "steps": steps}
    if not coupled and plain_step:
        out["zero_pixels"] = int((xh == 0).sum().item() + (xl == 0).sum().item())
    return out


def cone_extra(launches: int):
    """Cone-beam projector pair on a 512 x 512 x 64 volume, 360 views, 64 x 736
    detector (the metric fan with 64 rows): time per forward and per
    back-projection call, Joseph samples (ray, plane) per second, and the
    rate of the algorithmic bytes (volume read once, projections written
    once, or the reverse) against HBM."""
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    g = C.CONE
    vol = torch.as_tensor(P.cone_volume(g, 0, supersample=2), dtype=torch.float32).cuda()
    proj = torch.empty((g.n_views, g.n_rows, g.n_bins), device="cuda")
    back = torch.empty_like(vol)
    sp = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = HipEvents()
    dect.cone_project(vol, g, out=proj)
    dect.cone_backproject(proj, g, out=back)
    a0, a1, a2 = ev.event(), ev.event(), ev.event()
    ev.record(a0, sp)
    for _ in range(launches):
        dect.cone_project(vol, g, out=proj)
    ev.record(a1, sp)
    for _ in range(launches):
        dect.cone_backproject(proj, g, out=back)
    ev.record(a2, sp)
    torch.cuda.synchronize()
    fwd_ms, adj_ms = ev.ms(a0, a1) / launches, ev.ms(a1, a2) / launches
    rays = g.n_views * g.n_rows * g.n_bins
    samples = rays * g.nx  # every ray steps over all planes of its driving axis (nx == ny)
    nbytes = 4 * (g.nx * g.ny * g.nz + rays)
    return {"workload": "cone_512x512x64_360views_64x736det", "launches": launches,
            "fwd_ms": round(fwd_ms, 3), "back_ms": round(adj_ms, 3),
            "fwd_gsamples_per_s": round(samples / fwd_ms / 1e6, 2),
            "back_gsamples_per_s": round(samples / adj_ms / 1e6, 2),
            "fwd_algorithmic_gbs": round(nbytes / fwd_ms / 1e6, 1),
            "back_algorithmic_gbs": round(nbytes / adj_ms / 1e6, 1)}


def adm3_extra(iters: int):
    """3-D ADM-TV of both energies on the cone workload (512 x 512 x 64, 360
    views, 64 x 736 panel): wall time per iteration of the call (both
    energies, the stream synchronised at its end), from the difference of an
    iters-long and a 1-iteration run so that set-up is excluded."""
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    g = C.CONE
    vol = torch.as_tensor(P.cone_volume(g, 0, supersample=2), dtype=torch.float32).cuda()
    mh = dect.cone_project(vol, g)
    ml = dect.cone_project(vol * 1.3, g)
    p = C.AdmParams(mu=45.0 / g.n_views, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79,
                    max_iter=1)
    dect.adm_tv3(mh, ml, g, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dect.adm_tv3(mh, ml, g, p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = dect.adm_tv3(mh, ml, g, dataclasses.replace(p, max_iter=iters), want_log=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    per_it = ((t2 - t1) - (t1 - t0)) / (iters - 1)
    # 3-D PLS of the result (six-neighbour R), gamma 1e-3 and 1
    pls = {}
    for gamma in (1e-3, 1.0):
        dect.pls_decompose3(r.x_high, r.x_low, C.PlsParams(gamma=gamma))
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        _, _, prep = dect.pls_decompose3(r.x_high, r.x_low, C.PlsParams(gamma=gamma))
        torch.cuda.synchronize()
        pls[f"gamma_{gamma:g}"] = {"ms": round((time.perf_counter() - q0) * 1e3, 2),
                                   "pcg_iters": prep.iters}
    return {"workload": "adm_tv3_cone_512x512x64_360views_64x736det_2energies", "iters": iters,
            "ms_per_iteration_2energies": round(per_it * 1e3, 2),
            "iters_per_s": round(1.0 / per_it, 2), "pls3": pls,
            "J_first_last": [round(float(r.log[0, 0] + r.log[0, 1]), 1),
                             round(float(r.log[-1, 0] + r.log[-1, 1]), 1)]}


def fbp_extra(launches: int):
    """Filtered back-projection, the paper's analytic comparator, on the
    metric workload: time per call for both energies, and the image and
    material errors against the phantom truth beside those of ADM-TV (200
    iterations) + PLS."""
    import numpy as np
    import torch

    from paper_1607_01650_amd import configs as C, dect, phantom as P

    g = C.METRIC
    s = P.make_slice(g, 0)
    y = torch.as_tensor(s.sino, dtype=torch.float32).cuda()
    out = torch.empty((2, g.ny, g.nx), device="cuda")
    sp = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    ev = HipEvents()
    for _ in range(3):
        dect.fbp(y, g, out=out)
    a0, a1 = ev.event(), ev.event()
    ev.record(a0, sp)
    for _ in range(launches):
        dect.fbp(y, g, out=out)
    ev.record(a1, sp)
    torch.cuda.synchronize()
    fbp_us = ev.ms(a0, a1) / launches * 1e3
    r = dect.adm_tv(y[0], y[1], g, C.default_adm_params(g, 200))
    u_fbp = dect.pls_decompose(out[0], out[1], C.PlsParams(gamma=0.0, tol=1e-6))
    u_adm = dect.pls_decompose(r.x_high, r.x_low, C.PlsParams(gamma=1.0, tol=1e-6))

    def rel(a, b):
        a = a.detach().cpu().numpy().astype(np.float64)
        return round(float(np.linalg.norm(a - b) / np.linalg.norm(b)), 5)

    return {"workload": "adm_tv_512x512_360views_736bins_2energies, slice 0",
            "fbp_us_2energies": round(fbp_us, 2),
            "x_rel_err_fbp": [rel(out[e], s.x_true[e]) for e in (0, 1)],
            "x_rel_err_adm200": [rel(r.x_high, s.x_true[0]), rel(r.x_low, s.x_true[1])],
            "u_rel_err_fbp_direct": [rel(u_fbp[m], s.u_true[m]) for m in (0, 1)],
            "u_rel_err_adm200_pls": [rel(u_adm[m], s.u_true[m]) for m in (0, 1)]}


def warm_start_extra(n: int):
    """Time to the plain method's objective J(f^200), learned warm start vs
    plain ADM, on the first n held-out phantoms (512x512, 90 views) with the
    trained weights shipped in the package."""
    if n <= 0:
        return None
    import numpy as np
    from paper_1607_01650_amd import configs as C, nn as NN, warmstart as W
    path = os.path.join(ROOT, "paper_1607_01650_amd", "weights", "unet_warmstart_512_90v.npz")
    if not os.path.exists(path):
        return None
    geom = C.paper_geometry(512, 90)
    net = NN.UNet(seed=0)
    W.load_weights(net, path)
    sol = W.Solver(geom)
    rows = []
    for sd in range(W.EVAL_SEED0, W.EVAL_SEED0 + n):
        _, sino = W.make_case(geom, sd)
        r = W.evaluate_case(net, sol, sino, reps=3)
        rows.append(r)
    ok = [r for r in rows if r["k_cont"] >= 0]
    med = lambda a: float(np.median(a)) if len(a) else None
    return {"workload": "512x512, 90 views, 736 bins, 2 energies; J_ref = J(plain f^200)",
            "record_200_cases": "profiles/warmstart_eval_512x512_90v.md",
            "cases": n, "reached": len(ok),
            "median_iters_plain": med([r["k_plain"] for r in rows]),
            "median_iters_learned": med([W.EARLY + r["k_cont"] for r in ok]),
            "median_ms_plain": med([r["t_plain_ms"] for r in ok]),
            "median_ms_learned": med([r["t_learned_ms"] for r in ok]),
            "median_time_ratio": med([r["t_learned_ms"] / r["t_plain_ms"] for r in ok]),
            "fallbacks": sum(r["start"] != "net" for r in rows),
            "fbp_start": {"reached": sum(r["k_fbp"] >= 0 for r in rows),
                          "median_iters": med([r["k_fbp"] for r in rows if r["k_fbp"] >= 0]),
                          "median_ms": med([r["t_fbp_ms"] for r in rows if r["k_fbp"] >= 0]),
                          "median_time_ratio": med([r["t_fbp_ms"] / r["t_plain_ms"]
                                                    for r in rows if r["k_fbp"] >= 0])}}


def batched_extra(n_slices: int, iters: int):
    """Many slices of uneven size and view count (sizes {256, 384, 512}^2, views
    {60, 90, 180, 360}, seed 0), both energies, advanced together by the
    batched ADM (one launch per phase, graph replay, autotuned view
    grouping): slice-iterations/s, beside the same slices run one after
    another through dect_adm_tv."""
    import numpy as np
    import torch
    from paper_1607_01650_amd import configs as C, dect, warmstart as W
    rng = np.random.default_rng(0)
    sizes = rng.choice([256, 384, 512], n_slices)
    views = rng.choice([60, 90, 180, 360], n_slices)
    geoms = [C.paper_geometry(int(n), int(v)) for n, v in zip(sizes, views)]
    params = [C.default_adm_params(g, iters) for g in geoms]
    mh, ml = [], []
    for i, g in enumerate(geoms):
        _, sino = W.make_case(g, 3000 + i)
        mh.append(sino[0].contiguous())
        ml.append(sino[1].contiguous())
    b = dect.AdmBatch(geoms, params)
    b.run(mh, ml, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(mh, ml, iters)
    torch.cuda.synchronize()
    t_builtin = time.perf_counter() - t0
    t0 = time.perf_counter()
    groups, _ = b.tune(mh, ml, iters=4)
    t_tune = time.perf_counter() - t0
    per_slice, adj_cu, fwd_cu, _ = b.shape()
    b.run(mh, ml, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(mh, ml, iters)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    for i, g in enumerate(geoms):  # set-up (tables, states, graphs) outside the timing
        dect.adm_tv(mh[i], ml[i], g, dataclasses.replace(params[i], max_iter=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, g in enumerate(geoms):
        dect.adm_tv(mh[i], ml[i], g, params[i])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    samples = sum(2 * 2 * dect.count_samples(g) for g in geoms)  # fwd + adj, 2 energies
    return {"workload": f"{n_slices} slices x 2 energies, sizes {{256,384,512}}^2, views "
                        "{60,90,180,360}, seed 0",
            "iters": iters, "tuned_view_groups": groups,
            "tuned_depths": sorted(set(per_slice)), "tuned_adj_blocks_per_cu": adj_cu,
            "tuned_fwd_blocks_per_cu": fwd_cu, "tune_s": round(t_tune, 2),
            "ms_per_iteration_builtin_shape": round(1e3 * t_builtin / iters, 3),
            "slice_iters_per_s": round(n_slices * iters / t_batch, 1),
            "ray_updates_per_s": round(samples * iters / t_batch, 1),
            "ms_per_iteration_all_slices": round(1e3 * t_batch / iters, 3),
            "sequential_slice_iters_per_s": round(n_slices * iters / t_seq, 1),
            "speedup_vs_sequential": round(t_seq / t_batch, 3)}


def unet_extra(steps: int, batch: int = 8):
    """The learned warm start's network on the BF16 MFMA kernels: one training
    step (forward, MSE, backward, Adam) on a batch of 8 2-channel 512 x 512
    images, and one inference of one image; convolution flops per second."""
    import torch
    from paper_1607_01650_amd import nn as NN
    net = NN.UNet(seed=0)
    gen = torch.Generator(device="cuda").manual_seed(0)
    f = torch.rand((batch, 2, 512, 512), device="cuda", generator=gen) * 0.05
    x, base = NN.pack_input(f[:, 0], f[:, 1])
    tgt = (f.permute(0, 2, 3, 1) * NN.SCALE).contiguous()

    def train_step():
        r = net.forward(x, keep=True)
        y = (base + r).contiguous()
        dy = torch.empty_like(y)
        NN.mse(y, tgt, dy)
        net.backward(dy)
        net.adam_step(1e-4)

    for _ in range(2):
        train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        train_step()
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / steps
    x1 = x[:1].contiguous()
    for _ in range(2):
        net.forward(x1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(x1)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / steps
    fl = net.conv_flops(512, 512)
    return {"workload": f"U-Net {NN.CH}, batch {batch} x 2 x 512x512, BF16 MFMA",
            "train_step_ms": round(1e3 * t_train, 3), "infer_ms_1image": round(1e3 * t_inf, 3),
            "conv_gflop_fwd_per_image": round(fl / 1e9, 2),
            "train_conv_tflops": round(3 * fl * batch / t_train / 1e12, 2),
            "infer_conv_tflops": round(fl / t_inf / 1e12, 2)}


def unrolled_extra(steps: int, batch: int = 8):
    """One training step of 10 unrolled ADM-TV iterations with learnable
    per-step parameters (batch 8, 512^2, 180 views, checkpoint every 2): the
    projector and its adjoint run in the library, the image-domain steps are
    device tensor ops; milliseconds per forward + backward + Adam step."""
    import torch
    from paper_1607_01650_amd import configs as C, dect, unrolled as U, warmstart as W
    g = C.paper_geometry(512, 180)
    gd, xt = [], []
    for i in range(batch):
        x, sino = W.make_case(g, 4000 + i)
        gd.append(sino[0])
        xt.append(x[0])
    gdata, target = torch.stack(gd).contiguous(), torch.stack(xt).contiguous()
    # initial per-step sizes: the plain method's first ten BB steps on case 0
    p = C.default_adm_params(g, 10)
    log = dect.adm_tv(gdata[0], gdata[0], g, p, want_log=True).alpha[:10, 0]
    model = U.UnrolledADM(g, n_steps=10, mu=p.mu, rho=p.rho, xi=p.xi,
                          alphas=[float(a) for a in log], checkpoint_every=2).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=1e-2)

    def step():
        opt.zero_grad()
        f = model(gdata)
        loss = ((f - target) ** 2).mean()
        loss.backward()
        opt.step()
        return float(loss.detach())

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        last = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"workload": f"batch {batch} x 512x512, 180 views, 10 unrolled steps, checkpoint 2",
            "ms_per_train_step": round(ms, 2), "loss_mse": last}


def projector_launches(k: int):
    """The roofline entry's projector launches alone (for counter runs), with
    their average HIP-event time per launch."""
    import torch
    from paper_1607_01650_amd import configs as C, dect
    g = C.METRIC
    gen = torch.Generator(device="cuda").manual_seed(0)
    r = torch.randn((2, g.n_views, g.n_bins), device="cuda", generator=gen)
    img = torch.empty((2, g.ny, g.nx), device="cuda")
    x = torch.randn((2, g.ny, g.nx), device="cuda", generator=gen)
    sino = torch.empty((2, g.n_views, g.n_bins), device="cuda")
    ev = HipEvents()
    sp = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    dect.backproject(r, g, out=img)
    dect.project(x, g, out=sino)
    a0, a1, f0, f1 = ev.event(), ev.event(), ev.event(), ev.event()
    ev.record(a0, sp)
    for _ in range(k):
        dect.backproject(r, g, out=img)
    ev.record(a1, sp)
    ev.record(f0, sp)
    for _ in range(k):
        dect.project(x, g, out=sino)
    ev.record(f1, sp)
    torch.cuda.synchronize()
    S = dect.count_samples(g)
    M, N = g.n_views * g.n_bins, g.nx * g.ny
    print(json.dumps({"mode": "projectors", "launches": k, "samples": S,
                      "backproject_us": round(1e3 * ev.ms(a0, a1) / k, 2),
                      "project_us": round(1e3 * ev.ms(f0, f1) / k, 2),
                      "algorithmic_bytes_per_launch": 2 * (8 * S + 4 * M + 4 * N),
                      "kernel_hash": _counter_sources_hash()}), flush=True)


def copy_probe(mb: int, k: int):
    """Device copies of known size (read mb MiB, write mb MiB per launch)."""
    import torch
    n = mb * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(k):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "launches": k}), flush=True)


def _pmc_rows(path: str):
    import csv
    rows = list(csv.DictReader(open(path)))
    out = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
        cname = r.get("Counter_Name") or r.get("Counter-Name") or ""
        val = float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
        did = r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id") or ""
        out.setdefault((name, cname), {}).setdefault(did, 0.0)
        out[(name, cname)][did] += val
    return out


# Kernels of one ADM-TV iteration (and the bench's standalone projector
# launches) that the counter summary follows: label -> name test.
COUNTER_KERNELS = {
    "k_adj": lambda n: re.search(r"k_adj<", n) is not None,
    "k_adj_sum": lambda n: "k_adj_sum" in n,
    "k_fwd (ADM, residual fused)": lambda n: re.search(r"k_fwd<true", n) is not None,
    "k_fwd (plain)": lambda n: re.search(r"k_fwd<false", n) is not None,
    "k_tv_fused": lambda n: "k_tv_fused" in n,
    "k_scalar": lambda n: re.search(r"k_scalar\b", n) is not None and "k_scalar3" not in n,
    "k_update": lambda n: re.search(r"k_update\b", n) is not None,
}
SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES"]
# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a wave64 VALU instruction occupies a
# 16-lane SIMD for 4 cycles, so each CU issues at most one wave-level VALU
# instruction per cycle
VALU_PEAK_GINST = 256 * 2.4


def _counter_sources_hash() -> str:
    """Hash of the sources of the kernels the counter summary covers."""
    import hashlib
    h = hashlib.sha256()
    for name in ("projector.hip", "proj_device.h", "common.h", "adm.hip", "adm_device.h"):
        h.update(open(os.path.join(ROOT, "paper_1607_01650_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def counters_summary(pmc_dir: str):
    """Per-dispatch counters (median over the dispatches of each kernel) of
    the ADM-TV iteration's kernels from the counter runs under pmc_dir: sq/
    (SQ_COUNTERS), fetch/ and write/ (FETCH_SIZE, WRITE_SIZE), and the copy
    calibration (copy_fetch/, copy_write/, copy_meta.json).  HBM bytes are the
    counters scaled by what they read for a device copy of known size.
    Writes profiles/adm_tv_512x512_360v_counters.json and prints the table
    of profiles/adm_tv_512x512_360v_counters.md."""
    import glob
    import statistics

    def load(tag):
        files = glob.glob(os.path.join(pmc_dir, tag, "**", "*counter_collection.csv"),
                          recursive=True)
        if not files:
            raise SystemExit(f"no counter CSV under {pmc_dir}/{tag}")
        return _pmc_rows(files[0])

    def med(rows, match, counter):
        vals = []
        for (name, cname), d in rows.items():
            if cname == counter and match(name):
                vals += list(d.values())
        return (statistics.median(vals), len(vals)) if vals else (None, 0)

    meta = json.load(open(os.path.join(pmc_dir, "copy_meta.json")))
    is_copy = lambda n: "copy" in n.lower() or "elementwise" in n.lower()
    factor = {}
    for counter, tag, true_bytes in (("FETCH_SIZE", "copy_fetch", meta["bytes_read"]),
                                     ("WRITE_SIZE", "copy_write", meta["bytes_written"])):
        kib, _ = med(load(tag), is_copy, counter)
        factor[counter] = kib * 1024.0 / true_bytes
    sq, fetch, write = load("sq"), load("fetch"), load("write")
    kernels = {}
    for label, match in COUNTER_KERNELS.items():
        row = {}
        for c in SQ_COUNTERS:
            v, n = med(sq, match, c)
            row[c] = v
            row["dispatches"] = max(row.get("dispatches", 0), n)
        f, _ = med(fetch, match, "FETCH_SIZE")
        w, _ = med(write, match, "WRITE_SIZE")
        row["hbm_read_bytes"] = None if f is None else f * 1024.0 / factor["FETCH_SIZE"]
        row["hbm_write_bytes"] = None if w is None else w * 1024.0 / factor["WRITE_SIZE"]
        if row.get("SQ_WAVES"):
            row["valu_per_wave"] = row["SQ_INSTS_VALU"] / row["SQ_WAVES"]
            row["lds_per_wave"] = row["SQ_INSTS_LDS"] / row["SQ_WAVES"]
        kernels[label] = row
    out = {"kernel_hash": _counter_sources_hash(), "copy_factor": factor, "kernels": kernels,
           "pmc_dir": pmc_dir}
    base = os.path.join(ROOT, "profiles", "adm_tv_512x512_360v_counters")
    with open(base + ".json", "w") as fh:
        json.dump(out, fh, indent=1)
    lines = ["| kernel | dispatches | waves | VALU instr / wave | LDS instr / wave | VALU instr "
             "per dispatch | HBM read MB | HBM write MB |", "|---|---|---|---|---|---|---|---|"]
    for label, r in kernels.items():
        if not r.get("SQ_WAVES"):
            continue
        lines.append(f"| `{label}` | {r['dispatches']} | {r['SQ_WAVES']:.0f} | "
                     f"{r['valu_per_wave']:.0f} | {r['lds_per_wave']:.0f} | "
                     f"{r['SQ_INSTS_VALU']:.4g} | "
                     f"{(r['hbm_read_bytes'] or 0) / 1e6:.1f} | "
                     f"{(r['hbm_write_bytes'] or 0) / 1e6:.1f} |")
    print("\n".join(lines), flush=True)



if __name__ == "__main__":
    main()
