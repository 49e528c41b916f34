"""Write the stored oracle results used by the paper-scale GPU parity tests.

Calls only the FP64 oracle (oracle/) on the seeded synthetic inputs of the
paper-scale workloads (512x512, 90, 360 and 720 views over 360 degrees, 736 bins,
both energies, 200 ADM-TV iterations) and stores the images as float32 plus
the per-iteration objective.  Run from the repository root:
    python tests/golden/make_golden.py [90] [720] [siddon] [nonneg]
("siddon": the same runs on the Siddon ray model, files *_siddon.npz;
"nonneg": with every f-step projected onto f >= 0, files *_nonneg.npz.)
"""
import dataclasses
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1607_01650_amd import configs as C, phantom as P  # noqa: E402

ITERS = 200


def main(views, model=0, nonneg=False):
    for V in views:
        g = dataclasses.replace(C.paper_geometry(512, V), model=model)
        s = P.make_slice(g, 0)
        p = C.default_adm_params(g, ITERS)
        xs, Js = [], []
        for e, beta in ((0, p.beta_high), (1, p.beta_low)):
            t = time.time()
            m = np.asarray(s.sino[e], dtype=np.float32).astype(np.float64)
            r = O.adm(g, m, beta, p.mu, p.rho, p.xi, ITERS, nonneg=nonneg)
            xs.append(r.x.astype(np.float32))
            Js.append(r.J)
            print(f"V={V} energy {e}: {time.time() - t:.1f}s J0 {r.J[0]:.6g} J{ITERS} {r.J[-1]:.6g}",
                  flush=True)
        tag = ("_siddon" if model == 1 else "") + ("_nonneg" if nonneg else "")
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           f"adm512_v{V}_k{ITERS}{tag}.npz")
        np.savez_compressed(out, x=np.stack(xs), J=np.stack(Js), mu=p.mu, rho=p.rho, xi=p.xi,
                            beta=np.array([p.beta_high, p.beta_low]), iters=ITERS, seed=0)
        print("wrote", out, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    model = 1 if "siddon" in args else 0
    nonneg = "nonneg" in args
    main([int(a) for a in args if a not in ("siddon", "nonneg")] or [90, 360, 720], model, nonneg)
