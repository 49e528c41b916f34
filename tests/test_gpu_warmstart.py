"""Learned warm start on a held-out case (512x512, 90 views, both energies).

The U-Net weights in paper_1607_01650_amd/weights/ were trained by this
project's own BF16 MFMA kernels on phantoms 0-1999 (python -m
paper_1607_01650_amd.warmstart).  The case here is slice 2000 of the shared
input generator (analytic sinograms plus noise), which the training never saw.

Checked:
* ADM continued from the network output reaches the plain method's objective
  J_ref = J(plain f^200) in fewer iterations and less wall time than plain ADM;
* the fallback: a network output made non-finite, or one whose objective
  exceeds J(f^5), is not used; the plain run resumes at f^5 and ends bit for
  bit where plain ADM ends;
* the FP64 oracle's 200-iteration image of the same case: the GPU's plain
  f^200 is within 1e-4 of it, and
  the learned result is as close to the true phantom as the plain one
  (within 10 %), since both stop at the same objective value.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import need_gpu, rel_l2, to_np

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1607_01650_amd", "weights", "unet_warmstart_512_90v.npz")


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def test_warm_start_reaches_plain_objective_sooner(torch):
    from paper_1607_01650_amd import nn as NN
    from paper_1607_01650_amd import warmstart as W
    geom = C.paper_geometry(512, 90)
    s = P.make_slice(geom, W.EVAL_SEED0)
    net = NN.UNet(seed=0)
    W.load_weights(net, WEIGHTS)
    sol = W.Solver(geom)
    sino = torch.as_tensor(np.asarray(s.sino, dtype=np.float32)).cuda()
    row = W.evaluate_case(net, sol, sino, reps=3)
    assert row["start"] == "net"
    it_learned = W.EARLY + row["k_cont"]
    print(f"plain: {row['k_plain']} its {row['t_plain_ms']:.1f} ms; learned: {it_learned} its "
          f"{row['t_learned_ms']:.1f} ms (network start {row['t_start_ms']:.1f} ms); "
          f"J(net)/J_ref {row['J_start'] / row['J_ref']:.3f}", flush=True)
    assert row["k_cont"] >= 0
    assert it_learned < row["k_plain"]
    assert row["t_learned_ms"] < row["t_plain_ms"]

    sol.load(sino)
    sol.run(W.LATE)
    plain200 = to_np(sol.x)
    learned = to_np(row["learned_img"])
    p = C.default_adm_params(geom, W.LATE)
    for e, beta in ((0, p.beta_high), (1, p.beta_low)):
        m = np.asarray(s.sino[e], dtype=np.float32).astype(np.float64)
        ref = O.adm(geom, m, beta, p.mu, p.rho, p.xi, W.LATE).x
        err_plain = rel_l2(plain200[e], ref)
        err_learned = rel_l2(learned[e], ref)
        truth = s.x_true[e]
        t_plain, t_learned = rel_l2(plain200[e], truth), rel_l2(learned[e], truth)
        print(f"energy {e}: vs FP64 oracle f^200: plain {err_plain:.2e}, learned "
              f"{err_learned:.2e}; vs true phantom: plain {t_plain:.4f}, learned "
              f"{t_learned:.4f}", flush=True)
        assert err_plain <= 1e-4
        assert t_learned <= 1.1 * t_plain


@pytest.fixture(scope="module")
def trained():
    from paper_1607_01650_amd import nn as NN
    from paper_1607_01650_amd import warmstart as W
    import torch as T
    geom = C.paper_geometry(512, 90)
    s = P.make_slice(geom, W.EVAL_SEED0 + 1)
    net = NN.UNet(seed=0)
    W.load_weights(net, WEIGHTS)
    sol = W.Solver(geom)
    sino = T.as_tensor(np.asarray(s.sino, dtype=np.float32)).cuda()
    return net, sol, sino


@pytest.mark.parametrize("how", ["nonfinite", "objective"])
def test_warm_start_falls_back_to_plain(torch, trained, how):
    """The network output is corrupted from the host before the start check:
    one NaN pixel, or a uniform offset of 0.05/mm (J far above J(f^5)).  The
    continuation must resume the plain run at f^5, so the learned path reaches
    J_ref after exactly the plain method's iterations and ends on its image,
    bit for bit."""
    from paper_1607_01650_amd import warmstart as W
    net, sol, sino = trained

    def corrupt(yh, yl):
        if how == "nonfinite":
            yh[0, 200, 300] = float("nan")
        else:
            yh.add_(0.05)
            yl.add_(0.05)

    row = W.evaluate_case(net, sol, sino, reps=1, corrupt=corrupt)
    print(f"{how}: start {row['start']}, k_plain {row['k_plain']}, k_cont {row['k_cont']}, "
          f"t_plain {row['t_plain_ms']:.1f} ms, t_learned {row['t_learned_ms']:.1f} ms", flush=True)
    assert row["start"] == how
    assert row["k_cont"] == row["k_plain"] - W.EARLY
    assert torch.equal(row["learned_img"], row["plain_img"])
    # the uncorrupted network is used on the same case
    ok = W.evaluate_case(net, sol, sino, reps=1)
    assert ok["start"] == "net" and ok["k_cont"] + W.EARLY < ok["k_plain"]
