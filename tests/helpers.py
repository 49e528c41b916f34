"""Small shared test utilities (no method arithmetic)."""
import numpy as np
import pytest


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU")
    return torch


def to_dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    """The float32 values a GPU run sees, as float64 for the oracle."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def edge_weights_agree(w_gpu, em, rel: float = 1e-4):
    """Compare the GPU's pair weights with the FP64 oracle's edge map `em`.

    The edge map is a threshold decision on |Prewitt gradient|^2: the GPU
    takes it in FP32, the oracle in FP64, so the two may decide differently
    only at pixels whose m2 lies within a relative `rel` of the threshold.
    Every pair weight that touches no such pixel must be equal (as float32).
    w_gpu: [ndim][...] weights, axis k coupling neighbours along the k-th
    last array axis.  Returns (pairs that differ, pixels near the threshold)."""
    w_gpu = np.asarray(w_gpu)
    near = em.near_threshold(rel)
    ndim = near.ndim
    differ = 0
    for k, w_or in enumerate(em.weights):
        ax = ndim - 1 - k
        touch = near.copy()
        sl_dst = [slice(None)] * ndim
        sl_src = [slice(None)] * ndim
        sl_dst[ax] = slice(0, near.shape[ax] - 1)
        sl_src[ax] = slice(1, None)
        touch[tuple(sl_dst)] |= near[tuple(sl_src)]
        d = np.asarray(w_gpu[k], dtype=np.float32) != np.asarray(w_or, dtype=np.float32)
        assert not np.any(d & ~touch), f"axis {k}: pair weights differ away from the threshold"
        differ += int(d.sum())
    return differ, int(near.sum())
