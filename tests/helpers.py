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
