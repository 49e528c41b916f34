"""FP64 oracle of the unrolled ADM-TV steps (TEST INFRASTRUCTURE ONLY).

One step per given parameter set (mu_k, rho_k, xi_k, alpha_k), in the order of
the reconstruction procedure (Eq. 10) with a fixed step alpha_k in place of
the BB step: z-shrinkage (Eq. 8), the f-gradient of Eq. 9, the f step and the
multiplier step of Eq. 7.  Built from the C oracle's projector and finite
differences.
"""
import numpy as np

from . import oracle as O


def step(g_geom, g_data, f, lx, ly, mu, rho, xi, alpha):
    """One step from (f, lambda): returns (f', lambda_x', lambda_y')."""
    h = mu * O.backproject(g_geom, O.project(g_geom, f) - g_data)
    dx, dy = O.grad(f)
    zx, zy = O.shrink(dx - lx / rho, dy - ly / rho, 1.0 / rho)
    G = h + O.gradT(rho * (dx - zx) - lx, rho * (dy - zy) - ly)
    f = f - alpha * G
    nx_, ny_ = O.grad(f)
    return f, lx - xi * (nx_ - zx), ly - xi * (ny_ - zy)


def unrolled(g_geom, g_data, params, f0=None):
    """params: sequence of (mu, rho, xi, alpha); g_data [V][B] (beta-scaled)."""
    ny, nx = g_geom.ny, g_geom.nx
    f = np.zeros((ny, nx)) if f0 is None else np.array(f0, dtype=np.float64)
    lx = np.zeros((ny, nx))
    ly = np.zeros((ny, nx))
    for (mu, rho, xi, alpha) in params:
        f, lx, ly = step(g_geom, g_data, f, lx, ly, mu, rho, xi, alpha)
    return f
