"""ctypes front-end of the FP64 CPU oracle (dect_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package's smoke
check and by the benchmark's CPU-baseline leg, never by the GPU library or its
Python binding.  It shares no code with them; geometry is passed as plain
numbers following the same written conventions (image centred on the
isocentre, theta_v = 2 pi v / V, flat centred detector, sinogram [V][B]).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dect_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Geom(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("pixel", ct.c_double),
                ("n_views", ct.c_int32), ("angles", ct.POINTER(ct.c_double)),
                ("n_bins", ct.c_int32), ("bin", ct.c_double), ("det_offset", ct.c_double),
                ("sod", ct.c_double), ("sdd", ct.c_double), ("model", ct.c_int32)]


class _Geom3(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("voxel", ct.c_double), ("n_views", ct.c_int32),
                ("angles", ct.POINTER(ct.c_double)), ("n_bins", ct.c_int32),
                ("n_rows", ct.c_int32), ("bin", ct.c_double), ("row", ct.c_double),
                ("det_offset", ct.c_double), ("sod", ct.c_double), ("sdd", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        P = ct.POINTER
        d, i32, sz = ct.c_double, ct.c_int32, ct.c_size_t
        pd = P(ct.c_double)
        pf = P(ct.c_float)
        L.or_num_threads.restype = ct.c_int
        L.or_count_samples.argtypes = [P(_Geom)]
        L.or_count_samples.restype = ct.c_int64
        L.or_project.argtypes = [P(_Geom), pd, pd]
        L.or_backproject.argtypes = [P(_Geom), pd, pd]
        L.or_fbp.argtypes = [P(_Geom), pd, pd]
        L.or_grad.argtypes = [ct.c_int, ct.c_int, pd, pd, pd]
        L.or_gradT.argtypes = [ct.c_int, ct.c_int, pd, pd, pd]
        L.or_shrink.argtypes = [sz, pd, pd, d, pd, pd]
        L.or_tv.argtypes = [ct.c_int, ct.c_int, pd]
        L.or_tv.restype = d
        L.or_adm.argtypes = [P(_Geom), pd, d, d, d, d, ct.c_int, d, pd, pd, pd, pd, pd, ct.c_int,
                             ct.c_int]
        L.or_adm.restype = ct.c_int
        L.or_dinv.argtypes = [sz, d, d, d, d, pd, pd, pd, pd]
        L.or_edges.argtypes = [ct.c_int, ct.c_int, pd, d, d, pd, pd, P(ct.c_uint8), pd, pd]
        L.or_laplacian.argtypes = [ct.c_int, ct.c_int, pd, pd, pd, pd]
        L.or_pcg.argtypes = [ct.c_int, ct.c_int, pd, pd, d, pd, pd, ct.c_int, d, pd]
        L.or_pcg.restype = ct.c_int
        L.or_pcg_att.argtypes = [ct.c_int, ct.c_int, pd, pd, d, d, d, d, d, pd, pd, pd, pd,
                                 ct.c_int, d, pd]
        L.or_pcg_att.restype = ct.c_int
        L.or_adm_coupled.argtypes = [P(_Geom), pd, pd, d, d, d, ct.c_int, pd, pd, pd, ct.c_int]
        L.or_project3.argtypes = [P(_Geom3), pd, pd]
        L.or_backproject3.argtypes = [P(_Geom3), pd, pd]
        L.or_adm3.argtypes = [P(_Geom3), pd, d, d, d, d, ct.c_int, d, pd, pd, pd, ct.c_int,
                              ct.c_int]
        L.or_edges3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, d, d, pd, pd, pd,
                                P(ct.c_uint8), pd, pd]
        L.or_laplacian3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, pd, pd, pd, pd]
        L.or_pcg3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, pd, pd, d, pd, pd, ct.c_int, d,
                              pd]
        L.or_pcg3.restype = ct.c_int
        L.or_pcg_att3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, pd, pd, d, d, d, d, d, pd,
                                  pd, pd, pd, ct.c_int, d, pd]
        L.or_pcg_att3.restype = ct.c_int
        L.or_adm3_coupled.argtypes = [P(_Geom3), pd, pd, d, d, d, ct.c_int, pd, pd, pd,
                                      ct.c_int]
        L.or_adm3.restype = ct.c_int
        L.or_grad3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, pd]
        L.or_gradT3.argtypes = [ct.c_int, ct.c_int, ct.c_int, pd, pd]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def _p(a: Optional[np.ndarray], ctype=ct.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ct.POINTER(ctype))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OGeom:
    """Geometry in the oracle's own struct; keeps the angle array alive."""

    def __init__(self, nx, ny, pixel_mm, n_views, n_bins, bin_mm, sod_mm, sdd_mm,
                 det_offset_mm=0.0, angles_rad: Optional[Sequence[float]] = None,
                 model: int = 0):
        self.nx, self.ny, self.n_views, self.n_bins = int(nx), int(ny), int(n_views), int(n_bins)
        self._angles = None if angles_rad is None else _f64(angles_rad)
        self.s = _Geom(self.nx, self.ny, float(pixel_mm), self.n_views,
                       _p(self._angles), self.n_bins, float(bin_mm), float(det_offset_mm),
                       float(sod_mm), float(sdd_mm), int(model))

    @classmethod
    def of(cls, g) -> "OGeom":
        """From any object with the Geometry field names (model: 0 Joseph,
        1 Siddon; absent means Joseph)."""
        return cls(g.nx, g.ny, g.pixel_mm, g.n_views, g.n_bins, g.bin_mm, g.sod_mm, g.sdd_mm,
                   g.det_offset_mm, g.angles_rad, getattr(g, "model", 0))


def _og(g) -> OGeom:
    return g if isinstance(g, OGeom) else OGeom.of(g)


def count_samples(g) -> int:
    og = _og(g)
    return int(lib().or_count_samples(ct.byref(og.s)))


def project(g, img: np.ndarray) -> np.ndarray:
    og = _og(g)
    x = _f64(img).reshape(og.ny, og.nx)
    out = np.empty((og.n_views, og.n_bins))
    lib().or_project(ct.byref(og.s), _p(x), _p(out))
    return out


def backproject(g, sino: np.ndarray) -> np.ndarray:
    og = _og(g)
    y = _f64(sino).reshape(og.n_views, og.n_bins)
    out = np.empty((og.ny, og.nx))
    lib().or_backproject(ct.byref(og.s), _p(y), _p(out))
    return out


def fbp(g, sino: np.ndarray) -> np.ndarray:
    """Fan-beam filtered back-projection (full turn, ramp filter)."""
    og = _og(g)
    y = _f64(sino).reshape(og.n_views, og.n_bins)
    out = np.empty((og.ny, og.nx))
    lib().or_fbp(ct.byref(og.s), _p(y), _p(out))
    return out


class OGeom3:
    """Cone-beam geometry in the oracle's struct (any object with the
    ConeGeometry field names)."""

    def __init__(self, g):
        self.nx, self.ny, self.nz = int(g.nx), int(g.ny), int(g.nz)
        self.n_views, self.n_bins, self.n_rows = int(g.n_views), int(g.n_bins), int(g.n_rows)
        self._angles = None if g.angles_rad is None else _f64(g.angles_rad)
        self.s = _Geom3(self.nx, self.ny, self.nz, float(g.voxel_mm), self.n_views,
                        _p(self._angles), self.n_bins, self.n_rows, float(g.bin_mm),
                        float(g.row_mm), float(g.det_offset_mm), float(g.sod_mm),
                        float(g.sdd_mm))


def project3(g, vol: np.ndarray) -> np.ndarray:
    """Cone-beam Joseph projection of vol [nz][ny][nx] -> [V][rows][bins]."""
    og = OGeom3(g)
    x = _f64(vol).reshape(og.nz, og.ny, og.nx)
    out = np.empty((og.n_views, og.n_rows, og.n_bins))
    lib().or_project3(ct.byref(og.s), _p(x), _p(out))
    return out


def backproject3(g, proj: np.ndarray) -> np.ndarray:
    og = OGeom3(g)
    y = _f64(proj).reshape(og.n_views, og.n_rows, og.n_bins)
    out = np.empty((og.nz, og.ny, og.nx))
    lib().or_backproject3(ct.byref(og.s), _p(y), _p(out))
    return out


def adm3(g, m: np.ndarray, beta: float, mu: float, rho: float, xi: float, iters: int,
         tol: float = 0.0, x0: Optional[np.ndarray] = None, with_iters: bool = False,
         nonneg: bool = False, step: str = "bb1"):
    """ADM-TV (Eq. 10) of one energy on a volume with the cone-beam pair and
    the 3-D TV, from zero or from x0 (f = beta x0), stopping early when the
    relative image change falls below tol; nonneg and step as in adm().
    Returns (x = f / beta [nz][ny][nx], log [(iters+1)][5]) and, with
    with_iters, the iteration count."""
    og = OGeom3(g)
    mm = _f64(m).reshape(og.n_views, og.n_rows, og.n_bins)
    x = np.empty((og.nz, og.ny, og.nx))
    log = np.zeros((iters + 1, 5))
    x0c = None if x0 is None else _f64(x0).reshape(og.nz, og.ny, og.nx)
    k = lib().or_adm3(ct.byref(og.s), _p(mm), float(beta), float(mu), float(rho), float(xi),
                      int(iters), float(tol), _p(x0c), _p(x), _p(log), 1 if nonneg else 0,
                      {"bb1": 0, "bb2": 1, "abb": 2}[step])
    if with_iters:
        return x, log, int(k)
    return x, log


def grad3(x: np.ndarray) -> np.ndarray:
    """Backward differences along x, y, z of a volume: [3][nz][ny][nx]."""
    x = _f64(x)
    nz, ny, nx = x.shape
    out = np.empty((3, nz, ny, nx))
    lib().or_grad3(nx, ny, nz, _p(x), _p(out))
    return out


def gradT3(p3: np.ndarray) -> np.ndarray:
    p3 = _f64(p3)
    _, nz, ny, nx = p3.shape
    out = np.empty((nz, ny, nx))
    lib().or_gradT3(nx, ny, nz, _p(p3), _p(out))
    return out


def grad(x: np.ndarray):
    x = _f64(x)
    ny, nx = x.shape
    gx, gy = np.empty_like(x), np.empty_like(x)
    lib().or_grad(nx, ny, _p(x), _p(gx), _p(gy))
    return gx, gy


def gradT(px: np.ndarray, py: np.ndarray) -> np.ndarray:
    px, py = _f64(px), _f64(py)
    ny, nx = px.shape
    out = np.empty_like(px)
    lib().or_gradT(nx, ny, _p(px), _p(py), _p(out))
    return out


def shrink(vx, vy, t: float):
    vx, vy = _f64(vx), _f64(vy)
    zx, zy = np.empty_like(vx), np.empty_like(vy)
    lib().or_shrink(vx.size, _p(vx), _p(vy), float(t), _p(zx), _p(zy))
    return zx, zy


def tv(x) -> float:
    x = _f64(x)
    return float(lib().or_tv(x.shape[1], x.shape[0], _p(x)))


class AdmResult:
    def __init__(self, x, lam, z, log, iters):
        self.x, self.lam, self.z, self.log, self.iters = x, lam, z, log, iters

    @property
    def J(self):
        return self.log[: self.iters + 1, 0]

    @property
    def alpha(self):
        return self.log[: self.iters + 1, 1]


def adm(g, m: np.ndarray, beta: float, mu: float, rho: float, xi: float, iters: int,
        tol: float = 0.0, x0: Optional[np.ndarray] = None, nonneg: bool = False,
        step: str = "bb1") -> AdmResult:
    """ADM-TV (Eq. 10) for one energy; returns x = f / beta and the log.
    nonneg: project every f-step onto f >= 0.  step: "bb1", "bb2" or "abb"
    (adaptive: BB2 where BB2/BB1 < 1/2, else BB1)."""
    og = _og(g)
    mm = _f64(m).reshape(og.n_views, og.n_bins)
    x0c = None if x0 is None else _f64(x0).reshape(og.ny, og.nx)
    x = np.empty((og.ny, og.nx))
    lam = np.empty((2, og.ny, og.nx))
    z = np.empty((2, og.ny, og.nx))
    log = np.zeros((iters + 1, 5))
    k = lib().or_adm(ct.byref(og.s), _p(mm), float(beta), float(mu), float(rho), float(xi),
                     int(iters), float(tol), _p(x0c), _p(x), _p(lam), _p(z), _p(log),
                     1 if nonneg else 0, {"bb1": 0, "bb2": 1, "abb": 2}[step])
    return AdmResult(x, lam, z, log, int(k))


def adm_coupled(g, m_high, m_low, beta_high: float, beta_low: float, mu: float, rho: float,
                xi: float, iters: int, x0=None, nonneg: bool = False):
    """ADM-TV of both energies with the TV coupled across them (joint z-step).
    Returns (x [2][ny][nx], J [iters+1][2], alpha [iters+1][2]); energy 0's J
    column carries the joint TV, so the columns sum to the objective."""
    og = _og(g)
    m = np.ascontiguousarray(np.stack([_f64(m_high).reshape(og.n_views, og.n_bins),
                                       _f64(m_low).reshape(og.n_views, og.n_bins)]))
    beta = np.array([beta_high, beta_low], dtype=np.float64)
    x0c = None if x0 is None else np.ascontiguousarray(np.stack([_f64(x0[0]), _f64(x0[1])]))
    x = np.empty((2, og.ny, og.nx))
    log = np.zeros((2, iters + 1, 2))
    lib().or_adm_coupled(ct.byref(og.s), _p(m), _p(beta), float(mu), float(rho), float(xi),
                         int(iters), _p(x0c), _p(x), _p(log), 1 if nonneg else 0)
    return x, log[:, :, 0].T.copy(), log[:, :, 1].T.copy()


def dinv(xh, xl, eta_water_high, eta_bone_high, eta_water_low, eta_bone_low):
    xh, xl = _f64(xh), _f64(xl)
    u1, u2 = np.empty_like(xh), np.empty_like(xh)
    lib().or_dinv(xh.size, eta_water_high, eta_bone_high, eta_water_low, eta_bone_low,
                  _p(xh), _p(xl), _p(u1), _p(u2))
    return u1, u2


class EdgeMap:
    """Edge weights of the penalty and what decided them (FP64): pair weights,
    the edge flags, m2 = |Prewitt gradient|^2 per pixel and the threshold
    tau^2 max(m2)."""

    def __init__(self, weights, edge, m2, thr):
        self.weights, self.edge, self.m2, self.thr = weights, edge, m2, thr

    def near_threshold(self, rel: float) -> np.ndarray:
        """Pixels whose m2 lies within rel * thr of the threshold, where an
        evaluation in another precision may decide the other way."""
        return np.abs(self.m2 - self.thr) <= rel * self.thr


def edges(xl: np.ndarray, tau: float, eps: float) -> EdgeMap:
    """Prewitt edge weights of an image [ny][nx] in FP64: weights (e_right,
    e_down)."""
    x = _f64(xl)
    ny, nx = x.shape
    er, ed, m2 = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    e = np.empty(x.shape, dtype=np.uint8)
    thr = ct.c_double(0.0)
    lib().or_edges(nx, ny, _p(x), float(tau), float(eps), _p(er), _p(ed),
                   e.ctypes.data_as(ct.POINTER(ct.c_uint8)), _p(m2), ct.byref(thr))
    return EdgeMap((er, ed), e, m2, float(thr.value))


def laplacian(er, ed, u):
    er, ed, u = _f64(er), _f64(ed), _f64(u)
    ny, nx = u.shape
    out = np.empty_like(u)
    lib().or_laplacian(nx, ny, _p(er), _p(ed), _p(u), _p(out))
    return out


def pcg(er, ed, gamma: float, b, max_iter: int = 500, tol: float = 1e-12):
    er, ed, b = _f64(er), _f64(ed), _f64(b)
    ny, nx = b.shape
    u = np.empty_like(b)
    rr = ct.c_double(0.0)
    it = lib().or_pcg(nx, ny, _p(er), _p(ed), float(gamma), _p(b), _p(u), int(max_iter),
                      float(tol), ct.byref(rr))
    return u, int(it), float(rr.value)


def pcg_att(er, ed, eta, gamma: float, xh, xl, max_iter: int = 500, tol: float = 1e-12):
    """Attenuation-space PLS system (D^T D + gamma L) u = D^T x, both materials
    coupled; eta = (eta_water_high, eta_bone_high, eta_water_low, eta_bone_low)."""
    er, ed, xh, xl = _f64(er), _f64(ed), _f64(xh), _f64(xl)
    ny, nx = xh.shape
    u1, u2 = np.empty_like(xh), np.empty_like(xh)
    rr = ct.c_double(0.0)
    it = lib().or_pcg_att(nx, ny, _p(er), _p(ed), *[float(e) for e in eta], float(gamma),
                          _p(xh), _p(xl), _p(u1), _p(u2), int(max_iter), float(tol),
                          ct.byref(rr))
    return u1, u2, int(it), float(rr.value)


def edges3(xl: np.ndarray, tau: float, eps: float) -> EdgeMap:
    """3-D Prewitt edge weights of a volume [nz][ny][nx] in FP64: weights
    (e_x, e_y, e_z)."""
    x = _f64(xl)
    nz, ny, nx = x.shape
    ex, ey, ez, m2 = np.empty_like(x), np.empty_like(x), np.empty_like(x), np.empty_like(x)
    e = np.empty(x.shape, dtype=np.uint8)
    thr = ct.c_double(0.0)
    lib().or_edges3(nx, ny, nz, _p(x), float(tau), float(eps), _p(ex), _p(ey), _p(ez),
                    e.ctypes.data_as(ct.POINTER(ct.c_uint8)), _p(m2), ct.byref(thr))
    return EdgeMap((ex, ey, ez), e, m2, float(thr.value))


def laplacian3(ex, ey, ez, u):
    ex, ey, ez, u = _f64(ex), _f64(ey), _f64(ez), _f64(u)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    lib().or_laplacian3(nx, ny, nz, _p(ex), _p(ey), _p(ez), _p(u), _p(out))
    return out


def pcg3(ex, ey, ez, gamma: float, b, max_iter: int = 500, tol: float = 1e-12):
    ex, ey, ez, b = _f64(ex), _f64(ey), _f64(ez), _f64(b)
    nz, ny, nx = b.shape
    u = np.empty_like(b)
    rr = ct.c_double(0.0)
    it = lib().or_pcg3(nx, ny, nz, _p(ex), _p(ey), _p(ez), float(gamma), _p(b), _p(u),
                       int(max_iter), float(tol), ct.byref(rr))
    return u, int(it), float(rr.value)


def adm3_coupled(g, m_high, m_low, beta_high: float, beta_low: float, mu: float, rho: float,
                 xi: float, iters: int, x0=None, nonneg: bool = False):
    """ADM-TV of both energies on a volume with the 3-D TV coupled across them
    (joint z-step over the 6-vector).  Returns (x [2][nz][ny][nx], J
    [iters+1][2], alpha [iters+1][2]); energy 0's J column carries the joint
    TV."""
    og = OGeom3(g)
    shp = (og.n_views, og.n_rows, og.n_bins)
    m = np.ascontiguousarray(np.stack([_f64(m_high).reshape(shp), _f64(m_low).reshape(shp)]))
    beta = np.array([beta_high, beta_low], dtype=np.float64)
    vshp = (og.nz, og.ny, og.nx)
    x0c = None if x0 is None else np.ascontiguousarray(
        np.stack([_f64(x0[0]).reshape(vshp), _f64(x0[1]).reshape(vshp)]))
    x = np.empty((2,) + vshp)
    log = np.zeros((2, iters + 1, 2))
    lib().or_adm3_coupled(ct.byref(og.s), _p(m), _p(beta), float(mu), float(rho), float(xi),
                          int(iters), _p(x0c), _p(x), _p(log), 1 if nonneg else 0)
    return x, log[:, :, 0].T.copy(), log[:, :, 1].T.copy()


def pcg_att3(ex, ey, ez, eta, gamma: float, xh, xl, max_iter: int = 500, tol: float = 1e-12):
    """Attenuation-space PLS system on a volume [nz][ny][nx] with the
    six-neighbour L, both materials coupled; returns (u1, u2, iters, relres)."""
    ex, ey, ez, xh, xl = _f64(ex), _f64(ey), _f64(ez), _f64(xh), _f64(xl)
    nz, ny, nx = xh.shape
    u1, u2 = np.empty_like(xh), np.empty_like(xh)
    rr = ct.c_double(0.0)
    it = lib().or_pcg_att3(nx, ny, nz, _p(ex), _p(ey), _p(ez), *[float(e) for e in eta],
                           float(gamma), _p(xh), _p(xl), _p(u1), _p(u2), int(max_iter),
                           float(tol), ct.byref(rr))
    return u1, u2, int(it), float(rr.value)


def pls3(xh, xl, p, tol: float = 1e-12, edge_w=None):
    """3-D decomposition of volumes [nz][ny][nx]: D^{-1} x per voxel, 3-D
    Prewitt edge weights on x_l (or the given [3][nz][ny][nx] map), then PCG
    per material with the six-neighbour L (image mode) or the coupled
    attenuation-space system (p.mode == 1)."""
    if edge_w is None:
        ex, ey, ez = edges3(xl, p.edge_tau, p.edge_eps).weights
    else:
        ex, ey, ez = edge_w[0], edge_w[1], edge_w[2]
    if getattr(p, "mode", 0) == 1:
        eta = (p.eta_water_high, p.eta_bone_high, p.eta_water_low, p.eta_bone_low)
        u1, u2, it, _ = pcg_att3(ex, ey, ez, eta, p.gamma, xh, xl, p.max_iter, tol)
        return u1, u2, it
    b1, b2 = dinv(xh, xl, p.eta_water_high, p.eta_bone_high, p.eta_water_low, p.eta_bone_low)
    u1, i1, _ = pcg3(ex, ey, ez, p.gamma, b1, p.max_iter, tol)
    u2, i2, _ = pcg3(ex, ey, ez, p.gamma, b2, p.max_iter, tol)
    return u1, u2, max(i1, i2)


def pls(xh, xl, p, edge_w=None, tol: float = 1e-12):
    """Full decomposition: D^{-1} x, edge weights on x_l (FP32 decision), PCG.

    p carries eta_*, gamma, edge_eps, edge_tau, max_iter.  edge_w, when given,
    is a shared [2][ny][nx] (right, down) weight map.
    """
    b1, b2 = dinv(xh, xl, p.eta_water_high, p.eta_bone_high, p.eta_water_low, p.eta_bone_low)
    if edge_w is None:
        er, ed = edges(xl, p.edge_tau, p.edge_eps).weights
    else:
        er, ed = edge_w[0], edge_w[1]
    if getattr(p, "mode", 0) == 1:  # attenuation space
        eta = (p.eta_water_high, p.eta_bone_high, p.eta_water_low, p.eta_bone_low)
        u1, u2, it, r = pcg_att(er, ed, eta, p.gamma, xh, xl, p.max_iter, tol)
        return u1, u2, (it, it), (r, r)
    u1, it1, r1 = pcg(er, ed, p.gamma, b1, p.max_iter, tol)
    u2, it2, r2 = pcg(er, ed, p.gamma, b2, p.max_iter, tol)
    return u1, u2, (it1, it2), (r1, r2)
