"""GPU parity of the cone-beam Joseph projector pair (dect_cone_project /
dect_cone_backproject) against the FP64 oracle's pair (the 3-D scanner of
Sec. 3, Joseph's model of Sec. 2.4 with bilinear taps in the driving plane).

* ragged volumes (several 64-bin wavefronts plus a tail, odd slice and row
  counts, detector offset, irregular view angles, and views at multiples of
  45 degrees whose central rays lie on the x-major / y-major boundary): forward and back
  projection within 1e-5 of the oracle's largest value.  The GPU steps each
  ray's in-plane coordinate and height in 32.32 fixed point and interpolates
  in FP32 (summed in FP64 per four planes); the gather back-projection
  uses the same in-plane coordinate, the height in FP64, per-view FP32 sums
  accumulated in FP64;
* the 512 x 512 x 64 volume, 360 views, 64 x 736 detector: eight views
  against the oracle run on those views alone, and the adjoint identity of
  the GPU pair at full size;
* the central row of an odd-row detector equals the fan-beam GPU projector
  of the central slice; repeated forward and back-projection calls agree
  bit for bit;
* geometries the kernels do not support are refused.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

RAGGED = C.ConeGeometry(nx=64, ny=56, nz=33, voxel_mm=1.0, n_views=40, n_bins=97, n_rows=17,
                        bin_mm=1.4, row_mm=1.6, sod_mm=150.0, sdd_mm=300.0, det_offset_mm=0.6)
SMALL = C.ConeGeometry(nx=40, ny=36, nz=21, voxel_mm=1.0, n_views=24, n_bins=70, n_rows=9,
                       bin_mm=1.3, row_mm=1.1, sod_mm=150.0, sdd_mm=300.0, det_offset_mm=0.4)
# views at multiples of 45 degrees with an odd bin count and no offset: the
# central ray of the diagonal views lies on the x-major / y-major boundary
DIAG = C.ConeGeometry(nx=33, ny=33, nz=9, voxel_mm=1.0, n_views=8, n_bins=61, n_rows=5,
                      bin_mm=1.2, row_mm=1.3, sod_mm=120.0, sdd_mm=240.0)
IRREG = dataclasses.replace(
    SMALL, n_views=17,
    angles_rad=tuple(0.37 * v + 0.05 * math.sin(3.0 * v) for v in range(17)))


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _dect():
    from paper_1607_01650_amd import dect
    return dect


def _maxrel(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("geom", [RAGGED, SMALL, IRREG, DIAG],
                         ids=["ragged", "small", "irregular", "diagonal"])
def test_pair_parity(torch, geom):
    dect = _dect()
    rng = np.random.default_rng(5)
    vol = f32(rng.random((geom.nz, geom.ny, geom.nx)))
    y = f32(rng.random((geom.n_views, geom.n_rows, geom.n_bins)))
    p = to_np(dect.cone_project(to_dev(torch, vol), geom))
    b = to_np(dect.cone_backproject(to_dev(torch, y), geom))
    ef, eb = _maxrel(p, O.project3(geom, vol)), _maxrel(b, O.backproject3(geom, y))
    print(f"cone {geom.nx}x{geom.ny}x{geom.nz} V={geom.n_views}: forward max rel err "
          f"{ef:.2e}, back max rel err {eb:.2e}", flush=True)
    assert ef <= 1e-5 and eb <= 1e-5


def test_phantom_parity(torch):
    dect = _dect()
    g = RAGGED
    vol = f32(P.cone_volume(g, 3, supersample=2))
    p = to_np(dect.cone_project(to_dev(torch, vol), g))
    assert _maxrel(p, O.project3(g, vol)) <= 1e-5
    b = to_np(dect.cone_backproject(to_dev(torch, p.astype(np.float32)), g))
    assert _maxrel(b, O.backproject3(g, f32(p))) <= 1e-5


def test_full_size_sampled_views_and_adjoint(torch):
    dect = _dect()
    g = C.CONE
    vol = f32(P.cone_volume(g, 0, supersample=2))
    p = dect.cone_project(to_dev(torch, vol), g)
    torch.cuda.synchronize()
    views = [0, 45, 90, 133, 180, 222, 300, 359]
    th = [2.0 * math.pi * v / g.n_views for v in views]
    gs = dataclasses.replace(g, n_views=len(views), angles_rad=tuple(th))
    ref = O.project3(gs, vol)
    err = _maxrel(to_np(p)[views], ref)
    print(f"cone 512x512x64 V=360: sampled-view forward max rel err {err:.2e}", flush=True)
    assert err <= 1e-5
    rng = np.random.default_rng(9)
    y = torch.as_tensor(rng.random((g.n_views, g.n_rows, g.n_bins), dtype=np.float32)).cuda()
    x = to_dev(torch, rng.random((g.nz, g.ny, g.nx)))
    ax = dect.cone_project(x, g)
    aty = dect.cone_backproject(y, g)
    lhs = float(torch.sum(ax.double() * y.double()))
    rhs = float(torch.sum(x.double() * aty.double()))
    print(f"cone 512x512x64 V=360: adjoint identity rel gap {abs(lhs - rhs) / abs(lhs):.2e}",
          flush=True)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_central_row_equals_fan_beam(torch):
    dect = _dect()
    g = RAGGED
    rng = np.random.default_rng(2)
    vol = rng.random((g.nz, g.ny, g.nx)).astype(np.float32)
    p3 = to_np(dect.cone_project(to_dev(torch, vol), g))
    p2 = to_np(dect.project(to_dev(torch, vol[g.nz // 2]), g.central_plane()))
    assert _maxrel(p3[:, g.n_rows // 2, :], p2) <= 1e-5
    again = to_np(dect.cone_project(to_dev(torch, vol), g))
    assert np.array_equal(p3, again)
    y = to_dev(torch, p3)
    b1 = to_np(dect.cone_backproject(y, g))
    assert np.array_equal(b1, to_np(dect.cone_backproject(y, g)))


@pytest.mark.parametrize("change", [
    {"n_rows": 200, "row_mm": 2.0},       # cone half-angle above atan(1/2)
    {"sod_mm": 20.0},                     # orbit inside the volume (half-diagonal 26.9 mm)
    {"sdd_mm": 140.0},                    # SDD below SOD
    {"nz": 0},
    {"row_mm": -1.0},
], ids=["steep", "orbit", "sdd", "empty", "row"])
def test_refusals(torch, change):
    dect = _dect()
    g = dataclasses.replace(SMALL, **change)
    vol = torch.zeros((max(g.nz, 1), g.ny, g.nx), device="cuda")
    with pytest.raises((dect.DectError, ValueError)):
        dect.cone_project(vol, g)
        torch.cuda.synchronize()
