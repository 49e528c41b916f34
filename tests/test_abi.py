"""The C-ABI library loads and exports what include/dect.h declares; host-side
validation rejects bad arguments before any GPU work (runs without a GPU)."""
import ctypes as ct
import os
import re

import pytest

from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import dect

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="dect.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dect_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dect.LIB_PATH):
        pytest.skip("libdect.so not built")
    return dect.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dect.SIGNATURES), "binding and header disagree"


def test_every_header_symbol_is_exported(lib):
    """Every entry point that any header under include/ declares (the network
    kernels' dect_nn.h too) is exported by the one library."""
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert "dect_nn.h" in headers
    for h in headers:
        names = _declared(h)
        assert names, h
        for n in names:
            assert hasattr(lib, n), (h, n)


def test_version(lib):
    assert "gfx950" in dect.version()



def test_geometry_validation(lib):
    import dataclasses
    cases = [
        (dataclasses.replace(C.TINY, sod_mm=60.0), dect.DECT_ERR_GEOMETRY),   # source inside
        (dataclasses.replace(C.TINY, sdd_mm=400.0), dect.DECT_ERR_GEOMETRY),  # SDD < SOD
        (dataclasses.replace(C.TINY, n_bins=4000), dect.DECT_ERR_GEOMETRY),   # fan >= 90 deg
        (dataclasses.replace(C.TINY, nx=0), dect.DECT_ERR_INVALID_ARG),
        (dataclasses.replace(C.TINY, pixel_mm=-1.0), dect.DECT_ERR_INVALID_ARG),
        (dataclasses.replace(C.TINY, angles_rad=[float("nan")] * 60), dect.DECT_ERR_INVALID_ARG),
    ]
    buf = ct.c_void_p(16)  # never dereferenced: validation fails first
    for g, want in cases:
        st = lib.dect_project(dect.GeomArg(g).ref, buf, buf, 1, None)
        assert st == want, (g, st)
        assert lib.dect_last_error().decode() != ""
    assert lib.dect_project(None, buf, buf, 1, None) == dect.DECT_ERR_INVALID_ARG
    assert lib.dect_project(dect.GeomArg(C.TINY).ref, None, buf, 1, None) == dect.DECT_ERR_INVALID_ARG
    assert lib.dect_backproject(dect.GeomArg(C.TINY).ref, buf, buf, 0, None) == dect.DECT_ERR_INVALID_ARG


def test_parameter_validation(lib):
    buf = ct.c_void_p(16)
    g = dect.GeomArg(C.TINY)
    bad = dect.dect_adm_params(-1.0, 1.0, 1.0, 1.0, 1.0, 5, 0.0, 0, None)
    assert lib.dect_adm_tv(g.ref, buf, buf, ct.byref(bad), buf, buf, None, None, None) == \
        dect.DECT_ERR_INVALID_ARG
    p = dect.pls_params(C.PlsParams())
    sing = dect.dect_pls_params(1.0, 2.0, 2.0, 4.0, 1.0, 0.1, 0.25, 10, 1e-6)  # det D = 0
    assert lib.dect_pls_decompose(8, 8, buf, buf, ct.byref(sing), None, buf, buf, None, None) == \
        dect.DECT_ERR_INVALID_ARG
    assert lib.dect_pls_decompose(0, 8, buf, buf, ct.byref(p), None, buf, buf, None, None) == \
        dect.DECT_ERR_INVALID_ARG
    assert lib.dect_pls_edge_weights(8, 8, buf, -1.0, 0.1, buf, None) == dect.DECT_ERR_INVALID_ARG


def test_calls_fail_loudly_without_a_device(lib):
    """No CPU fallback: the binding requires device tensors."""
    import numpy as np
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        dect.project(torch.zeros((C.TINY.ny, C.TINY.nx)), C.TINY)


def test_volume_entry_points_validate_first(lib):
    """The cone-beam pair, the 3-D ADM and the 3-D PLS reject bad arguments
    on the host before any device work."""
    import dataclasses
    buf = ct.c_void_p(16)  # never dereferenced: validation fails first
    g = C.ConeGeometry(nx=40, ny=36, nz=21, voxel_mm=1.0, n_views=24, n_bins=70, n_rows=9,
                       bin_mm=1.3, row_mm=1.1, sod_mm=150.0, sdd_mm=300.0)
    cases = [
        (dataclasses.replace(g, n_rows=200, row_mm=2.0), dect.DECT_ERR_GEOMETRY),  # steep cone
        (dataclasses.replace(g, sod_mm=20.0), dect.DECT_ERR_GEOMETRY),            # orbit inside
        (dataclasses.replace(g, sdd_mm=140.0), dect.DECT_ERR_GEOMETRY),           # SDD < SOD
        (dataclasses.replace(g, nz=0), dect.DECT_ERR_INVALID_ARG),
        (dataclasses.replace(g, row_mm=-1.0), dect.DECT_ERR_INVALID_ARG),
    ]
    for gg, want in cases:
        assert lib.dect_cone_project(dect.ConeArg(gg).ref, buf, buf, None) == want, gg
        assert lib.dect_cone_backproject(dect.ConeArg(gg).ref, buf, buf, None) == want, gg
    assert lib.dect_cone_project(None, buf, buf, None) == dect.DECT_ERR_INVALID_ARG
    assert lib.dect_cone_project(dect.ConeArg(g).ref, None, buf, None) == dect.DECT_ERR_INVALID_ARG
    for flags, tol in ((dect.DECT_COUPLED_TV, 1e-3), (dect.DECT_COUPLED_TV | dect.DECT_STEP_ABB, 0.0),
                       (dect.DECT_STEP_BB2 | dect.DECT_STEP_ABB, 0.0), (64, 0.0),
                       (0, -1e-3), (0, float("nan")), (dect.DECT_WARM_START, float("inf"))):
        prm = dect.dect_adm_params(1.0, 16.0, 4.0, 1.0, 0.8, 5, tol, flags, None)
        assert lib.dect_adm_tv3(dect.ConeArg(g).ref, buf, buf, ct.byref(prm), buf, buf, None,
                                None) == dect.DECT_ERR_INVALID_ARG
    p = dect.pls_params(C.PlsParams())
    sing = dect.dect_pls_params(1.0, 2.0, 2.0, 4.0, 1.0, 0.1, 0.25, 10, 1e-6, 0)
    bad_mode = dect.pls_params(C.PlsParams(mode=7))
    for nz, prm in ((4, bad_mode), (4, sing), (0, p)):
        assert lib.dect_pls_decompose3(8, 8, nz, buf, buf, ct.byref(prm), None, buf, buf, None,
                                       None) == dect.DECT_ERR_INVALID_ARG
    assert lib.dect_pls_edge_weights3(8, 8, 0, buf, 0.25, 0.1, buf, None) == \
        dect.DECT_ERR_INVALID_ARG
    assert lib.dect_pls_edge_weights3(8, 8, 4, buf, -1.0, 0.1, buf, None) == \
        dect.DECT_ERR_INVALID_ARG


def test_unrolled_entry_points_validate_first(lib):
    """The unrolled step and its backward reject bad sizes, NULL buffers and
    outputs that overlap inputs on the host, before any device work."""
    a, b, c, d, e, p = (ct.c_void_p(4096 * k) for k in range(1, 7))
    o1, o2, o3 = (ct.c_void_p(1 << 24 + k) for k in range(3))
    inv = dect.DECT_ERR_INVALID_ARG
    assert lib.dect_unrolled_residual(-1, a, b, c, None) == inv
    assert lib.dect_unrolled_residual(8, None, b, c, None) == inv
    assert lib.dect_unrolled_residual(0, None, None, None, None) == dect.DECT_OK
    assert lib.dect_unrolled_step(0, 8, 1, a, b, c, d, p, o1, o2, o3, None) == inv
    assert lib.dect_unrolled_step(8, 8, -1, a, b, c, d, p, o1, o2, o3, None) == inv
    assert lib.dect_unrolled_step(8, 8, 1, a, b, None, d, p, o1, o2, o3, None) == inv
    assert lib.dect_unrolled_step(8, 8, 1, a, b, c, d, p, a, o2, o3, None) == inv  # f_out = f
    assert lib.dect_unrolled_step(8, 8, 1, a, b, c, d, p, o1, o1, o3, None) == inv
    assert lib.dect_unrolled_step(8, 8, 0, a, b, c, d, p, o1, o2, o3, None) == dect.DECT_OK
    g4 = ct.c_void_p(1 << 28)
    assert lib.dect_unrolled_step_backward(8, 8, 1, a, b, c, d, p, e, o1, o2, o3,
                                           ct.c_void_p(1 << 27), ct.c_void_p(1 << 26),
                                           None, g4, None) == inv  # ghb NULL
    assert lib.dect_unrolled_step_backward(8, 8, 1, a, b, c, d, p, e, o1, o2, e,
                                           ct.c_void_p(1 << 27), ct.c_void_p(1 << 26),
                                           ct.c_void_p(1 << 25), g4, None) == inv  # gf = gf_out
