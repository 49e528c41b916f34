"""Batched ADM-TV over slices of uneven size and view count (dect_adm_tv_batched).

* with the built-in view grouping the batch reproduces the single-slice path
  bit for bit (same kernels bodies and reduction trees);
* with any autotuned grouping it matches the FP64 oracle per slice
  (rel-L2 <= 1e-4) after the iterations;
* the autotuner returns one of the offered shapes, and a batch of the same
  slice shapes takes the remembered choice without timing;
* at the configuration's sizes (512 x 512 at 360 views, 384 x 384 at 90,
  256 x 256 at 60) every slice matches the oracle after 200 iterations;
* Siddon slices and slices with the coupled TV, the projection onto f >= 0
  and the BB2 / adaptive steps, mixed with plain Joseph ones, reproduce their
  single-slice runs bit for bit, also after one and two iterations (the
  projected slices' first step runs outside the captured graph).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_01650_amd import configs as C
from paper_1607_01650_amd import phantom as P

from helpers import f32, need_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _slices():
    specs = [(64, 30), (96, 45), (128, 60), (64, 90), (96, 20)]
    out = []
    for i, (n, V) in enumerate(specs):
        g = C.Geometry(nx=n, ny=n, pixel_mm=1.0, n_views=V, n_bins=int(round(1.4375 * n)),
                       bin_mm=2.4, sod_mm=500.0, sdd_mm=1000.0)
        s = P.make_slice(g, 40 + i, n_inserts=4, r_obj=0.4 * n)
        p = C.AdmParams(mu=45.0 / V, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79)
        out.append((g, s, p))
    return out


def test_batch_matches_single_bitwise_and_oracle(torch):
    from paper_1607_01650_amd import dect
    sl = _slices()
    iters = 24
    mh = [to_dev(torch, s.sino[0]) for _, s, _ in sl]
    ml = [to_dev(torch, s.sino[1]) for _, s, _ in sl]
    b = dect.AdmBatch([g for g, _, _ in sl], [p for _, _, p in sl])
    xh, xl, obj = b.run(mh, ml, iters, want_objective=True)
    for i, (g, s, p) in enumerate(sl):
        import dataclasses
        r = dect.adm_tv(mh[i], ml[i], g, dataclasses.replace(p, max_iter=iters), want_log=True)
        assert np.array_equal(to_np(xh[i]), to_np(r.x_high)), i
        assert np.array_equal(to_np(xl[i]), to_np(r.x_low)), i
        assert obj[i] == pytest.approx(r.report.objective, rel=1e-12)
    # another grouping: same method, different summation order -> oracle parity
    b.set_groups(4)
    xh4, xl4, _ = b.run(mh, ml, iters)
    for i, (g, s, p) in enumerate(sl):
        for e, (beta, x) in enumerate(((p.beta_high, xh4[i]), (p.beta_low, xl4[i]))):
            ref = O.adm(g, f32(s.sino[e]), beta, p.mu, p.rho, p.xi, iters)
            err = rel_l2(to_np(x), ref.x)
            assert err <= 1e-4, (i, e, err)
    b.close()


def test_batch_autotune(torch):
    from paper_1607_01650_amd import dect
    sl = _slices()
    mh = [to_dev(torch, s.sino[0]) for _, s, _ in sl]
    ml = [to_dev(torch, s.sino[1]) for _, s, _ in sl]
    b = dect.AdmBatch([g for g, _, _ in sl], [p for _, _, p in sl])
    builtin = b.shape()[0]
    groups, ms = b.tune(mh, ml, iters=4)
    per_slice, adj_cu, fwd_cu, cached = b.shape()
    print(f"tuned: depth per slice {per_slice} (built-in {builtin}), adjoint blocks/CU {adj_cu}, "
          f"forward {fwd_cu}, {ms:.3f} ms per iteration, cached {cached}", flush=True)
    assert groups in per_slice and ms > 0 and not cached
    # each slice keeps its built-in depth or takes a timed candidate its
    # view count allows
    for g, g0, (gg, _, _) in zip(per_slice, builtin, sl):
        assert g == g0 or (g in (1, 2, 4, 8, 16) and g <= max(1, gg.n_views // 8)), (g, g0)
    assert adj_cu in (0, 1, 2) and fwd_cu in (0, 1, 2)
    xh, xl, obj = b.run(mh, ml, 6, want_objective=True)
    assert all(np.isfinite(o) for o in obj)
    b.close()
    # the same slice shapes in another order: the remembered shape, no timing
    order = [4, 2, 0, 3, 1]
    b2 = dect.AdmBatch([sl[i][0] for i in order], [sl[i][2] for i in order])
    groups2, _ = b2.tune([mh[i] for i in order], [ml[i] for i in order], iters=4)
    per2, adj2, fwd2, cached2 = b2.shape()
    assert cached2 and groups2 == groups and (adj2, fwd2) == (adj_cu, fwd_cu)
    assert per2 == [per_slice[i] for i in order]
    b2.close()


def test_batch_paper_scale_parity(torch):
    """A batch of the configuration's sizes: a 512 x 512 slice at 360 views
    (the stored FP64 oracle run of slice 0, 200 iterations), a 384 x 384 slice
    at 90 views and a 256 x 256 slice at 60 views (the oracle run live), all
    advanced together for 200 iterations with the built-in grouping and with
    a tuned one; every image within rel-L2 1e-4 of the oracle."""
    import os
    from paper_1607_01650_amd import dect
    g512 = C.paper_geometry(512, 360)
    g384 = C.paper_geometry(384, 90)
    g256 = C.paper_geometry(256, 60)
    geoms = [g384, g512, g256]
    sl = [P.make_slice(g384, 7), P.make_slice(g512, 0), P.make_slice(g256, 8)]
    params = [C.default_adm_params(g, 200) for g in geoms]
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "adm512_v360_k200.npz"))
    assert float(gold["mu"]) == params[1].mu
    refs = {}
    for i in (0, 2):
        p = params[i]
        refs[i] = [O.adm(geoms[i], f32(sl[i].sino[e]), beta, p.mu, p.rho, p.xi, 200).x
                   for e, beta in ((0, p.beta_high), (1, p.beta_low))]
    refs[1] = [gold["x"][0], gold["x"][1]]
    mh = [to_dev(torch, s.sino[0]) for s in sl]
    ml = [to_dev(torch, s.sino[1]) for s in sl]
    b = dect.AdmBatch(geoms, params)
    for label in ("built-in", "tuned"):
        if label == "tuned":
            groups, ms = b.tune(mh, ml, iters=4)
            print(f"tuned grouping {groups}, {ms:.3f} ms per iteration", flush=True)
        xh, xl, _ = b.run(mh, ml, 200)
        for i, g in enumerate(geoms):
            for e, x in enumerate((xh[i], xl[i])):
                err = rel_l2(to_np(x), refs[i][e])
                print(f"batch {label} {g.nx}x{g.ny} V={g.n_views} energy {e}: rel-L2 {err:.2e}",
                      flush=True)
                assert err <= 1e-4
    b.close()


def test_batch_siddon_and_coupled_bitwise(torch):
    """A batch that mixes both projector models and coupled / per-energy TV
    (their own persistent launches per phase) equals each slice's
    single-slice run bit for bit, objective included."""
    import dataclasses
    from paper_1607_01650_amd import dect
    specs = [(64, 30, 0, False), (96, 45, 1, False), (80, 36, 0, True), (64, 40, 1, True),
             (72, 24, 1, False)]
    sl = []
    for i, (n, V, model, coupled) in enumerate(specs):
        g = C.Geometry(nx=n, ny=n, pixel_mm=1.0, n_views=V, n_bins=int(round(1.4375 * n)),
                       bin_mm=2.4, sod_mm=500.0, sdd_mm=1000.0, model=model)
        s = P.make_slice(g, 60 + i, n_inserts=4, r_obj=0.4 * n)
        p = C.AdmParams(mu=45.0 / V, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79,
                        coupled_tv=coupled)
        sl.append((g, s, p))
    iters = 21  # odd: the last iteration runs outside the graph
    mh = [to_dev(torch, s.sino[0]) for _, s, _ in sl]
    ml = [to_dev(torch, s.sino[1]) for _, s, _ in sl]
    b = dect.AdmBatch([g for g, _, _ in sl], [p for _, _, p in sl])
    xh, xl, obj = b.run(mh, ml, iters, want_objective=True)
    for i, (g, s, p) in enumerate(sl):
        r = dect.adm_tv(mh[i], ml[i], g, dataclasses.replace(p, max_iter=iters), want_log=True)
        assert np.array_equal(to_np(xh[i]), to_np(r.x_high)), i
        assert np.array_equal(to_np(xl[i]), to_np(r.x_low)), i
        assert obj[i] == pytest.approx(r.report.objective, rel=1e-12), i
    b.close()


def test_batch_variants_bitwise(torch):
    """Projected (Joseph and Siddon, with and without the coupled TV), BB2
    and adaptive slices in one batch with a plain one: each equals its
    single-slice run bit for bit after 1, 2 and 21 iterations; the
    combinations the single-slice path refuses are refused."""
    import dataclasses
    from paper_1607_01650_amd import dect
    specs = [(64, 30, 0, dict(nonneg=True)), (72, 36, 1, dict(nonneg=True)),
             (80, 40, 0, dict(step="bb2")), (64, 30, 1, dict(step="abb")),
             (96, 45, 0, dict(nonneg=True, coupled_tv=True)),
             (64, 24, 0, dict(step="abb", coupled_tv=True)), (72, 30, 0, {})]
    sl = []
    rng = np.random.default_rng(5)
    for i, (n, V, model, kw) in enumerate(specs):
        g = C.Geometry(nx=n, ny=n, pixel_mm=1.0, n_views=V, n_bins=int(round(1.4375 * n)),
                       bin_mm=2.4, sod_mm=500.0, sdd_mm=1000.0, model=model)
        s = P.make_slice(g, 80 + i, n_inserts=4, r_obj=0.4 * n)
        # noisy data, so that the projection binds at many pixels
        sino = [f32(a + 0.05 * a.max() * rng.standard_normal(a.shape)) for a in s.sino]
        p = C.AdmParams(mu=45.0 / V, rho=1024.0, xi=256.0, beta_high=1.0, beta_low=0.79, **kw)
        sl.append((g, sino, p))
    mh = [to_dev(torch, s[0]) for _, s, _ in sl]
    ml = [to_dev(torch, s[1]) for _, s, _ in sl]
    b = dect.AdmBatch([g for g, _, _ in sl], [p for _, _, p in sl])
    for iters in (1, 2, 21):
        xh, xl, obj = b.run(mh, ml, iters, want_objective=True)
        for i, (g, s, p) in enumerate(sl):
            r = dect.adm_tv(mh[i], ml[i], g, dataclasses.replace(p, max_iter=iters),
                            want_log=True)
            assert np.array_equal(to_np(xh[i]), to_np(r.x_high)), (iters, i)
            assert np.array_equal(to_np(xl[i]), to_np(r.x_low)), (iters, i)
            assert obj[i] == pytest.approx(r.report.objective, rel=1e-12), (iters, i)
            if p.nonneg:
                assert to_np(xh[i]).min() >= 0.0 and to_np(xl[i]).min() >= 0.0
    b.close()
    g, _, p = sl[-1]
    for change in ({"nonneg": True, "step": "bb2"}, {"coupled_tv": True, "tol": 1e-4}):
        with pytest.raises(dect.DectError):
            dect.AdmBatch([g], [dataclasses.replace(p, **change)])
