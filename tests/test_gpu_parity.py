"""GPU parity: the HIP transport kernel against the FP64 oracle, through the
C-ABI.

* FP64 validation mode: per cell and per pixel |gpu - oracle| <= 1e-9 |oracle|
  (plus 16 spacings of the subnormal range, 16 x 2^-1074, where relative
  agreement is not representable) and identical zero patterns; identical
  event and cell counters.  The only allowed differences are the order of
  the atomic additions and of the factors of a product.
* FP32 production mode: on cells and pixels with an effective number of
  contributions >= 10, at most 0.5 % may differ from the oracle by more than
  3 sigma (sigma from the oracle's per-packet second moments); global sums
  within 1e-5 relative (1e-4 for images); energy balance within 1e-5.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1705_04702_amd import mcrt, scenes

pytestmark = pytest.mark.gpu

REL_FP64 = 1e-9
# Below the smallest normal double (2^-1022) values are spaced 2^-1074 apart,
# so relative agreement degrades there (a pixel of 1e-317 holds 7 significant
# digits).  The two sides form a value with the same factors in different
# orders, each rounding at most half a spacing: 16 spacings of absolute slack
# cover that, and nothing above the subnormal range.
ABS_SUBNORMAL = 16 * 2.0 ** -1074


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = mcrt.Context(0)
    yield c
    c.close()


def gpu_run(ctx, sc, N, seed=0, precision=mcrt.FP64_VALIDATE, first_id=0, count=None, **tune):
    say(f"run {sc.name} N={N} seed={seed} prec={precision} ids=[{first_id},+{count}) {tune}")
    return mcrt.run_scene(sc, N, seed=seed, precision=precision, first_id=first_id, count=count,
                          ctx=ctx, **tune)


def assert_fp64_parity(g, o, counters=True):
    for name, a, b in [("table", g["table"], o["table"])] + [
            (f"image{j}", x, y) for j, (x, y) in enumerate(zip(g["images"], o["images"]))]:
        assert np.array_equal(a == 0, b == 0), f"{name}: zero patterns differ"
        nz = b != 0
        d = np.abs(a[nz] - b[nz])
        rel = d / np.abs(b[nz])
        say(f"{name}: {nz.sum()} nonzero, max rel err {rel.max() if rel.size else 0:.3e}")
        bad = d > REL_FP64 * np.abs(b[nz]) + ABS_SUBNORMAL
        assert not bad.any(), f"{name}: max rel {rel[bad].max()} at |oracle| {np.abs(b[nz][bad]).min():.3e}"
    # global FP64 sums: the summation order differs (bound ~ N eps)
    np.testing.assert_allclose(g["energy"], o["energy"], rtol=REL_FP64)
    if counters:
        for k in ("packets", "events", "prop_cells", "peel_adds", "peel_dropped", "capped"):
            assert g["stats"][k] == o["stats"][k], k


def assert_fp32_statistical(g, o, N, sigmas=3.0, frac=0.005):
    e = g["energy"]
    assert abs(e[0] - e[1] - e[2] - e[3]) / e[0] < 1e-5
    assert abs(e[1] - o["energy"][1]) / o["energy"][1] < 1e-5 + 3 * _rel_sigma_total(o, N)
    pairs = [(g["table"], o["table"], o["table_m2"])] + list(zip(g["images"], o["images"], o["image_m2"]))
    for a, T, m2 in pairs:
        var = np.maximum(m2 - T * T / N, 0.0)
        neff = np.where(m2 > 0, T * T / np.where(m2 > 0, m2, 1.0), 0.0)
        sel = neff >= 10
        if sel.sum() == 0:
            continue
        bad = np.abs(a[sel] - T[sel]) > sigmas * np.sqrt(var[sel]) + 1e-7 * np.abs(T[sel])
        assert bad.mean() <= frac, f"{bad.mean()} of {sel.sum()} beyond {sigmas} sigma"
        assert abs(a.sum() - T.sum()) <= 1e-4 * abs(T.sum()) + 3 * np.sqrt(var.sum())


def _rel_sigma_total(o, N):
    T = o["table"]
    var = np.maximum(o["table_m2"] - T * T / N, 0).sum()
    return np.sqrt(var) / max(T.sum(), 1e-300)


# ---------------------------------------------------------------------------

def test_sphere_c1_fp64_full(ctx):
    """Uniform sphere, tau = 1, albedo 0.5, g = 0.5, 32^3 grid, 64^2 image,
    1e5 packets, seed 0: the whole run matches the oracle."""
    sc = scenes.sphere()
    N = 100000
    o = oracle.run(sc, N, seed=0)
    g = gpu_run(ctx, sc, N, seed=0)
    assert_fp64_parity(g, o)


@pytest.mark.parametrize("make,N", [
    (lambda: scenes.disk((32, 32, 16), 8, 64), 600),
    (lambda: scenes.torus(6, 5, 4, 128, n_clumps=60), 400),
    (lambda: scenes.sphere(n=24, tau=6.0, albedo=0.9, g=-0.3, incl_deg=35, azim_deg=80), 3000),
    (lambda: scenes.uniform_cube(3, 2.0, 0.7, 0.8, src=(0.3, -0.9, 0.99)), 3000),
])
def test_fp64_parity_scene_families(ctx, make, N):
    sc = make()
    o = oracle.run(sc, N, seed=5)
    g = gpu_run(ctx, sc, N, seed=5)
    assert_fp64_parity(g, o)


def test_disk_full_grid_fp64_and_fp32(ctx):
    """The exponential disk at its full 256^3 grid and 3 x 512^2 instruments,
    on 4 of the 64 wavelengths and a packet subset."""
    sc = scenes.disk()
    keep = [0, 21, 42, 63]
    for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
        setattr(sc, f, getattr(sc, f)[keep])
    sc.name = "disk256_4l"
    N = 300
    o = oracle.run(sc, N, seed=3, moments=True)
    g = gpu_run(ctx, sc, N, seed=3)
    assert_fp64_parity(g, o)
    g32 = gpu_run(ctx, sc, N, seed=3, precision=mcrt.FP32)
    e = g32["energy"]
    assert abs(e[0] - e[1] - e[2] - e[3]) / e[0] < 1e-5


def test_ragged_ranges_and_split_runs_add(ctx):
    sc = scenes.disk((16, 16, 8), 3, 32)
    N = 1000
    o = oracle.run(sc, N, seed=8, first_id=123, count=777)
    g = gpu_run(ctx, sc, N, seed=8, first_id=123, count=777, chunk=37)
    assert_fp64_parity(g, o)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE, chunk=64)
    try:
        full = sim.run(N, 8)
        part = sim.new_result()
        sim.run_into(part, N, 8, 0, 401)
        sim.run_into(part, N, 8, 401, 599)
        np.testing.assert_allclose(part.table(), full.table(), rtol=1e-12, atol=0)
        np.testing.assert_allclose(part.image(0), full.image(0), rtol=1e-12, atol=0)
        np.testing.assert_allclose(part.energy(), full.energy(), rtol=1e-12)
        empty = sim.new_result()
        sim.run_into(empty, N, 8, N, 0)
        assert not empty.table().any() and not empty.energy().any()
        for r in (full, part, empty):
            r.close()
    finally:
        sim.close()


@pytest.mark.parametrize("tune", [dict(chunk=1, threshold=1, waves_per_cu=1),
                                  dict(chunk=1000, threshold=64, waves_per_cu=2),
                                  dict(chunk=64, threshold=8, waves_per_cu=32)])
def test_schedule_invariance(ctx, tune):
    """Results do not depend on the queue chunk, the compaction threshold or
    the number of persistent waves (beyond atomic ordering)."""
    sc = scenes.sphere(n=16, tau=2.0)
    N = 4000
    o = oracle.run(sc, N, seed=12)
    g = gpu_run(ctx, sc, N, seed=12, **tune)
    assert_fp64_parity(g, o)


def test_event_cap_reports_elimit(ctx):
    sc = scenes.sphere(n=16, tau=4.0, albedo=0.95)
    sc.event_cap = 1
    N = 2000
    o = oracle.run(sc, N, seed=2)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    try:
        res = sim.new_result()
        rc = sim.run_into(res, N, 2)
        assert rc == mcrt.ELIMIT
        g = {"table": res.table(), "images": res.images(), "energy": res.energy(), "stats": res.stats()}
        assert g["stats"]["capped"] == o["stats"]["capped"] > 0
        assert_fp64_parity(g, o)
        res.close()
    finally:
        sim.close()


def test_degenerate_media(ctx):
    # empty medium: everything escapes, the image is the direct light only
    sc = scenes.sphere(n=8)
    sc.density = np.zeros_like(sc.density)
    g = gpu_run(ctx, sc, 500, seed=1)
    assert g["energy"][2] == pytest.approx(1.0, rel=1e-12) and g["energy"][1] == 0
    assert np.count_nonzero(g["images"][0]) == 1
    # no scattering
    sc = scenes.sphere(n=8, albedo=0.0)
    o = oracle.run(sc, 500, seed=1)
    assert_fp64_parity(gpu_run(ctx, sc, 500, seed=1), o)
    # source outside the grid, no instruments
    sc = scenes.uniform_cube(2, 1.0, 0.6, 0.2, src=(3.0, 0.2, -0.1))
    sc.instruments = []
    o = oracle.run(sc, 2000, seed=4)
    assert_fp64_parity(gpu_run(ctx, sc, 2000, seed=4), o)


def test_errors_are_reported(ctx, monkeypatch):
    sc = scenes.sphere(n=8)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    try:
        res = sim.new_result()
        with pytest.raises(mcrt.MCRTError) as ei:
            sim.run_into(res, 100, 0, 50, 51)
        assert ei.value.code == mcrt.EINVAL
        with pytest.raises(mcrt.MCRTError) as ei:
            sim.run_into(res, 0, 0)
        assert ei.value.code == mcrt.EINVAL
        monkeypatch.setenv("MCRT_DEBUG_FAIL_ALLOC", "1")
        with pytest.raises(mcrt.MCRTError) as ei:
            sim.new_result()
        assert ei.value.code == mcrt.ENOMEM
        monkeypatch.delenv("MCRT_DEBUG_FAIL_ALLOC")
        res.close()
    finally:
        sim.close()


def test_concurrent_run_is_busy(ctx):
    """A second run on a sim that is still running is refused with EBUSY."""
    sc = scenes.disk((64, 64, 32), 16, 64)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    try:
        r1, r2 = sim.new_result(), sim.new_result()
        out = {}

        def long_run():
            out["rc"] = sim.run_into(r1, 4000000, 0)

        t = threading.Thread(target=long_run)
        t.start()
        busy = 0
        while t.is_alive() and busy == 0:
            try:
                sim.run_into(r2, 10, 0)
            except mcrt.MCRTError as e:
                assert e.code == mcrt.EBUSY
                busy += 1
            time.sleep(0.01)
        t.join()
        assert busy == 1
        assert out["rc"] == mcrt.OK
        r1.close()
        r2.close()
    finally:
        sim.close()


def test_full_size_disk_in_the_bench_launch_configuration(ctx):
    """The disk workload at full size in bench.py's launch (ids [0, 1e6) of
    all 64 wavelengths, 6.4e7 packets, FP32): properties that hold at any
    size -- energy balance, packet count, two half-ranges adding up to the
    whole -- and the absorbed total per wavelength against the oracle's
    estimate from a packet subset (4 sigma)."""
    sc = scenes.disk()
    N = 10_000_000
    B = 1_000_000
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    try:
        say("full-size disk launch: ids [0, 1e6) x 64 wavelengths")
        whole = sim.run(N, 0, 0, B)
        halves = sim.new_result()
        sim.run_into(halves, N, 0, 0, B // 2)
        sim.run_into(halves, N, 0, B // 2, B - B // 2)
        e = whole.energy()
        assert abs(e[0] - e[1] - e[2] - e[3]) / e[0] < 1e-5
        st = whole.stats()
        assert st["packets"] == B * sc.n_lambda and st["capped"] == 0
        np.testing.assert_allclose(halves.energy(), e, rtol=1e-6)
        tw, th = whole.table(), halves.table()
        per_l_w, per_l_h = tw.sum(axis=0), th.sum(axis=0)
        np.testing.assert_allclose(per_l_h, per_l_w, rtol=1e-5)
        # oracle estimate of the absorbed luminosity per packet on 4 of the
        # wavelengths (one-wavelength copies of the scene, own streams): K
        # independent batches give the mean and its standard error
        K, n_b = 16, 16
        bad = 0
        for ell in (0, 21, 42, 63):
            sub = type(sc)(**{**sc.__dict__})
            for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
                setattr(sub, f, np.ascontiguousarray(getattr(sc, f)[ell:ell + 1]))
            means = np.array([oracle.run(sub, N, seed=7, first_id=k * n_b, count=n_b)["energy"][1] / n_b
                              for k in range(K)])
            m, se = means.mean(), means.std(ddof=1) / np.sqrt(K)
            g_mean = per_l_w[ell] / B
            say(f"lambda {ell}: gpu {g_mean:.6e} per packet, oracle {m:.6e} +- {se:.2e}")
            bad += abs(g_mean - m) > 4.5 * se + 1e-9 * abs(m)
        assert bad == 0
        for r in (whole, halves):
            r.close()
    finally:
        sim.close()


def test_full_size_torus(ctx):
    """The clumpy torus at full size (2.24e6 leaves to depth 9, 1024^2
    edge-on instrument): FP64 parity with the oracle on 3 of the 32
    wavelengths for a packet-id range inside the full N; then bench.py's FP32
    launch (ids [0, 1e6) of all 32 wavelengths): energy balance, packet
    count, no capped packets, no octree walk stopped by its step guard, and
    two half-ranges adding up to the whole."""
    sc = scenes.torus()
    N = 3_125_000
    sub = type(sc)(**{**sc.__dict__})
    keep = [0, 15, 31]
    for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
        setattr(sub, f, np.ascontiguousarray(getattr(sc, f)[keep]))
    sub.name = "torus_full_3l"
    first, count = 1_234_567, 400
    o = oracle.run(sub, N, seed=4, first_id=first, count=count)
    g = gpu_run(ctx, sub, N, seed=4, first_id=first, count=count)
    assert_fp64_parity(g, o)
    B = 1_000_000
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    try:
        say("full-size torus launch: ids [0, 1e6) x 32 wavelengths")
        whole = sim.run(N, 0, 0, B)
        halves = sim.new_result()
        sim.run_into(halves, N, 0, 0, B // 2)
        sim.run_into(halves, N, 0, B // 2, B - B // 2)
        e = whole.energy()
        assert abs(e[0] - e[1] - e[2] - e[3]) / e[0] < 1e-5
        st = whole.stats()
        assert st["packets"] == B * sc.n_lambda and st["capped"] == 0 and st["guard"] == 0
        np.testing.assert_allclose(halves.energy(), e, rtol=1e-6)
        np.testing.assert_allclose(halves.table().sum(axis=0), whole.table().sum(axis=0), rtol=1e-5)
        for r in (whole, halves):
            r.close()
    finally:
        sim.close()


def test_axis_aligned_instruments_fp64(ctx):
    """Peel-offs along the six grid axes (column maps, no march) next to an
    oblique one, on flat cells with sources inside and outside the grid and
    peel-offs dropped at tau_peel_max: FP64 parity per pixel."""
    sc = scenes.disk((20, 16, 10), 3, 20, tau_v_faceon=4.0)
    sc.instruments = [scenes.Instrument(i, a, 1.0e4, (40.0, 40.0), (20, 20))
                      for i, a in [(0, 0), (180, 0), (90, 0), (90, 180), (90, 90), (90, 270), (60, 30)]]
    sc.tau_peel_max = 1.0
    N = 600
    o = oracle.run(sc, N, seed=13)
    assert o["stats"]["peel_dropped"] > 0
    g = gpu_run(ctx, sc, N, seed=13)
    assert_fp64_parity(g, o)


@pytest.mark.parametrize("cut", [float("inf"), 0.7])
def test_octree_axis_aligned_instruments_fp64(ctx, cut):
    """Octree grids: peel-offs along the six grid axes read the lattice
    column maps (two reads, no march) beside an oblique instrument that
    marches; a random octree with random densities and a source inside, the
    same with the source outside the grid, and a small clumpy torus: FP64
    parity per pixel with the oracle's leaf-by-leaf marches, drops at a tau
    cut included."""
    from test_lanesim import AXES, _random_octree_scene
    for sc in (_random_octree_scene(5, (0.137, -0.421, 0.25)), _random_octree_scene(6, (1.7, 0.3, -0.2)),
               scenes.torus(5, 4, 2, 16, n_clumps=25, tau_eq=8.0)):
        small = sc.box[3] < 5
        sc.instruments = [scenes.Instrument(i, a, 100.0 if small else 1.0e4, (2.2, 2.2) if small else (30.0, 30.0),
                                            (16, 16)) for i, a in AXES]
        sc.tau_peel_max = cut
        o = oracle.run(sc, 700, seed=14)
        if cut < 1e30:
            assert o["stats"]["peel_dropped"] > 0
        g = gpu_run(ctx, sc, 700, seed=14)
        assert_fp64_parity(g, o)
        assert 0 < g["stats"]["peel_cells"] < o["stats"]["peel_cells"] / 3


def _deep_octree_scene(depth=12):
    """An octree refined to depth 12 around two points (a few random coarse
    refinements besides): leaves from level 1 to 12, so the walk chains
    blocks three deep below its top table; deeper than the lattice column
    maps go (10), so the axis-aligned instruments march."""
    pts = np.array([[0.6173, 0.3391, 0.5527], [0.2468, 0.7113, 0.4029]])
    rng = np.random.default_rng(21)

    def refine(level, ix, iy, iz):
        n = 1 << level
        hit = np.zeros(ix.shape, bool)
        for p in pts:
            c = np.floor(p * n).astype(np.int64)
            hit |= (ix == c[0]) & (iy == c[1]) & (iz == c[2])
        return hit | ((level < 3) & (rng.random(ix.shape[0]) < 0.5)) | (level == 0)

    fc, leaves, D = scenes.octree_from_levels(refine, depth)
    nl = leaves[0].shape[0]
    dens = np.random.default_rng(22).uniform(0.2, 3.0, nl).astype(np.float32)
    src = tuple(-1.0 + 2.0 * pts[0] + 1e-4)  # inside the deepest leaves
    sc = scenes.Scene(grid_type="octree", box=(-1.0, -1.0, -1.0, 1.0, 1.0, 1.0), first_child=fc, density=dens,
                      lambdas=np.array([0.55, 3.0]), kappa=np.array([1.2, 0.3]), albedo=np.array([0.6, 0.4]),
                      hg_g=np.array([0.3, 0.0]), lum=np.array([1.0, 0.5]), source="point_iso", src_pos=src,
                      instruments=[scenes.Instrument(i, a, 100.0, (2.2, 2.2), (32, 32))
                                   for i, a in ((90, 0), (0, 0), (50, 20))], name="deep_octree12")
    return sc, D


def test_deep_octree_fp64_and_fp32(ctx):
    sc, D = _deep_octree_scene()
    assert D == 12
    o = oracle.run(sc, 2000, seed=3)
    g = gpu_run(ctx, sc, 2000, seed=3)
    assert_fp64_parity(g, o)
    assert g["stats"]["guard"] == 0 and g["stats"]["peel_cells"] == o["stats"]["peel_cells"]
    f = gpu_run(ctx, sc, 20000, seed=3, precision=mcrt.FP32)
    e = f["energy"]
    assert abs(e[0] - e[1] - e[2] - e[3]) / e[0] < 1e-5 and f["stats"]["guard"] == 0


def test_largest_packet_ids_fp64(ctx):
    """The largest run the boundary accepts, 2^32 packets per wavelength:
    its last ids (up to 2^32 - 1, the full width of the stream counter's
    packet word) against the oracle."""
    sc = scenes.disk((16, 16, 8), 2, 24)
    N = 1 << 32
    first, count = N - 257, 257
    o = oracle.run(sc, N, seed=5, first_id=first, count=count)
    g = gpu_run(ctx, sc, N, seed=5, first_id=first, count=count)
    assert g["stats"]["packets"] == 2 * count
    assert_fp64_parity(g, o)
