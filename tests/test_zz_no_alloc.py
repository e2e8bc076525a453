"""The allocation-free entry point (mcrt_run_into_noalloc) against
mcrt_run_into, through the C-ABI.

Its kernels are mcrt_run_into's; only the launch's scratch (the work-queue
counter and the per-wavelength optics) comes from the library's per-GPU
array, prepared on the device.  Two calls in a row, the second with a
smaller input (fewer wavelengths, fewer packets), each equal to the
existing entry point's result: FP64 validation per cell and pixel to 1e-9
(and to the oracle), FP32 to the order of the atomic additions; a sim with
a learned proposal; the size limit; results that add up across calls.
"""
import numpy as np
import pytest

import oracle
from paper_1705_04702_amd import mcrt, scenes

from test_gpu_parity import assert_fp64_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = mcrt.Context(0)
    yield c
    c.close()


def _both(ctx, sc, N, seed, precision, first_id=0, count=None, theta=None):
    sim = mcrt.Sim(ctx, sc, precision)
    prop = None
    if theta is not None:
        prop = mcrt.Proposal(ctx, params=theta)
        sim.set_proposal(prop, 0.2)
    ra, rb = sim.new_result(), sim.new_result()
    say(f"noalloc {sc.name} N={N} prec={precision} ids=[{first_id},+{count})")
    ca = sim.run_into(ra, N, seed=seed, first_id=first_id, count=count)
    cb = sim.run_into_noalloc(rb, N, seed=seed, first_id=first_id, count=count)
    out = []
    for r in (ra, rb):
        out.append({"table": r.table(), "images": r.images(), "energy": r.energy(), "stats": r.stats()})
        r.close()
    sim.close()
    if prop is not None:
        prop.close()
    assert ca == cb
    return out[0], out[1]


def _same_fp64(a, b):
    assert_fp64_parity(b, a)
    for k in mcrt.STAT_FIELDS:
        assert a["stats"][k] == b["stats"][k], k


def test_noalloc_fp64_two_calls_second_smaller(ctx):
    big = scenes.disk((16, 16, 8), 5, 24)
    a, b = _both(ctx, big, 1500, 3, mcrt.FP64_VALIDATE)
    _same_fp64(a, b)
    assert_fp64_parity(b, oracle.run(big, 1500, seed=3))
    assert b["stats"]["kernel_ms"] == 0.0
    small = scenes.sphere(n=12, tau=2.0, albedo=0.6)
    a, b = _both(ctx, small, 400, 4, mcrt.FP64_VALIDATE, first_id=37, count=211)
    _same_fp64(a, b)
    assert_fp64_parity(b, oracle.run(small, 400, seed=4, first_id=37, count=211))


def test_noalloc_fp32_two_calls_second_smaller(ctx):
    for sc, N, seed in ((scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0), 6000, 5),
                        (scenes.sphere(n=16, tau=1.0), 2000, 6)):
        a, b = _both(ctx, sc, N, seed, mcrt.FP32)
        # the same packets with the same arithmetic; only the order of the
        # atomic additions differs (FP64 table sums, FP32 pixels)
        for k in ("packets", "events", "prop_cells", "locate_cells", "peel_cells", "peel_adds", "capped"):
            assert a["stats"][k] == b["stats"][k], k
        np.testing.assert_allclose(b["table"], a["table"], rtol=1e-10, atol=1e-300)
        for x, y in zip(b["images"], a["images"]):
            np.testing.assert_allclose(x, y, rtol=1e-5, atol=1e-6 * np.abs(y).max())
        np.testing.assert_allclose(b["energy"], a["energy"], rtol=1e-10)


def test_noalloc_learned_fp64(ctx):
    sc = scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0)
    theta = scenes.init_mlp(2, scale=1.5).astype(np.float32)
    a, b = _both(ctx, sc, 300, 7, mcrt.FP64_VALIDATE, theta=theta)
    _same_fp64(a, b)


def test_noalloc_results_add_and_limits(ctx):
    sc = scenes.disk((16, 16, 8), 3, 24)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    whole, parts = sim.new_result(), sim.new_result()
    sim.run_into(whole, 900, seed=9)
    sim.run_into_noalloc(parts, 900, seed=9, first_id=0, count=500)
    sim.run_into_noalloc(parts, 900, seed=9, first_id=500, count=400)
    np.testing.assert_allclose(parts.table(), whole.table(), rtol=1e-12, atol=0)
    np.testing.assert_allclose(parts.energy(), whole.energy(), rtol=1e-12)
    with pytest.raises(mcrt.MCRTError) as ei:
        sim.run_into_noalloc(parts, 900, seed=9, first_id=800, count=200)
    assert ei.value.code == mcrt.EINVAL
    for r in (whole, parts):
        r.close()
    sim.close()
    # more wavelengths than the scratch array holds
    many = scenes.sphere(n=2)
    nl = 4097
    many.lambdas = np.exp(np.linspace(np.log(0.1), np.log(1000.0), nl))
    for f in ("kappa", "albedo", "hg_g", "lum"):
        setattr(many, f, np.repeat(getattr(many, f), nl))
    sim = mcrt.Sim(ctx, many, mcrt.FP32)
    r = sim.new_result()
    with pytest.raises(mcrt.MCRTError) as ei:
        sim.run_into_noalloc(r, 10, seed=0)
    assert ei.value.code == mcrt.EINVAL and "4096" in str(ei.value)
    r.close()
    sim.close()
