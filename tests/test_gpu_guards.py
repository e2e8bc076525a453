"""Guards of the transport kernels, forced from the host, through the C-ABI.

* Non-finite luminosity: a learned proposal whose parameters hold a NaN (as a
  diverged training would leave them) gives every packet a NaN weight at its
  first scattering on the disk (whose emission stays physical).  Each such
  packet is ended there, counted in stats.nonfinite, its luminosity before
  the weight truncated, and the launch returns MCRT_ENONFINITE.  Up to that
  point the packet is the plain estimator's, so the FP64 validation run
  equals, per cell and pixel, the oracle's plain run with an event cap of 1
  (which ends every packet after its first scattering peel-offs and
  truncates the same luminosity), and the non-finite count equals the
  oracle's capped count.
* The event-cap code describes the launch that returns it: a launch that
  caps nothing returns MCRT_OK even into a result whose earlier launch
  capped packets.
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


def _nan_params():
    th = scenes.init_mlp(1, scale=1.0).astype(np.float32)
    th[-1] = np.nan  # the last output bias
    return th


def _run_nan(ctx, sc, N, precision, seed):
    sim = mcrt.Sim(ctx, sc, precision)
    prop = mcrt.Proposal(ctx, params=_nan_params())
    sim.set_proposal(prop, 0.2)
    res = sim.new_result()
    rc = sim.run_into(res, N, seed=seed)
    out = {"table": res.table(), "images": res.images(), "energy": res.energy(), "stats": res.stats(), "rc": rc}
    res.close()
    sim.close()
    prop.close()
    return out


def test_nonfinite_weights_fp64_equal_capped_plain_oracle(ctx):
    sc = scenes.disk((16, 16, 8), 3, 24)
    N = 300
    say(f"nonfinite fp64 disk N={N}")
    g = _run_nan(ctx, sc, N, mcrt.FP64_VALIDATE, 5)
    capped = scenes.disk((16, 16, 8), 3, 24)
    capped.event_cap = 1
    o = oracle.run(capped, N, seed=5)
    assert g["rc"] == mcrt.ENONFINITE
    assert o["stats"]["capped"] > 0
    assert g["stats"]["nonfinite"] == o["stats"]["capped"]
    assert g["stats"]["capped"] == 0
    assert all(np.isfinite(g["table"]).ravel()) and all(np.isfinite(im).all() for im in g["images"])
    assert_fp64_parity(g, o, counters=False)
    for k in ("packets", "events", "prop_cells", "peel_adds"):
        assert g["stats"][k] == o["stats"][k], k
    e = g["energy"]
    assert abs(e[0] - e[1] - e[2] - e[3]) <= 1e-12 * e[0]


def test_nonfinite_weights_fp32_match_capped_plain(ctx):
    sc = scenes.disk((16, 16, 8), 3, 24)
    N = 4000
    say(f"nonfinite fp32 disk N={N}")
    g = _run_nan(ctx, sc, N, mcrt.FP32, 6)
    capped = scenes.disk((16, 16, 8), 3, 24)
    capped.event_cap = 1
    p = mcrt.run_scene(capped, N, seed=6, precision=mcrt.FP32, ctx=ctx)
    assert g["rc"] == mcrt.ENONFINITE
    assert g["stats"]["nonfinite"] == p["stats"]["capped"] > 0
    # same packets, same arithmetic per packet; only the order of the atomic
    # additions differs between the two kernels
    np.testing.assert_allclose(g["table"], p["table"], rtol=1e-5, atol=1e-12 * p["table"].max())
    for a, b in zip(g["images"], p["images"]):
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6 * b.max())
    e = g["energy"]
    assert abs(e[0] - e[1] - e[2] - e[3]) <= 1e-5 * e[0]


def test_event_cap_code_describes_its_own_launch(ctx):
    # a cap of 2 events and w_min = 0.3: about half the packets hit the cap
    sc = scenes.sphere(n=8, tau=1.0, albedo=0.9, g=0.3)
    sc.event_cap = 2
    sc.w_min = 0.3
    # which ids hit the cap: one-packet oracle runs
    capped = [oracle.run(sc, 64, seed=2, first_id=i, count=1)["stats"]["capped"] for i in range(64)]
    hit = [i for i in range(64) if capped[i]]
    free = [i for i in range(64) if not capped[i]]
    assert hit and free
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    res = sim.new_result()
    say("event cap code per launch")
    assert sim.run_into(res, 64, seed=2, first_id=hit[0], count=1) == mcrt.ELIMIT
    assert sim.run_into(res, 64, seed=2, first_id=free[0], count=1) == mcrt.OK
    assert res.stats()["capped"] == 1
    assert sim.run_into(res, 64, seed=2, first_id=hit[-1], count=1) == mcrt.ELIMIT
    assert res.stats()["capped"] == 2
    res.zero()
    assert sim.run_into(res, 64, seed=2, first_id=free[-1], count=1) == mcrt.OK
    res.close()
    sim.close()
