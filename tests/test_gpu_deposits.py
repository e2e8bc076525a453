"""Every FP32 deposit reaches the table exactly once, through the C-ABI.

A deposit's FP32 value converts exactly to FP64, and the lane adds the same
value to its FP64 absorbed-energy tally; the tallies are summed per wave and
the table entries by FP64 atomics.  So over a whole run the table's sum
equals the absorbed energy up to the order of FP64 additions (about
1e-16 sqrt(additions) relative; 1e-10 allowed), whatever the deposit path:
held runs (Cartesian), flushes every other iteration (octree, learned
octree, batch), loop exits at any iteration (the queue threshold and chunk
move them).  A deposit lost or issued twice at a flush would move the sum
by far more (one deposit is ~1e-7 of the total here).
"""
import numpy as np
import pytest

from paper_1705_04702_amd import mcrt, scenes

from test_gpu_parity import say

pytestmark = pytest.mark.gpu

TUNINGS = [dict(), dict(chunk=16, threshold=4, waves_per_cu=4), dict(chunk=512, threshold=48, waves_per_cu=16)]
# the batch kernel's two deposit tiles: 8 slots per lane issued every march
# iteration, 16 every other one
BATCH_TUNINGS = TUNINGS + [dict(deposit_slots=8), dict(deposit_slots=8, chunk=16, threshold=4, waves_per_cu=4)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = mcrt.Context(0)
    yield c
    c.close()


def _check(res, what):
    T = res.table()
    e = res.energy()
    st = res.stats()
    say(f"{what}: table sum {T.sum():.17g}, absorbed {e[1]:.17g}, packets {st['packets']}")
    assert st["packets"] > 0 and e[1] > 0
    assert abs(T.sum() - e[1]) <= 1e-10 * e[1], what


SCENES = {
    "disk": (lambda: scenes.disk((64, 64, 32), 8, 32), 20000),
    "torus": (lambda: scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0), 20000),
}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("tune", range(len(TUNINGS)))
def test_fp32_table_sum_equals_absorbed(ctx, name, tune):
    make, N = SCENES[name]
    sim = mcrt.Sim(ctx, make(), mcrt.FP32, **TUNINGS[tune])
    res = sim.new_result()
    sim.run_into(res, N, seed=3, first_id=0, count=N // 2)
    sim.run_into(res, N, seed=3, first_id=N // 2, count=N - N // 2)
    _check(res, f"{name} {TUNINGS[tune]}")
    res.close()
    sim.close()


@pytest.mark.parametrize("tune", range(len(TUNINGS)))
def test_fp32_learned_octree_table_sum_equals_absorbed(ctx, tune):
    sc = scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32, **TUNINGS[tune])
    prop = mcrt.Proposal(ctx, params=scenes.init_mlp(2, scale=1.0).astype(np.float32))
    sim.set_proposal(prop, 0.2)
    res = sim.new_result()
    sim.run_into(res, 20000, seed=4)
    _check(res, f"learned torus {TUNINGS[tune]}")
    res.close()
    sim.close()
    prop.close()


@pytest.mark.parametrize("tune", range(len(BATCH_TUNINGS)))
def test_fp32_batch_table_sums_equal_absorbed(ctx, tune):
    models = scenes.batch(256, seed=4)[::32]
    sims = [mcrt.Sim(ctx, m.scene, mcrt.FP32, **BATCH_TUNINGS[tune]) for m in models]
    res = [s.new_result() for s in sims]
    mcrt.batch_run_into(sims, res, [5000] * len(sims), seed=6)
    for i, r in enumerate(res):
        _check(r, f"batch model {i} {BATCH_TUNINGS[tune]}")
        r.close()
    for s in sims:
        s.close()
