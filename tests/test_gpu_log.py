"""The run log (MCRT_LOG, MCRT_LOG_FILE) through the C-ABI.

Every timed launch appends one JSON line whose counters are what THAT
launch added (two launches into one result add up to the result's stats),
whose rates follow from its counters and its kernel time, and whose return
code is the launch's.  A batch writes one line for all its models; autotuner
trials and allocation-free launches write none; without MCRT_LOG nothing is
written.
"""
import json
import math

import pytest

from paper_1705_04702_amd import mcrt, scenes

from test_gpu_parity import say

pytestmark = pytest.mark.gpu

COUNTERS = ("packets", "events", "prop_cells", "locate_cells", "peel_cells", "peel_adds", "peel_dropped", "capped",
            "guard", "nonfinite")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = mcrt.Context(0)
    yield c
    c.close()


@pytest.fixture
def logfile(tmp_path, monkeypatch):
    path = tmp_path / "run.jsonl"
    monkeypatch.setenv("MCRT_LOG", "1")
    monkeypatch.setenv("MCRT_LOG_FILE", str(path))
    return path


def _lines(path):
    if not path.exists():
        return []
    return [json.loads(l) for l in path.read_text().splitlines()]


def _check_rates(rec, fp32):
    t = rec["kernel_ms"] * 1e-3
    assert t > 0
    nbytes = 12 * rec["prop_cells"] + 4 * (rec["locate_cells"] + rec["peel_cells"]) + \
        (4 if fp32 else 8) * rec["peel_adds"]
    assert rec["algorithmic_bytes"] == pytest.approx(nbytes, rel=1e-8)
    assert rec["packets_per_s"] == pytest.approx(rec["packets"] / t, rel=1e-6)
    assert rec["deposits_per_s"] == pytest.approx((rec["prop_cells"] + rec["peel_adds"]) / t, rel=1e-6)
    assert rec["achieved_GBps"] == pytest.approx(nbytes / t * 1e-9, rel=1e-6)
    assert rec["hbm_frac"] == pytest.approx(rec["achieved_GBps"] / 8000.0, rel=1e-6)


def test_launch_lines_carry_their_own_counters(ctx, logfile):
    sc = scenes.disk((16, 16, 8), 3, 24)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    res = sim.new_result()
    say("run log: two launches into one result")
    sim.run_into(res, 1000, seed=4, first_id=0, count=600)
    sim.run_into(res, 1000, seed=4, first_id=600, count=400)
    st = res.stats()
    recs = _lines(logfile)
    assert [r["entry"] for r in recs] == ["run_into", "run_into"]
    a, b = recs
    assert (a["first_id"], a["count"], b["first_id"], b["count"]) == (0, 600, 600, 400)
    assert a["packets"] == 600 * 3 and b["packets"] == 400 * 3
    for k in COUNTERS:
        assert a[k] + b[k] == st[k], k
    assert b["kernel_ms"] == pytest.approx(st["kernel_ms"], rel=1e-6)
    for r in recs:
        assert (r["grid"], r["cells"], r["n_lambda"], r["instruments"]) == ("cartesian", 16 * 16 * 8, 3, len(sc.instruments))
        assert (r["precision"], r["learned"], r["models"], r["rc"], r["seed"]) == ("fp32", False, 1, mcrt.OK, 4)
        _check_rates(r, fp32=True)
    res.close()
    sim.close()


def test_octree_fp64_and_event_cap_code(ctx, logfile):
    tor = scenes.torus(4, 3, 1, 8, n_clumps=5)
    sim = mcrt.Sim(ctx, tor, mcrt.FP64_VALIDATE)
    res = sim.run(200, seed=1)
    st = res.stats()
    rec = _lines(logfile)[-1]
    assert (rec["grid"], rec["precision"], rec["count"], rec["n_per_lambda"]) == ("octree", "fp64", 200, 200)
    for k in COUNTERS:
        assert rec[k] == st[k], k
    _check_rates(rec, fp32=False)
    sim.close()
    # a launch that hits the event cap logs MCRT_ELIMIT
    sph = scenes.sphere(n=8, tau=1.0, albedo=0.9, g=0.3)
    sph.event_cap = 2
    sph.w_min = 0.3
    sim = mcrt.Sim(ctx, sph, mcrt.FP64_VALIDATE)
    res = sim.new_result()
    rc = sim.run_into(res, 64, seed=2)
    rec = _lines(logfile)[-1]
    assert rc == mcrt.ELIMIT and rec["rc"] == mcrt.ELIMIT and rec["capped"] == res.stats()["capped"] > 0
    res.close()
    sim.close()


def test_batch_line_tuner_and_noalloc_silence(ctx, logfile, monkeypatch):
    models = [scenes.sphere(n=8, npix=16), scenes.disk((16, 16, 8), 2, 16)]
    sims = [mcrt.Sim(ctx, m, mcrt.FP32) for m in models]
    res = [s.new_result() for s in sims]
    say("run log: batch, autotune, noalloc")
    mcrt.batch_run_into(sims, res, [300, 200], seed=5)
    recs = _lines(logfile)
    assert len(recs) == 1 and recs[0]["entry"] == "batch_run_into"
    rec = recs[0]
    assert rec["models"] == 2 and rec["n_lambda"] == 1 + 2
    assert rec["cells"] == 8 ** 3 + 16 * 16 * 8
    assert rec["packets"] == 300 + 2 * 200 == rec["count"]
    sts = [r.stats() for r in res]
    for k in COUNTERS:
        assert rec[k] == sum(s[k] for s in sts), k
    _check_rates(rec, fp32=True)
    mcrt.autotune(sims, [50, 50], seed=5)
    assert len(_lines(logfile)) == 1
    r1 = sims[0].new_result()
    sims[0].run_into_noalloc(r1, 100, seed=1)
    assert len(_lines(logfile)) == 1
    monkeypatch.delenv("MCRT_LOG")
    sims[0].run_into(r1, 100, seed=2)
    assert len(_lines(logfile)) == 1
    monkeypatch.setenv("MCRT_LOG", "0")
    sims[0].run_into(r1, 100, seed=3)
    assert len(_lines(logfile)) == 1
    for r in res + [r1]:
        r.close()
    for s in sims:
        s.close()
    assert not math.isnan(rec["hbm_frac"])
