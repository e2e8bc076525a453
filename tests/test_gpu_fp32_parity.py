"""FP32 production mode against the FP64 oracle, cell by cell and pixel by
pixel, at the production layouts of every workload, with the error stated
per result.

The FP32 kernels draw the same random numbers as the oracle, so most packets
follow the oracle's path exactly and differ by rounding; a packet whose
decision sits on a rounding edge (a cell boundary, the termination
threshold, the interaction segment, a bf16 activation of the network) takes
another path.  The bar is the Monte Carlo one: on cells and pixels with at
least 10 effective contributions (T^2 / sum of squared per-packet
contributions), at most 0.5 % may differ from the oracle by more than 3
sigma plus an FP32 arithmetic allowance of 1e-3 |T| (which only matters
where sigma vanishes), sigma^2 = sum_p s_p^2 - T^2 / N from the oracle's
per-packet second moments; result totals within 1e-4 (images) or 1e-5 (tables) relative plus
3 sigma; energy balance 1e-5.  Every result's maximum, 99th-percentile and
median relative error (over the selected entries) and its total's relative
error are printed as a JSON line tagged [fp32-err] (and appended to the file
named by MCRT_FP32_REPORT, if set).

Workloads: the exponential disk at its full 256^3 grid with all three 512^2
instruments (face-on and edge-on read column maps, 60 deg marches), on 4 of
its wavelengths; the clumpy torus at full size (2.24e6 leaves, 1024^2) on 8
of its wavelengths; a subset of the 256-model batch in one batched launch;
the learned proposal (MFMA network) on the full torus against the oracle's
FP64 network with the same parameters; the learned proposal's Cartesian kernel on a
disk; history-recording runs (training data collection) on a disk and a
torus; dust packets of a disk (the dust emission phase) emitted from the
same absorption as the oracle's.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import oracle_par
from paper_1705_04702_amd import mcrt, scenes

from test_gpu_parity import say

pytestmark = pytest.mark.gpu

NEFF_MIN = 10.0
# FP32 arithmetic allowance, for entries whose Monte Carlo sigma vanishes (a
# point source's emission peel-off adds the same value for every packet).
# Such an entry differs from the oracle only by FP32 rounding: its optical
# depth summed over n cells carries at most (n + 3) 2^-24 tau (about 8e-4 for
# the torus's ~250-cell edge-on ray at tau ~ 50), and its k atomic additions
# (a wave's 64 adds are combined first) at most k 2^-24 (2e-5 for 20000
# packets).
FP32_ALLOWANCE = 1e-3


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = mcrt.Context(0)
    yield c
    c.close()


def _errors(name, a, T, m2, N, sum_tol):
    """Checks one result (FP32 a against oracle T with moments m2) and
    returns its error record."""
    a = np.asarray(a, dtype=np.float64)
    var = np.maximum(m2 - T * T / N, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        neff = np.where(m2 > 0, T * T / np.where(m2 > 0, m2, 1.0), 0.0)
    sel = neff >= NEFF_MIN
    rec = {"result": name, "entries": int(T.size), "nonzero": int(np.count_nonzero(T)), "selected": int(sel.sum())}
    tot_sig = math.sqrt(var.sum())
    rec["total_rel_err"] = float(abs(a.sum() - T.sum()) / abs(T.sum())) if T.sum() else 0.0
    rec["total_sigma_rel"] = float(tot_sig / abs(T.sum())) if T.sum() else 0.0
    assert abs(a.sum() - T.sum()) <= sum_tol * abs(T.sum()) + 3.0 * tot_sig, (name, rec)
    if sel.any():
        d = np.abs(a[sel] - T[sel])
        rel = d / np.abs(T[sel])
        beyond = d > 3.0 * np.sqrt(var[sel]) + FP32_ALLOWANCE * np.abs(T[sel])
        worst = np.argsort(-(d / (3.0 * np.sqrt(var[sel]) + FP32_ALLOWANCE * np.abs(T[sel]))))[:3]
        rec["worst"] = [dict(rel=float(rel[w]), sigma_rel=float(np.sqrt(var[sel][w]) / abs(T[sel][w])),
                             neff=float(neff[sel][w])) for w in worst]
        rec.update(frac_beyond_3sigma=float(beyond.mean()), max_rel_err=float(rel.max()),
                   p99_rel_err=float(np.quantile(rel, 0.99)), median_rel_err=float(np.median(rel)))
        assert beyond.mean() <= 0.005, (name, rec)
    nz = T != 0
    if nz.any():
        rel_all = np.abs(a[nz] - T[nz]) / np.abs(T[nz])
        rec["median_rel_err_all_nonzero"] = float(np.median(rel_all))
    # entries the oracle leaves at zero: the FP32 run may only add there what
    # a packet that diverged on a rounding edge deposits
    rec["fp32_only_nonzero"] = int(np.count_nonzero(a[~nz]))
    return rec


def report(workload, g, o, N, extra=None, balance_tol=1e-5, below=None, zero=None):
    """below: wavelengths whose packet luminosity is below FP32's normal
    range, left out of the comparison with the oracle; zero: those among
    them whose packet luminosity rounds to 0 in FP32, which the FP32 run must
    leave exactly zero."""
    e = g["energy"]
    bal = abs(e[0] - e[1] - e[2] - e[3]) / e[0]
    assert bal < balance_tol
    keep = np.ones(o["table"].shape[1], bool)
    if below is not None:
        keep = ~np.asarray(below)
    if zero is not None:
        zero = np.asarray(zero)
        assert not g["table"][:, zero].any()
        for a in g["images"]:
            assert not a[zero].any()
    recs = [_errors("table", g["table"][:, keep], o["table"][:, keep], o["table_m2"][:, keep], N, 1e-5)]
    for j, (a, T, m2) in enumerate(zip(g["images"], o["images"], o["image_m2"])):
        recs.append(_errors(f"image{j}", a[keep], T[keep], m2[keep], N, 1e-4))
    line = {"workload": workload, "packets_per_lambda": N, "energy_balance": bal,
            "absorbed_rel_err": float(abs(e[1] - o["energy"][1]) / o["energy"][1]), "results": recs}
    if below is not None:
        line["wavelengths_below_fp32_range"] = [int(l) for l in np.nonzero(~keep)[0]]
    if extra:
        line.update(extra)
    say("[fp32-err] " + json.dumps(line))
    path = os.environ.get("MCRT_FP32_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(line) + "\n")
    return line


def _gpu(ctx, sc, N, seed, precision=mcrt.FP32, theta=None):
    sim = mcrt.Sim(ctx, sc, precision)
    prop = None
    if theta is not None:
        prop = mcrt.Proposal(ctx, params=theta)
        sim.set_proposal(prop, 0.2)
    res = sim.new_result()
    sim.run_into(res, N, seed=seed)
    out = {"table": res.table(), "images": res.images(), "energy": res.energy(), "stats": res.stats()}
    res.close()
    sim.close()
    if prop is not None:
        prop.close()
    return out


def test_sphere_c1_fp32_per_cell_and_pixel(ctx):
    """The uniform sphere (tau 1, albedo 0.5, g 0.5, 32^3, 64^2) with its
    full 1e5 packets, seed 0."""
    sc = scenes.sphere()
    N = 100_000
    say(f"fp32 parity sphere 32^3, {N} packets")
    g = _gpu(ctx, sc, N, seed=0)
    o = oracle_par.run(sc, N, seed=0, moments=True)
    report("sphere 32^3, 64^2, 1e5 packets", g, o, N)


def test_disk_full_grid_fp32_per_cell_and_pixel(ctx):
    sc = oracle_par.subset_lambdas(scenes.disk(), [0, 21, 42, 63])
    N = 50_000
    say(f"fp32 parity disk 256^3, 4 wavelengths, {N} ids each")
    g = _gpu(ctx, sc, N, seed=11)
    o = oracle_par.run(sc, N, seed=11, moments=True, threads=8)
    report("disk 256^3, 3 x 512^2 (i = 0/60/90), wavelengths 0/21/42/63 of 64", g, o, N)


def test_torus_full_size_fp32_per_cell_and_pixel(ctx):
    sc = oracle_par.subset_lambdas(scenes.torus(), list(range(0, 32, 4)))
    N = 20_000
    say(f"fp32 parity torus full size, 8 wavelengths, {N} ids each")
    g = _gpu(ctx, sc, N, seed=12)
    o = oracle_par.run(sc, N, seed=12, moments=True)
    report("torus 2.24e6 leaves, 1024^2 edge-on, wavelengths 0, 4, ..., 28 of 32", g, o, N)


def test_batch_fp32_per_cell_and_pixel(ctx):
    """Every 16th model of the 256-model table (sides 16-128, tau 0.1-20,
    spheres and slabs), 20000 packets each, in one batched FP32 launch; the
    model index (the fourth Philox word) is the position in this batch."""
    models = scenes.batch(256, seed=4)[::16]
    N = 20_000
    sims = [mcrt.Sim(ctx, m.scene, mcrt.FP32) for m in models]
    res = [s.new_result() for s in sims]
    say(f"fp32 parity batch of {len(models)} models, {N} packets each")
    mcrt.batch_run_into(sims, res, [N] * len(models), seed=13)
    for i, (m, r) in enumerate(zip(models, res)):
        g = {"table": r.table(), "images": r.images(), "energy": r.energy()}
        o = oracle_par.run(m.scene, N, seed=13, model=i, moments=True)
        report(f"batch model {i} ({m.scene.name}, tau {m.tau:.3g})", g, o, N)
    for r in res:
        r.close()
    for s in sims:
        s.close()


def _learned_params(seed):
    from oracle import learned as L
    th = scenes.init_mlp(seed, scale=1.5).astype(np.float64)
    p = L.unpack(th)
    rng = np.random.default_rng(seed + 100)
    for b in ("b1", "b2", "b3"):
        p[b] = rng.normal(scale=0.1, size=p[b].shape)
    return L.pack(p).astype(np.float32)


def test_learned_torus_fp32_per_cell_and_pixel(ctx):
    """The learned proposal in FP32 (network on the matrix cores, bf16 weights
    and activations, FP32 sums) against the oracle's FP64 network with the
    same parameters, on the full torus: per cell and pixel at 3 sigma of the
    learned estimator's own noise (the oracle's moments of the learned run)."""
    sc = oracle_par.subset_lambdas(scenes.torus(), [0, 10, 21, 31])
    N = 20_000
    theta = _learned_params(11)
    say(f"fp32 parity learned torus full size, 4 wavelengths, {N} ids each")
    g = _gpu(ctx, sc, N, seed=14, theta=theta)
    o = oracle_par.run(sc, N, seed=14, moments=True, mlp=theta)
    # the weights W = p/q conserve energy in expectation only (E[W] = 1)
    eo = o["energy"]
    report("learned torus 2.24e6 leaves, 1024^2, wavelengths 0/10/21/31 of 32", g, o, N, balance_tol=0.05,
           extra={"learned_energy_balance_oracle": float(abs(eo[0] - eo[1] - eo[2] - eo[3]) / eo[0])})


DUST = {
    # scene, dust parameters (T0, beta), label
    "disk": (lambda: scenes.disk(n=(32, 32, 16), n_lambda=6, npix=32, tau_v_faceon=5.0), (20.0, 2.0),
             "dust packets of the disk 32x32x16 (emission from 2000 stellar ids per wavelength), 6 wavelengths"),
    "torus": (lambda: scenes.torus(5, 4, 4, 16, n_clumps=20), (30.0, 1.8),
              "dust packets of a clumpy torus (octree leaves; emission from 2000 stellar ids per wavelength)"),
}


@pytest.mark.parametrize("name", list(DUST))
def test_dust_packets_fp32_per_cell_and_pixel(ctx, name):
    """Dust packets in FP32 against the oracle's dust packets, cell by cell
    and pixel by pixel (Cartesian cells and octree leaves): both emit from
    the same absorption -- the oracle's stellar run and the GPU's FP64
    validation run of the same scene, which match to 1e-9 -- so the FP32
    sim's dust object is built from the FP64 sim's result (same table
    layout), and both draw the same dust packets."""
    make, (T0, beta), label = DUST[name]
    sc = make()
    N_star, N = 2000, 20_000
    sim64 = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    sim32 = mcrt.Sim(ctx, sc, mcrt.FP32)
    say(f"fp32 parity dust packets, {name}, {N} ids each")
    st = sim64.run(N_star, seed=1)
    d = sim32.dust([st], T0=T0, beta=beta)
    r = sim32.run_dust(d, N, seed=9)
    g = {"table": r.table(), "images": r.images(), "energy": r.energy()}
    o = oracle_par.run(sc, N_star, seed=1)
    _, em = oracle.dust_emission(sc, o["table"], T0=T0, beta=beta)
    np.testing.assert_allclose(d.luminosity(), em.sum(axis=0), rtol=1e-9, atol=0)
    od = oracle_par.run(oracle.dust_scene(sc, em), N, seed=9, moments=True)
    # the Wien tail of the cold dust: on the disk, wavelength 2 (4 um) emits
    # ~1e-56 in all, ~7e-61 per packet, which FP32 cannot hold (the two
    # shortest emit exactly nothing)
    lpp = em.sum(axis=0) / N
    below = lpp < np.finfo(np.float32).tiny
    zero = lpp < 2.0 ** -150  # rounds to 0 in FP32
    assert not below.all()
    if name == "disk":
        assert zero.any()
    report(label, g, od, N, below=below, zero=zero)
    for h in (d, r, st):
        h.close()
    sim32.close()
    sim64.close()


def test_learned_disk_fp32_per_cell_and_pixel(ctx):
    """The learned proposal's Cartesian FP32 kernel (the torus test above
    covers the octree one) on a disk with all three instruments (two column
    maps, one marched), against the oracle's FP64 network with the same
    parameters, per cell and pixel at 3 sigma of the learned run's noise."""
    sc = scenes.disk(n=(32, 32, 16), n_lambda=4, npix=32)
    N = 20_000
    theta = _learned_params(11)
    say(f"fp32 parity learned disk 32x32x16, 4 wavelengths, {N} ids each")
    g = _gpu(ctx, sc, N, seed=15, theta=theta)
    o = oracle_par.run(sc, N, seed=15, moments=True, mlp=theta)
    eo = o["energy"]
    report("learned disk 32x32x16, 3 x 32^2 (i = 0/60/90), 4 wavelengths", g, o, N, balance_tol=0.05,
           extra={"learned_energy_balance_oracle": float(abs(eo[0] - eo[1] - eo[2] - eo[3]) / eo[0])})


@pytest.mark.parametrize("name", ["disk", "torus"])
def test_history_runs_fp32_per_cell_and_pixel(ctx, name):
    """A history-recording run (the training data collection) is the plain
    estimator run by the kernels' history variants (Cartesian: held deposit
    runs; octree: flushes every other iteration): its FP32 table and images
    against the oracle's plain run, per cell and pixel."""
    if name == "disk":
        sc = scenes.disk(n=(32, 32, 16), n_lambda=4, npix=32)
    else:
        sc = scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0)
    N = 20_000
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    res = sim.new_result()
    say(f"fp32 parity history run {name}, {N} ids per wavelength")
    h = sim.collect(res, N, seed=16, max_events=16)
    g = {"table": res.table(), "images": res.images(), "energy": res.energy()}
    o = oracle_par.run(sc, N, seed=16, moments=True)
    report(f"history-recording run, {name} ({sc.name})", g, o, N)
    h.close()
    res.close()
    sim.close()
