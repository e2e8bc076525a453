"""Throughput benchmark of the photon-packet life cycle on one MI355X.

Workload (default): the exponential-disk galaxy -- 256^3 Cartesian grid, 64
log-spaced wavelengths 0.1-1000 um with power-law opacity and albedo, three
512^2 instruments at inclinations 0/60/90 deg, 1e7 packets per wavelength,
FP32 transport with FP64 table totals.  One step runs one contiguous block of
packet ids of every wavelength (run_into: the blocks of consecutive steps add
up to the whole job); the timed region holds exactly K steps with the scene
already resident in HBM.

Prints ONE JSON line with packets/s, the roofline of the transport kernel
(algorithmic bytes from the kernel's own cell/pixel counters over its HIP-event
duration, against 8 TB/s HBM) and the FP64 CPU oracle timed on the host cores
on a bounded sample; then the metric's second half, the image RMS error x
time of the learned direction proposal against the plain sampler on the
clumpy torus (learned_vs_plain; --no-learned skips it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packets/s on 1 MI355X; image RMS err x time, learned vs plain"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per unit (FP32 production mode)
B_PROP = 4 + 8      # density read + FP64 atomic payload per propagation cell
B_LOCATE = 4        # density read per cell of the interaction search
B_PEEL = 4          # density read per peel-off cell
B_PIXEL = 4         # FP32 pixel atomic payload


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_04702_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith("transport") or f in ("internal.h", "det_math.h", "proposal.h"):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st: dict) -> int:
    return (B_PROP * st["prop_cells"] + B_LOCATE * st["locate_cells"] + B_PEEL * st["peel_cells"]
            + B_PIXEL * st["peel_adds"])


WORKLOADS = {
    # name: (packets per wavelength of the whole job, description)
    "disk": (10_000_000, "exponential-disk galaxy: 256^3 Cartesian grid, 64 wavelengths 0.1-1000 um, "
                         "3 x 512^2 instruments (i = 0/60/90 deg), 1e7 packets per wavelength, "
                         "FP32 transport, FP64 table totals"),
    "sphere": (100_000, "uniform sphere tau=1, albedo 0.5, g=0.5: 32^3 grid, 1 wavelength, "
                        "64^2 instrument at 100 radii, 1e5 packets"),
    "torus": (3_125_000, "clumpy AGN torus: octree (~2.2e6 leaves, depth 9), 3% clumps of 0.4 pc, "
                         "contrast 100, equatorial tau_V=50, anisotropic source, 32 wavelengths, "
                         "1e8 packets, 1024^2 edge-on instrument"),
}


def make_scene(name: str):
    from paper_1705_04702_amd import scenes
    if name == "disk":
        return scenes.disk(), WORKLOADS[name][1]
    if name == "sphere":
        return scenes.sphere(), WORKLOADS[name][1]
    if name == "torus":
        return scenes.torus(), WORKLOADS[name][1]
    raise SystemExit(f"unknown workload {name}")


def bench_batch(args):
    """256 uneven uniform-sphere / exponential-slab models (16^3 .. 128^3,
    1e5 .. 1e7 packets each, 128^2 images) in one persistent launch per step,
    with the queue tuned by the library's autotuner first (cached by problem
    class; --no-autotune keeps the defaults)."""
    import torch
    from paper_1705_04702_amd import mcrt, scenes
    models = scenes.batch(256, seed=4)
    if args.tau_peel_max is not None:
        for m in models:
            m.scene.tau_peel_max = args.tau_peel_max
    ctx = mcrt.Context(0)
    order = {"cost": mcrt.QUEUE_COST, "caller": mcrt.QUEUE_CALLER, "paired": mcrt.QUEUE_PAIRED}[args.queue_order]
    sims = [mcrt.Sim(ctx, m.scene, mcrt.FP32, chunk=args.chunk or None, waves_per_cu=args.waves_per_cu or None,
                     threshold=args.threshold or None, queue_order=order) for m in models]
    npl = [m.n_packets for m in models]
    tuning = None
    if not args.no_autotune:
        # trials of an eighth of every model's packets: the shape of the full
        # launch (its tail weighs more in a short trial)
        tuning = mcrt.autotune(sims, [max(1, n // 8) for n in npl], seed=0,
                               cache_path=os.path.join(ROOT, "_build", "tune_cache.txt"))
        print(f"[bench] autotune {tuning}", file=sys.stderr, flush=True)
    res = [s.new_result() for s in sims]
    for w in range(args.warmup):
        mcrt.batch_run_into(sims, res, npl, seed=0)
    for r in res:
        r.zero()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for k in range(args.steps):
        mcrt.batch_run_into(sims, res, npl, seed=0)
        kms.append(res[0].stats()["kernel_ms"])
        print(f"[bench] batch step {k}: kernel {kms[-1]:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    packets = sum(npl) * args.steps
    worst = max(abs(e[0] - e[1] - e[2] - e[3]) / e[0] for e in (r.energy() for r in res))
    sts = [r.stats() for r in res]
    deposits = sum(s["prop_cells"] for s in sts) / args.steps
    out = {"metric": METRIC, "value": packets / T, "unit": "packets/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": T / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch of 256 uniform-sphere / exponential-slab models, grids 16^3-128^3 "
                                  "log-uniform, tau 0.1-20, packets 1e5-1e7 each (total %d), 128^2 images, "
                                  "one persistent launch" % sum(npl), "models": 256,
                      "queue_order": args.queue_order},
           "kernel_ms_avg": sum(kms) / len(kms), "energy_balance_worst": worst,
           "atomics_per_s": deposits / (sum(kms) / len(kms) / 1e3), "tuning": tuning,
           "counters_per_packet": {f: sum(s[f] for s in sts) / max(sum(s["packets"] for s in sts), 1)
                                   for f in ("events", "prop_cells", "locate_cells", "peel_cells", "peel_adds")}}
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)


def bench_dust(args):
    """Dust emission phase on the disk: one stellar launch (1e6 packets per
    wavelength), the dust emission computed from its absorption, then timed
    launches of dust packets of the same size; plus two self-absorption
    cycles at 1e5 packets per wavelength."""
    import numpy as np
    import torch
    from paper_1705_04702_amd import mcrt, scenes
    scene = scenes.disk()
    if args.tau_peel_max is not None:
        scene.tau_peel_max = args.tau_peel_max
    N = WORKLOADS["disk"][0]
    B = min(args.step_packets, N)
    nl = scene.n_lambda
    ctx = mcrt.Context(0)
    sim = mcrt.Sim(ctx, scene, mcrt.FP32)
    stellar = sim.new_result()
    sim.run_into(stellar, N, seed=0, first_id=0, count=B)
    torch.cuda.synchronize()
    print("[bench] stellar launch done", file=sys.stderr, flush=True)
    t = time.perf_counter()
    dust = sim.dust([stellar])
    create_s = time.perf_counter() - t
    L = dust.luminosity()
    T = dust.temperature()
    res = sim.new_result()
    for w in range(args.warmup):
        sim.run_dust_into(dust, res, N, seed=1, first_id=w * B % N, count=B)
    res.zero()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        sim.run_dust_into(dust, res, N, seed=1, first_id=(k * B) % N, count=B)
        kms.append(res.stats()["kernel_ms"])
        print(f"[bench] dust step {k}: kernel {kms[-1]:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    Tt = time.perf_counter() - t0
    e = res.energy()
    st = res.stats()
    packets = B * nl * args.steps
    per = {f: st[f] / max(st["packets"], 1) for f in ("events", "prop_cells", "locate_cells", "peel_cells",
                                                     "peel_adds")}
    achieved = (algorithmic_bytes({f: st[f] for f in mcrt.STAT_FIELDS}) / args.steps
                / (sum(kms) / len(kms) / 1e3) / 1e9)
    t = time.perf_counter()
    d2, r2, cycles = sim.self_absorption(stellar, 100_000, seed=2, max_cycles=2, tol=0.0)
    sa_s = time.perf_counter() - t
    L2 = d2.luminosity()
    out = {"metric": "dust photon packets/s on 1 MI355X", "value": packets / Tt, "unit": "packets/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": Tt / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 emission)",
           "data": "synthetic",
           "config": {"workload": "dust emission phase of the exponential-disk galaxy (256^3, 64 wavelengths, "
                                  "3 x 512^2 instruments): emission from one stellar launch of %d packets, "
                                  "modified blackbody T0 = 20 K, beta = 2" % (B * nl),
                      "packets_per_step": B * nl},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None},
           "kernel_ms_avg": sum(kms) / len(kms),
           "dust_create_ms": create_s * 1e3,
           "dust_luminosity": float(L.sum()), "stellar_absorbed": float(stellar.table().sum()),
           "temperature_K": {"median": float(np.median(T[T > 0])), "max": float(T.max())},
           "energy_balance": abs(e[0] - e[1] - e[2] - e[3]) / e[0],
           "counters_per_packet": per,
           "self_absorption": {"cycles": cycles, "packets_per_lambda": 100_000, "seconds": sa_s,
                               "dust_luminosity_first_cycle": float(L.sum()),
                               "dust_luminosity_last_cycle": float(L2.sum())}}
    sim.close()
    print(json.dumps(out), flush=True)


def _image_cube(res, n_ins):
    import numpy as np
    return np.concatenate([res.image(j).ravel() for j in range(n_ins)])


def learned_vs_plain(args):
    """Learned direction proposal on the clumpy-torus workload: collect plain
    histories (1e7 packets, seed 1), train the network (Adam, lr 1e-3), then
    compare the image error of a learned run (1e8 packets, seed 2) with a
    plain run of equal transport time (seed 3), both against a plain
    reference of 1e9 packets (seed 4).  RMS = sqrt(sum (I - I_ref)^2) /
    sqrt(sum I_ref^2) over all pixels and wavelengths, with the reference's
    own noise (from its two halves) subtracted; figure of merit 1 / (RMS^2 t)
    with t the transport time.  Collection and training are reported
    separately.  Returns (learned packets/s, learned seconds, the comparison,
    the configuration)."""
    import numpy as np
    import torch
    from paper_1705_04702_amd import mcrt, scenes
    sc = scenes.torus()
    if args.tau_peel_max is not None:
        sc.tau_peel_max = args.tau_peel_max
    nl = sc.n_lambda
    n_hist = args.hist_packets // nl
    n_learn = args.learned_packets // nl
    n_ref = args.ref_packets // nl
    ctx = mcrt.Context(0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    n_ins = len(sc.instruments)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    def log(msg):
        print(f"[bench-learned] {msg}", file=sys.stderr, flush=True)

    # 1. histories of plain packets
    r_hist = sim.new_result()
    hist, t_collect = timed(lambda: sim.collect(r_hist, n_hist, seed=1, max_events=args.max_events))
    log(f"collected {hist.n_packets} packets, {hist.n_samples} samples in {t_collect:.2f} s")
    r_hist.close()
    # 2. training
    prop = mcrt.Proposal(ctx, seed=7, init_scale=1.0)
    loss0 = prop.eval(hist)
    _, t_train = timed(lambda: prop.train(hist, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=3))
    loss1 = prop.eval(hist)
    log(f"trained {args.epochs} epochs in {t_train:.2f} s: loss {loss0:.4f} -> {loss1:.4f}")
    hist.close()

    def run(n_per_lambda, seed, learned, first=0, count=None):
        """Runs ids [first, first + count) in blocks; returns the image cube and
        the summed kernel time."""
        count = n_per_lambda - first if count is None else count
        sim.set_proposal(prop if learned else None, args.alpha)
        res = sim.new_result()
        block = 3_000_000
        kms = 0.0
        for b0 in range(first, first + count, block):
            cnt = min(block, first + count - b0)
            sim.run_into(res, n_per_lambda, seed=seed, first_id=b0, count=cnt)
            kms = res.stats()["kernel_ms"] + kms
            log(f"{'learned' if learned else 'plain'} ids [{b0}, {b0 + cnt}) of {n_per_lambda}/lambda done")
        img = _image_cube(res, n_ins)
        e = res.energy()
        st = res.stats()
        res.close()
        per = {f: st[f] / max(st["packets"], 1) for f in ("events", "prop_cells", "locate_cells", "peel_cells",
                                                          "peel_adds")}
        counters[("learned" if learned else "plain")] = per
        return img, kms / 1e3, e

    counters = {}

    # 3. reference in two halves, learned run, plain run of equal transport time
    half = n_ref // 2
    ref_a, t_ra, _ = run(n_ref, 4, False, 0, half)
    ref_b, t_rb, _ = run(n_ref, 4, False, half, n_ref - half)
    ref = ref_a + ref_b
    t_ref = t_ra + t_rb
    learned, t_learned, e_learned = run(n_learn, 2, True)
    plain_rate = n_ref * nl / t_ref
    n_plain = max(1, int(plain_rate * t_learned / nl))
    plain, t_plain, _ = run(n_plain, 3, False)
    ref2 = float(np.sum(ref * ref))
    noise = float(np.sum((ref_a - ref_b) ** 2))  # estimates the reference's own variance sum
    rms_l = float(np.sqrt(max(np.sum((learned - ref) ** 2) - noise, 0.0) / ref2))
    rms_p = float(np.sqrt(max(np.sum((plain - ref) ** 2) - noise, 0.0) / ref2))
    fom_l = 1.0 / (rms_l ** 2 * t_learned)
    fom_p = 1.0 / (rms_p ** 2 * t_plain)
    tot_l, tot_p, tot_r = float(learned.sum()), float(plain.sum()), float(ref.sum())
    log(f"rms learned {rms_l:.4e} ({t_learned:.2f} s), plain {rms_p:.4e} ({t_plain:.2f} s), "
        f"gain {fom_l / fom_p:.3f}")
    config = {"workload": "clumpy AGN torus (octree ~2.2e6 leaves, 32 wavelengths, 1024^2 edge-on "
                          "instrument) with the learned vMF-mixture direction proposal",
              "history_packets": n_hist * nl, "learned_packets": n_learn * nl,
              "reference_packets": n_ref * nl, "plain_packets_equal_time": n_plain * nl,
              "alpha": args.alpha, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
              "max_events": args.max_events, "tau_peel_max": sc.tau_peel_max}
    cmp = {"rms_learned": rms_l, "rms_plain": rms_p, "t_learned_s": t_learned,
           "t_plain_s": t_plain, "rms2_t_learned": rms_l ** 2 * t_learned,
           "rms2_t_plain": rms_p ** 2 * t_plain, "fom_gain": fom_l / fom_p,
           "fom_gain_with_training": (rms_p ** 2 * t_plain) / (rms_l ** 2 * (t_learned + t_collect + t_train)),
           "flux_learned_over_ref": tot_l / tot_r, "flux_plain_over_ref": tot_p / tot_r,
           "reference_noise_fraction": noise / ref2,
           "collect_s": t_collect, "train_s": t_train, "loss_before": loss0,
           "loss_after": loss1, "counters_per_packet": counters,
           "energy_balance_learned":
               abs(e_learned[0] - e_learned[1] - e_learned[2] - e_learned[3]) / e_learned[0],
           "workload": config["workload"], "history_packets": n_hist * nl, "learned_packets": n_learn * nl,
           "reference_packets": n_ref * nl, "plain_packets_equal_time": n_plain * nl,
           "alpha": args.alpha, "epochs": args.epochs}
    prop.close()
    sim.close()
    return n_learn * nl / t_learned, t_learned, cmp, config


def bench_learned(args):
    """The learned-proposal workload on its own: value = learned packets/s."""
    rate, t_learned, cmp, config = learned_vs_plain(args)
    out = {"metric": METRIC, "value": rate, "unit": "packets/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": t_learned * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
           "config": config, "learned_vs_plain": cmp}
    print(json.dumps(out), flush=True)


def bench_curve(args, scene, workload, N):
    """Throughput against the packets of one launch (1e4 .. the full run): the
    fixed launch and tail costs amortised over more packets.  Each point is
    the median of 3 launches after one warm-up launch of the same size."""
    import torch
    from paper_1705_04702_amd import mcrt
    ctx = mcrt.Context(0)
    sim = mcrt.Sim(ctx, scene, mcrt.FP32)
    nl = scene.n_lambda
    full = N * nl
    totals = [t for t in (10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7, 10 ** 8) if t < full] + [full]
    rows = []
    for tot in totals:
        cnt = max(1, tot // nl)
        res = sim.new_result()
        walls, kms = [], []
        for k in range(4):
            res.zero()
            torch.cuda.synchronize()
            t = time.perf_counter()
            sim.run_into(res, N, seed=0, first_id=0, count=cnt)
            torch.cuda.synchronize()
            w = time.perf_counter() - t
            if k:
                walls.append(w)
                kms.append(res.stats()["kernel_ms"])
        res.close()
        wall, km = sorted(walls)[1], sorted(kms)[1]
        rows.append({"packets": cnt * nl, "kernel_ms": km, "wall_ms": wall * 1e3,
                     "packets_per_s_kernel": cnt * nl / (km / 1e3),
                     "packets_per_s_wall": cnt * nl / wall})
        print(f"[curve] {cnt * nl} packets: kernel {km:.3f} ms, wall {wall * 1e3:.3f} ms", file=sys.stderr, flush=True)
    sim.close()
    print(json.dumps({"metric": "packets/s against packets per launch", "workload": workload,
                      "unit": "packets/s", "dtype": "f32", "points": rows}), flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, one wavelength per task, tasks spread over
# processes (replicated scene, per-process tables summed -- the paper's task
# parallel mode).
# ---------------------------------------------------------------------------
_SC = None


def _oracle_task(args):
    ell, n_per_lambda, count, seed = args
    import numpy as np
    import oracle
    sc = _SC
    sub = type(sc)(**{**sc.__dict__})
    for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
        setattr(sub, f, np.ascontiguousarray(getattr(sc, f)[ell:ell + 1]))
    t = time.perf_counter()
    # a one-wavelength copy of the scene: same optics and cost, own streams
    r = oracle.run(sub, n_per_lambda, seed=seed, first_id=0, count=count, model=0)
    return r["stats"]["packets"], time.perf_counter() - t


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, n_per_lambda, seconds_target=15.0):
    global _SC
    import numpy as np
    import oracle
    oracle.lib()
    _SC = scene
    # P = nproc (the CPUs this process may run on), within the host's share of
    # 16 CPUs per GPU
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, nproc))
    # calibrate on one task
    t0 = time.perf_counter()
    _oracle_task((scene.n_lambda // 2, n_per_lambda, 50, 0))
    per_packet = (time.perf_counter() - t0) / 50.0
    count = min(n_per_lambda, max(20, int(seconds_target * cores / max(per_packet, 1e-7) / scene.n_lambda)))
    # one core: the same ids over 8 wavelengths spread across the grid, serially
    c1 = min(n_per_lambda, max(10, int(seconds_target / 4 / max(per_packet, 1e-7) / 8)))
    lams = sorted({int(round(x)) for x in np.linspace(0, scene.n_lambda - 1, 8)})
    t = time.perf_counter()
    p1 = sum(_oracle_task((ell, n_per_lambda, c1, 0))[0] for ell in lams)
    single = p1 / (time.perf_counter() - t)
    tasks = [(ell, n_per_lambda, count, 0) for ell in range(scene.n_lambda)]
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_task, tasks, chunksize=1)
    wall = time.perf_counter() - t
    packets = sum(r[0] for r in res)
    return {"value": packets / wall, "unit": "packets/s", "cores": cores, "kind": "oracle",
            "sample": f"packet ids [0, {count}) of each of the {scene.n_lambda} wavelengths "
                      f"({packets} packets, {wall:.1f} s wall), one wavelength per task on "
                      f"{cores} processes",
            "single_core": {"value": single, "unit": "packets/s",
                            "sample": f"packet ids [0, {c1}) of wavelengths {lams}, one process"},
            "host": {"nproc": nproc, "cpu_count": os.cpu_count(), "cpu_model": _cpu_model()}}


def microbenchmarks():
    """Random-access rates at the working-set sizes of the workloads."""
    from paper_1705_04702_amd import mcrt
    out = {}
    for mb in (2, 64, 256, 1024, 8192):
        b = mb << 20
        row = {}
        for kind in ("gather4", "atomic_f64", "atomic_f64_wg", "atomic_f32", "atomic_f64_run4"):
            row[kind] = mcrt.microbench(kind, b, 1 << 28)
        row["copy_Bps"] = mcrt.microbench("copy", b)
        out[f"{mb}MiB"] = row
        print(f"[microbench] {mb} MiB {row}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="disk",
                    choices=("disk", "sphere", "torus", "batch", "torus-learned", "disk-dust"))
    ap.add_argument("--n-per-lambda", type=int, default=0, help="0 = the workload's own")
    ap.add_argument("--autotune", action="store_true", help="tune the queue before timing (batch: always)")
    ap.add_argument("--no-autotune", action="store_true", help="batch: time the library's default queue")
    ap.add_argument("--step-packets", type=int, default=1_000_000,
                    help="packet ids per wavelength in one step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--threshold", type=int, default=0)
    ap.add_argument("--queue-order", choices=("cost", "caller", "paired"), default="paired",
                    help="batch: model order in the work queue")
    ap.add_argument("--brick", default="", help="log2 brick sizes, e.g. 1,0,4")
    ap.add_argument("--top-level", type=int, default=-1, help="octree top-table level (-1: the library's)")
    ap.add_argument("--curve", action="store_true",
                    help="packets/s against packets per launch, 1e4 up to the full workload (one JSON line)")
    ap.add_argument("--microbench", action="store_true",
                    help="only print the memory-system microbenchmarks (one JSON line)")
    ap.add_argument("--hist-packets", type=int, default=10_000_000, help="torus-learned: history packets")
    ap.add_argument("--learned-packets", type=int, default=100_000_000, help="torus-learned: learned packets")
    ap.add_argument("--ref-packets", type=int, default=1_000_000_000, help="torus-learned: reference packets")
    ap.add_argument("--epochs", type=int, default=2, help="torus-learned: training epochs")
    ap.add_argument("--batch", type=int, default=16384, help="torus-learned: samples per Adam step")
    ap.add_argument("--lr", type=float, default=1e-3, help="torus-learned: Adam learning rate")
    ap.add_argument("--alpha", type=float, default=0.1,
                    help="torus-learned: weight of the HG component in the defensive mixture")
    ap.add_argument("--max-events", type=int, default=16, help="torus-learned: recorded events per packet")
    ap.add_argument("--no-learned", action="store_true",
                    help="default line: skip the learned-vs-plain comparison on the torus")
    ap.add_argument("--tau-peel-max", type=float, default=None,
                    help="peel-off optical-depth cut (default: none, every peel-off counts)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.microbench:
        print(json.dumps(microbenchmarks()))
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(how the path would shard is documented, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1705_04702_amd import mcrt

    torch.cuda.set_device(0)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "torus-learned":
        bench_learned(args)
        return
    if args.workload == "disk-dust":
        bench_dust(args)
        return
    scene, workload = make_scene(args.workload)
    if args.tau_peel_max is not None:
        scene.tau_peel_max = args.tau_peel_max
    N = args.n_per_lambda or WORKLOADS[args.workload][0]
    if args.curve:
        bench_curve(args, scene, workload, N)
        return
    B = min(args.step_packets, N)
    ctx = mcrt.Context(0)
    brick = tuple(int(x) for x in args.brick.split(",")) if args.brick else None
    sim = mcrt.Sim(ctx, scene, mcrt.FP32, chunk=args.chunk or None,
                   waves_per_cu=args.waves_per_cu or None, threshold=args.threshold or None,
                   brick=brick, top_level=args.top_level if args.top_level >= 0 else None)
    if args.autotune:
        # trials of one full step: a shorter launch is dominated by its tail
        # (the longest packet histories), whose best queue differs
        t = mcrt.autotune([sim], [min(N, B)], seed=0,
                          cache_path=os.path.join(ROOT, "_build", "tune_cache.txt"))
        print(f"[bench] autotune {t}", file=sys.stderr, flush=True)
    res = sim.new_result()
    nl = scene.n_lambda
    print(f"[bench] workload={args.workload} n_lambda={nl} step={B} ids/lambda "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)

    def step(k):
        first = (k * B) % N
        cnt = min(B, N - first)
        sim.run_into(res, N, seed=0, first_id=first, count=cnt)
        st = res.stats()
        return cnt * nl, st

    for w in range(args.warmup):
        step(w)
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    res.zero()
    torch.cuda.synchronize()
    prev = res.stats()
    kernel_ms, packets, bytes_alg = [], 0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        n, st = step(k)
        packets += n
        kernel_ms.append(st["kernel_ms"])
        delta = {f: st[f] - prev[f] for f in mcrt.STAT_FIELDS}
        bytes_alg += algorithmic_bytes(delta)
        prev = st
        print(f"[bench] step {k}: {n} packets, kernel {st['kernel_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    e = res.energy()
    balance = abs(e[0] - e[1] - e[2] - e[3]) / e[0]
    st = res.stats()

    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    achieved = bytes_alg / args.steps / avg_kernel_s / 1e9
    traffic, req_per_packet = None, None
    prof = os.path.join(ROOT, "profiles", f"transport_{args.workload}_traffic.json")
    if os.path.exists(prof):
        meta = json.load(open(prof))
        if meta.get("kernel_hash") == kernel_sources_hash():
            traffic = meta["hbm_bytes_per_packet"] * packets / args.steps
            req_per_packet = meta.get("atomic_requests_per_packet")
    # The atomic ceiling measured on this device: random FP64 atomic adds over a
    # working set the size of one wavelength slice of the table, one L2 atomic
    # request each (the L2 forwards every atomic request to the memory side).
    # The kernel's requests per packet come from the TCC_ATOMIC counter of the
    # committed profile while the kernel sources are unchanged.
    slice_bytes = 8 * scene.n_cells
    atomic_ceiling = mcrt.microbench("atomic_f64", max(slice_bytes, 1 << 21), 1 << 28)
    n_atomic = st["prop_cells"] * packets / max(st["packets"], 1)
    atomics_per_s = n_atomic / args.steps / avg_kernel_s
    req_per_s = req_per_packet * packets / args.steps / avg_kernel_s if req_per_packet else None
    out = {
        "metric": METRIC,
        "value": packets / T,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n_per_lambda": N, "packets_per_step": B * nl,
                   "grid": list(scene.n), "n_lambda": nl,
                   "instruments": [list(i.npix) for i in scene.instruments],
                   "tau_peel_max": scene.tau_peel_max},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "atomic_roofline": {"achieved": req_per_s, "peak": atomic_ceiling, "unit": "atomic requests/s",
                            "frac": req_per_s / atomic_ceiling if req_per_s else None,
                            "deposits_per_s": atomics_per_s,
                            "peak_kind": "measured random FP64 atomic adds (one request each), device scope"},
        "energy_balance": balance,
        "counters_per_packet": {f: st[f] / max(st["packets"], 1) for f in
                                ("events", "prop_cells", "locate_cells", "peel_cells", "peel_adds")},
        "kernel_ms_avg": avg_kernel_s * 1e3,
    }
    res.close()
    sim.close()
    # The same kernel against what this device measurably sustains, in this
    # run: a streaming copy, and random 4-byte gathers over a working set the
    # size of the density array (useful bytes only); 8 TB/s is context.
    copy_Bps = mcrt.microbench("copy", 1 << 30)
    gathers = mcrt.microbench("gather4", max(4 * scene.n_cells, 1 << 21), 1 << 28)
    traffic_GBps = traffic / avg_kernel_s / 1e9 if traffic else None
    out["bandwidth_context"] = {
        "copy_GBps": copy_Bps / 1e9, "random_gather_useful_GBps": 4 * gathers / 1e9,
        "random_gathers_per_s": gathers, "gather_working_set_bytes": max(4 * scene.n_cells, 1 << 21),
        "algorithmic_GBps": achieved, "algorithmic_over_copy": achieved / (copy_Bps / 1e9),
        "algorithmic_over_random_gather": achieved / (4 * gathers / 1e9),
        "measured_traffic_GBps": traffic_GBps,
        "measured_traffic_over_copy": traffic_GBps / (copy_Bps / 1e9) if traffic_GBps else None,
        "note": "algorithmic = the roofline's bytes; measured traffic = FETCH_SIZE + WRITE_SIZE of the "
                "committed profile (null when the kernel changed since); the deposits' bound is the "
                "atomic_roofline"}
    if args.workload == "disk" and not args.no_learned:
        print("[bench] learned vs plain on the torus (the metric's second half)", file=sys.stderr, flush=True)
        _, _, cmp, _ = learned_vs_plain(args)
        out["learned_vs_plain"] = cmp
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on host cores)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scene, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
