"""The oracle over disjoint packet-id ranges in threads (test harness).

ctypes releases the interpreter lock while the oracle runs and the oracle
keeps no mutable global state, so ranges run in parallel; their tables,
images, energy sums, counters and per-packet second moments add up exactly
to one run over the union of the ranges (every packet has its own stream).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def threads_default() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run(scene, n_per_lambda: int, seed: int, first_id: int = 0, count=None, threads=None, **kw):
    """oracle.run over ids [first_id, first_id + count), split in threads."""
    if count is None:
        count = n_per_lambda - first_id
    T = max(1, min(threads or threads_default(), count))
    edges = [first_id + (count * t) // T for t in range(T + 1)]
    jobs = [(edges[t], edges[t + 1] - edges[t]) for t in range(T) if edges[t + 1] > edges[t]]

    def one(job):
        return oracle.run(scene, n_per_lambda, seed=seed, first_id=job[0], count=job[1], **kw)

    with ThreadPoolExecutor(len(jobs)) as ex:
        parts = list(ex.map(one, jobs))
    out = parts[0]
    for p in parts[1:]:
        out["table"] += p["table"]
        for a, b in zip(out["images"], p["images"]):
            a += b
        out["energy"] = out["energy"] + p["energy"]
        for k in out["stats"]:
            out["stats"][k] += p["stats"][k]
        if "table_m2" in out:
            out["table_m2"] += p["table_m2"]
            for a, b in zip(out["image_m2"], p["image_m2"]):
                a += b
        del p
    return out


def subset_lambdas(scene, keep):
    """A copy of the scene on the wavelengths `keep` (its own streams: the
    wavelength index of the copy is the position in `keep`)."""
    sub = type(scene)(**{**scene.__dict__})
    for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
        setattr(sub, f, np.ascontiguousarray(np.asarray(getattr(scene, f))[list(keep)]))
    sub.name = f"{scene.name}_{len(keep)}l"
    return sub
