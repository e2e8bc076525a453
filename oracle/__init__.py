"""Serial FP64 CPU oracle of the Monte Carlo photon-packet life cycle.

TEST INFRASTRUCTURE ONLY: this package is imported by the test suite, the
smoke check and the CPU-baseline leg of the benchmark, never by the GPU
library or its Python binding.  It wraps ``libmcrt_oracle.so`` (plain C,
built from ``mcrt_oracle.c`` with gcc, no floating-point contraction) through
ctypes and accepts any scene object with the attributes of
``paper_1705_04702_amd.scenes.Scene`` (duck typing; nothing is imported from
the GPU package).

The estimator it implements is the stellar emission phase of the
hybrid-parallel SKIRT paper (Section 3.2): launch, propagation with
continuous absorption into the (cell, wavelength) table, forced interaction,
Henyey-Greenstein scattering and peel-off at emission and at each scattering.
Parity pins live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcrt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmcrt_oracle.so")

GCC_FLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(ctypes.Structure):
    _fields_ = [
        ("grid_type", ctypes.c_int32),
        ("box", ctypes.c_double * 6),
        ("n", ctypes.c_int32 * 3),
        ("n_nodes", ctypes.c_int64),
        ("first_child", ctypes.POINTER(ctypes.c_int32)),
        ("n_cells", ctypes.c_int64),
        ("density", ctypes.POINTER(ctypes.c_float)),
        ("n_lambda", ctypes.c_int32),
        ("kappa", ctypes.POINTER(ctypes.c_double)),
        ("albedo", ctypes.POINTER(ctypes.c_double)),
        ("hg_g", ctypes.POINTER(ctypes.c_double)),
        ("source_type", ctypes.c_int32),
        ("src_pos", ctypes.c_double * 3),
        ("disk_hR", ctypes.c_double),
        ("disk_zs", ctypes.c_double),
        ("lum", ctypes.POINTER(ctypes.c_double)),
        ("n_ins", ctypes.c_int32),
        ("ins_geom", ctypes.POINTER(ctypes.c_double)),
        ("ins_npix", ctypes.POINTER(ctypes.c_int32)),
        ("w_min", ctypes.c_double),
        ("event_cap", ctypes.c_int64),
        ("tau_peel_max", ctypes.c_double),
        ("mlp", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
        ("lambda_um", ctypes.POINTER(ctypes.c_double)),
        ("r_out", ctypes.c_double),
        ("lam_feature", ctypes.POINTER(ctypes.c_double)),
        ("rho_mean", ctypes.c_double),
        ("dust_cdf", ctypes.POINTER(ctypes.c_double)),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in
                ("packets", "events", "prop_cells", "peel_cells", "peel_adds",
                 "peel_dropped", "capped")]


class _Out(ctypes.Structure):
    _fields_ = [
        ("table", ctypes.POINTER(ctypes.c_double)),
        ("images", ctypes.POINTER(ctypes.c_double)),
        ("energy", ctypes.POINTER(ctypes.c_double)),
        ("table_m2", ctypes.POINTER(ctypes.c_double)),
        ("image_m2", ctypes.POINTER(ctypes.c_double)),
        ("stats", _Stats),
        ("hist", ctypes.POINTER(ctypes.c_double)),
        ("hist_total", ctypes.POINTER(ctypes.c_double)),
        ("hist_events", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # MCRT_ORACLE_LIB: another build of the same source (the sanitizer
        # build of the CPU tests)
        path = os.environ.get("MCRT_ORACLE_LIB")
        if not path:
            if not os.path.exists(_LIB_PATH):
                build()
            path = _LIB_PATH
        L = ctypes.CDLL(path)
        L.or_run.argtypes = [ctypes.POINTER(_Scene), ctypes.c_uint64, ctypes.c_uint64,
                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Out)]
        L.or_run.restype = ctypes.c_int
        L.or_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.or_philox4x32_10.restype = None
        L.or_uniform64.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint32]
        L.or_uniform64.restype = ctypes.c_double
        L.or_uniform32.argtypes = L.or_uniform64.argtypes
        L.or_uniform32.restype = ctypes.c_float
        L.or_march.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
        L.or_march.restype = ctypes.c_int64
        L.or_mlp_forward.argtypes = [ctypes.POINTER(ctypes.c_double)] * 3
        L.or_mlp_forward.restype = None
        L.or_hg_phase.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_hg_phase.restype = ctypes.c_double
        L.or_hg_sample.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_hg_sample.restype = ctypes.c_double
        L.or_rotate.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double)]
        L.or_rotate.restype = None
        L.or_dust_emission.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.or_dust_emission.restype = ctypes.c_int
        L.or_planck.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_planck.restype = ctypes.c_double
        L.or_bin_widths.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.or_bin_widths.restype = None
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


_SOURCES = {"point_iso": 0, "point_aniso": 1, "expdisk": 2, "dust": 3}


class _SceneHolder:
    """Keeps the numpy arrays behind a ctypes scene alive."""

    def __init__(self, sc):
        self.density = np.ascontiguousarray(sc.density, dtype=np.float32)
        self.kappa = np.ascontiguousarray(sc.kappa, dtype=np.float64)
        self.albedo = np.ascontiguousarray(sc.albedo, dtype=np.float64)
        self.g = np.ascontiguousarray(sc.hg_g, dtype=np.float64)
        self.lum = np.ascontiguousarray(sc.lum, dtype=np.float64)
        geom = [[i.incl_deg, i.azim_deg, i.distance, i.fov[0], i.fov[1]] for i in sc.instruments]
        npix = [[i.npix[0], i.npix[1]] for i in sc.instruments]
        self.geom = np.ascontiguousarray(np.array(geom, dtype=np.float64).reshape(-1, 5))
        self.npix = np.ascontiguousarray(np.array(npix, dtype=np.int32).reshape(-1, 2))
        s = _Scene()
        s.grid_type = 1 if sc.grid_type == "octree" else 0
        for a in range(6):
            s.box[a] = float(sc.box[a])
        if sc.grid_type == "octree":
            self.first_child = np.ascontiguousarray(sc.first_child, dtype=np.int32)
            s.n_nodes = int(self.first_child.shape[0])
            s.first_child = _ptr(self.first_child, ctypes.c_int32)
        else:
            for a in range(3):
                s.n[a] = int(sc.n[a])
        s.n_cells = int(self.density.shape[0])
        s.density = _ptr(self.density, ctypes.c_float)
        s.n_lambda = int(self.kappa.shape[0])
        s.kappa = _ptr(self.kappa, ctypes.c_double)
        s.albedo = _ptr(self.albedo, ctypes.c_double)
        s.hg_g = _ptr(self.g, ctypes.c_double)
        s.source_type = _SOURCES[sc.source]
        for a in range(3):
            s.src_pos[a] = float(sc.src_pos[a])
        s.disk_hR = float(sc.disk_hR)
        s.disk_zs = float(sc.disk_zs)
        s.lum = _ptr(self.lum, ctypes.c_double)
        s.n_ins = len(sc.instruments)
        s.ins_geom = _ptr(self.geom, ctypes.c_double)
        s.ins_npix = _ptr(self.npix, ctypes.c_int32)
        s.w_min = float(sc.w_min)
        s.event_cap = int(sc.event_cap)
        s.tau_peel_max = float(sc.tau_peel_max)
        self.lambdas = np.ascontiguousarray(sc.lambdas, dtype=np.float64)
        s.lambda_um = _ptr(self.lambdas, ctypes.c_double)
        if sc.source == "dust":
            self.dust_cdf = np.ascontiguousarray(sc.dust_cdf, dtype=np.float64)
            s.dust_cdf = _ptr(self.dust_cdf, ctypes.c_double)
        self.s = s


def run(scene, n_per_lambda: int, seed: int = 0, first_id: int = 0, count=None,
        model: int = 0, moments: bool = False, mlp=None, alpha: float = 0.2, histories: int = 0):
    """Runs packet ids [first_id, first_id + count) of every wavelength.

    Returns a dict with ``table`` [n_cells, n_lambda] (element (i, j) = cell i,
    wavelength j), ``images`` (list of [n_lambda, ny, nx] flux arrays),
    ``energy`` (emitted, absorbed, escaped, truncated), ``stats`` and, with
    moments=True, per-packet second moments ``table_m2`` / ``image_m2``.
    """
    if count is None:
        count = n_per_lambda - first_id
    h = _SceneHolder(scene)
    if mlp is not None:
        from oracle import learned
        h.mlp = np.ascontiguousarray(learned.round_weights(np.asarray(mlp, dtype=np.float64)))
        h.s.mlp = _ptr(h.mlp, ctypes.c_double)
        h.s.alpha = float(alpha)
    nl = h.s.n_lambda
    table = np.zeros(h.s.n_cells * nl, dtype=np.float64)
    shapes = [(nl, i.npix[1], i.npix[0]) for i in scene.instruments]
    nimg = sum(int(np.prod(s)) for s in shapes)
    images = np.zeros(max(nimg, 1), dtype=np.float64)
    energy = np.zeros(4, dtype=np.float64)
    out = _Out()
    out.table = _ptr(table, ctypes.c_double)
    out.images = _ptr(images, ctypes.c_double)
    out.energy = _ptr(energy, ctypes.c_double)
    if moments:
        tm2 = np.zeros_like(table)
        im2 = np.zeros_like(images)
        out.table_m2 = _ptr(tm2, ctypes.c_double)
        out.image_m2 = _ptr(im2, ctypes.c_double)
    if histories:
        npk = int(count) * nl
        hist = np.zeros(npk * histories * 14)
        htot = np.zeros(npk)
        out.hist = _ptr(hist, ctypes.c_double)
        out.hist_total = _ptr(htot, ctypes.c_double)
        out.hist_events = int(histories)
    rc = lib().or_run(ctypes.byref(h.s), int(n_per_lambda), int(first_id), int(count),
                      int(seed), int(model), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle or_run failed with code {rc}")
    res = {
        "table": table.reshape(h.s.n_cells, nl),
        "images": _split(images, shapes),
        "energy": energy,
        "stats": {name: int(getattr(out.stats, name)) for name, _ in _Stats._fields_},
    }
    if moments:
        res["table_m2"] = tm2.reshape(h.s.n_cells, nl)
        res["image_m2"] = _split(im2, shapes)
    if histories:
        res["hist"] = hist.reshape(-1, histories, 14)
        res["hist_total"] = htot
    return res


# ---------------------------------------------------------------------------
# Dust emission phase and self-absorption cycles (Section 3.2), Cartesian grids
# ---------------------------------------------------------------------------
def planck(lambda_um, T):
    return lib().or_planck(float(lambda_um), float(T))


def bin_widths(lambda_um):
    lam = np.ascontiguousarray(lambda_um, dtype=np.float64)
    w = np.zeros_like(lam)
    lib().or_bin_widths(_ptr(lam, ctypes.c_double), lam.size, _ptr(w, ctypes.c_double))
    return w


def dust_emission(scene, table, T0: float = 20.0, beta: float = 2.0):
    """Cell temperatures [n_cells] and emission [n_cells, n_lambda] from an
    absorbed-luminosity table [n_cells, n_lambda] (or_dust_emission)."""
    h = _SceneHolder(scene)
    tab = np.ascontiguousarray(table, dtype=np.float64)
    T = np.zeros(h.s.n_cells)
    emis = np.zeros((h.s.n_cells, h.s.n_lambda))
    rc = lib().or_dust_emission(ctypes.byref(h.s), _ptr(tab, ctypes.c_double), float(T0), float(beta),
                                _ptr(T, ctypes.c_double), _ptr(emis, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle or_dust_emission failed with code {rc}")
    return T, emis


def dust_scene(scene, emis):
    """The scene with its source replaced by the dust emission emis [n_cells,
    n_lambda]: running sums over the cells per wavelength, luminosity per
    wavelength = the last running sum."""
    cdf = np.ascontiguousarray(np.cumsum(np.asarray(emis, dtype=np.float64).T, axis=1))
    sc = type(scene)(**{**scene.__dict__})
    sc.source = "dust"
    sc.lum = cdf[:, -1].copy()
    sc.dust_cdf = cdf
    return sc


def self_absorption(scene, stellar_table, n_per_lambda: int, seed: int, cycles: int, T0: float = 20.0,
                    beta: float = 2.0):
    """Dust self-absorption cycles: cycle k (k = 1..cycles) emits from the
    stellar plus the previous cycle's dust absorption and runs its packets
    with seed + k - 1.  Returns per cycle (dust luminosity per wavelength,
    the cycle's run result)."""
    dust_abs = np.zeros_like(np.asarray(stellar_table))
    out = []
    for k in range(1, cycles + 1):
        _, emis = dust_emission(scene, np.asarray(stellar_table) + dust_abs, T0, beta)
        sc = dust_scene(scene, emis)
        r = run(sc, n_per_lambda, seed=seed + k - 1)
        out.append((sc.lum, r))
        dust_abs = r["table"]
    return out


def mlp_forward(theta, f):
    """The C oracle's network evaluation (bf16-rounded inputs/activations)."""
    t = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(f, dtype=np.float64)
    o = np.zeros(40)
    lib().or_mlp_forward(_ptr(t, ctypes.c_double), _ptr(x, ctypes.c_double), _ptr(o, ctypes.c_double))
    return o


def _split(flat, shapes):
    out, off = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(flat[off:off + n].reshape(s))
        off += n
    return out


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform64(seed, packet, lam, model, slot):
    return lib().or_uniform64(seed, packet, lam, model, slot)


def uniform32(seed, packet, lam, model, slot):
    return lib().or_uniform32(seed, packet, lam, model, slot)


def march(scene, r, k, max_seg: int = 1 << 16):
    """Segments (cell, length) of the ray r + t k, t >= 0, through the grid."""
    h = _SceneHolder(scene)
    rr = (ctypes.c_double * 3)(*r)
    kk = (ctypes.c_double * 3)(*k)
    cells = np.zeros(max_seg, dtype=np.int64)
    lens = np.zeros(max_seg, dtype=np.float64)
    n = lib().or_march(ctypes.byref(h.s), rr, kk, _ptr(cells, ctypes.c_int64),
                       _ptr(lens, ctypes.c_double), max_seg)
    if n < 0:
        raise RuntimeError("oracle march failed")
    return cells[:n].copy(), lens[:n].copy()


def hg_phase(g, mu):
    return lib().or_hg_phase(g, mu)


def hg_sample(g, u):
    return lib().or_hg_sample(g, u)


def rotate(k, mu, phi):
    kk = (ctypes.c_double * 3)(*k)
    o = (ctypes.c_double * 3)()
    lib().or_rotate(kk, mu, phi, o)
    return [o[0], o[1], o[2]]
