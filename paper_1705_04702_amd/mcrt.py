"""Python binding of the C-ABI in include/mcrt.h (ctypes; argument marshalling
only -- every step of the photon life cycle runs in the HIP kernels of
libmcrt.so).  PyTorch supplies the stream (and, optionally, device output
buffers); the library allocates its own device memory.

The binding fails loudly when libmcrt.so is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MCRT_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MCRT_LIBRARY") or os.path.join(HERE, "libmcrt.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ELIMIT, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FP32, FP64_VALIDATE = 0, 1

EXPORTS = [
    "mcrt_options_default", "mcrt_context_create", "mcrt_context_destroy",
    "mcrt_grid_create_cartesian", "mcrt_grid_create_octree", "mcrt_grid_destroy",
    "mcrt_medium_create", "mcrt_medium_destroy", "mcrt_source_create_point",
    "mcrt_source_create_expdisk", "mcrt_source_destroy", "mcrt_instrument_create",
    "mcrt_instrument_destroy", "mcrt_sim_create", "mcrt_sim_destroy", "mcrt_result_create",
    "mcrt_result_zero", "mcrt_run_into", "mcrt_run_into_noalloc", "mcrt_run", "mcrt_run_range",
    "mcrt_result_absorption",
    "mcrt_result_image", "mcrt_result_energy", "mcrt_result_stats", "mcrt_result_destroy",
    "mcrt_sim_info", "mcrt_last_error", "mcrt_microbench", "mcrt_microbench_error",
    "mcrt_batch_run_into", "mcrt_sim_set_tuning", "mcrt_autotune",
    "mcrt_proposal_create", "mcrt_proposal_destroy", "mcrt_proposal_set_params",
    "mcrt_proposal_get_params", "mcrt_proposal_get_weights", "mcrt_proposal_forward",
    "mcrt_proposal_grad", "mcrt_sim_set_proposal", "mcrt_proposal_collect", "mcrt_histories_info",
    "mcrt_histories_records", "mcrt_histories_samples", "mcrt_histories_destroy",
    "mcrt_train_opts_default", "mcrt_proposal_train", "mcrt_proposal_eval",
    "mcrt_result_sed", "mcrt_result_write", "mcrt_fits_cube_create", "mcrt_fits_cube_write_slices",
    "mcrt_sed_write_text", "mcrt_dust_params_default", "mcrt_dust_create", "mcrt_dust_luminosity",
    "mcrt_dust_temperature", "mcrt_dust_destroy", "mcrt_run_dust_into", "mcrt_dust_self_absorption",
]
MLP_PARAMS = 7400


class MCRTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mcrt error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("w_min", ctypes.c_double),
        ("event_cap", ctypes.c_int64),
        ("tau_peel_max", ctypes.c_double),
        ("chunk", ctypes.c_int32),
        ("waves_per_cu", ctypes.c_int32),
        ("threshold", ctypes.c_int32),
        ("top_level", ctypes.c_int32),
        ("brick", ctypes.c_int32 * 3),
        ("queue_order", ctypes.c_int32),
        ("chunk_shift", ctypes.c_int32),
        ("deposit_slots", ctypes.c_int32),
    ]


QUEUE_COST, QUEUE_CALLER, QUEUE_PAIRED = 0, 1, 2


STAT_FIELDS = ["packets", "events", "prop_cells", "locate_cells", "peel_cells", "peel_adds",
               "peel_dropped", "capped", "guard", "nonfinite"]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("from_cache", ctypes.c_int32), ("default_ms", ctypes.c_double),
                ("chunk_shift", ctypes.c_int32), ("deposit_slots", ctypes.c_int32)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("init_seed", ctypes.c_uint64), ("init_scale", ctypes.c_float)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in STAT_FIELDS] + [("kernel_ms", ctypes.c_double)]


_lib = None
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
DP = ctypes.POINTER(ctypes.c_double)
FP = ctypes.POINTER(ctypes.c_float)
IP = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Loads libmcrt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1705_04702_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "mcrt_options_default": (None, [ctypes.POINTER(Options)]),
        "mcrt_context_create": (ctypes.c_int, [ctypes.c_int, P, PP]),
        "mcrt_context_destroy": (None, [P]),
        "mcrt_grid_create_cartesian": (ctypes.c_int, [P, DP, IP, PP]),
        "mcrt_grid_create_octree": (ctypes.c_int, [P, DP, ctypes.c_int64, IP, PP]),
        "mcrt_grid_destroy": (None, [P]),
        "mcrt_medium_create": (ctypes.c_int, [P, FP, ctypes.c_int32, DP, DP, DP, DP, PP]),
        "mcrt_medium_destroy": (None, [P]),
        "mcrt_source_create_point": (ctypes.c_int, [P, DP, ctypes.c_int32, ctypes.c_int32, DP, PP]),
        "mcrt_source_create_expdisk": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_int32, DP, PP]),
        "mcrt_source_destroy": (None, [P]),
        "mcrt_instrument_create": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, DP, IP, PP]),
        "mcrt_instrument_destroy": (None, [P]),
        "mcrt_sim_create": (ctypes.c_int, [P, P, P, PP, ctypes.c_int32,
                                           ctypes.POINTER(Options), PP]),
        "mcrt_sim_destroy": (None, [P]),
        "mcrt_result_create": (ctypes.c_int, [P, PP]),
        "mcrt_result_zero": (ctypes.c_int, [P]),
        "mcrt_run_into": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, P]),
        "mcrt_run_into_noalloc": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, P]),
        "mcrt_run": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_uint64, PP]),
        "mcrt_run_range": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, PP]),
        "mcrt_result_absorption": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_result_image": (ctypes.c_int, [P, ctypes.c_int32, P, ctypes.c_size_t]),
        "mcrt_result_energy": (ctypes.c_int, [P, DP, DP, DP, DP]),
        "mcrt_result_stats": (ctypes.c_int, [P, ctypes.POINTER(Stats)]),
        "mcrt_result_destroy": (None, [P]),
        "mcrt_sim_info": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "mcrt_last_error": (ctypes.c_char_p, []),
        "mcrt_microbench": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_double)]),
        "mcrt_microbench_error": (ctypes.c_char_p, []),
        "mcrt_batch_run_into": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                               ctypes.c_uint64, PP]),
        "mcrt_sim_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "mcrt_autotune": (ctypes.c_int, [PP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64,
                                         ctypes.c_char_p, ctypes.POINTER(Tuning)]),
        "mcrt_proposal_create": (ctypes.c_int, [P, ctypes.POINTER(MlpDesc), PP]),
        "mcrt_proposal_destroy": (None, [P]),
        "mcrt_proposal_set_params": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_proposal_get_params": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_proposal_get_weights": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_proposal_forward": (ctypes.c_int, [P, P, ctypes.c_int64, P]),
        "mcrt_proposal_grad": (ctypes.c_int, [P, P, P, P, ctypes.c_int64, DP, P]),
        "mcrt_sim_set_proposal": (ctypes.c_int, [P, P, ctypes.c_double]),
        "mcrt_proposal_collect": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                 ctypes.c_uint64, ctypes.c_int32, P, PP]),
        "mcrt_histories_info": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int64), DP]),
        "mcrt_histories_records": (ctypes.c_int, [P, P, ctypes.c_size_t, P, ctypes.c_size_t]),
        "mcrt_histories_samples": (ctypes.c_int, [P, P, P, P, ctypes.c_size_t]),
        "mcrt_histories_destroy": (None, [P]),
        "mcrt_train_opts_default": (None, [ctypes.POINTER(TrainOpts)]),
        "mcrt_proposal_train": (ctypes.c_int, [P, P, ctypes.POINTER(TrainOpts), DP]),
        "mcrt_proposal_eval": (ctypes.c_int, [P, P, DP]),
        "mcrt_result_sed": (ctypes.c_int, [P, ctypes.c_int32, P, ctypes.c_size_t]),
        "mcrt_result_write": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_char_p]),
        "mcrt_fits_cube_create": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                 P]),
        "mcrt_fits_cube_write_slices": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int64, ctypes.c_int64,
                                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]),
        "mcrt_sed_write_text": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int32, P, P]),
        "mcrt_dust_params_default": (None, [ctypes.POINTER(DustParams)]),
        "mcrt_dust_create": (ctypes.c_int, [P, PP, ctypes.c_int32, ctypes.POINTER(DustParams), PP]),
        "mcrt_dust_luminosity": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_dust_temperature": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "mcrt_dust_destroy": (None, [P]),
        "mcrt_run_dust_into": (ctypes.c_int, [P, P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_uint64, P]),
        "mcrt_dust_self_absorption": (ctypes.c_int, [P, P, ctypes.POINTER(DustParams), ctypes.c_uint64,
                                                     ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, PP, PP,
                                                     ctypes.POINTER(ctypes.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise MCRTError(rc, lib().mcrt_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(DP)


MICROBENCH_KINDS = {"gather4": 0, "atomic_f64": 1, "atomic_f64_wg": 2, "atomic_f32": 3, "copy": 4,
                    "atomic_f64_run4": 5, "atomic_f64_line8": 6, "atomic_f64_wave64": 7}


def microbench(kind: str, nbytes: int, n_ops: int = 1 << 28, device: int = 0) -> float:
    """Operations/s (bytes/s for "copy") of a memory-system microbenchmark."""
    r = ctypes.c_double()
    rc = lib().mcrt_microbench(int(device), MICROBENCH_KINDS[kind], int(nbytes), int(n_ops), ctypes.byref(r))
    if rc != OK:
        raise MCRTError(rc, lib().mcrt_microbench_error().decode())
    return r.value


class DustParams(ctypes.Structure):
    _fields_ = [("T0", ctypes.c_double), ("beta", ctypes.c_double)]


class Dust:
    """Dust emission of a Cartesian sim's cells (device-resident running sums
    of the emission per wavelength, temperatures)."""

    def __init__(self, sim: "Sim", h):
        self.sim = sim
        self.h = h

    def luminosity(self) -> np.ndarray:
        out = np.empty(self.sim.n_lambda, dtype=np.float64)
        _check(lib().mcrt_dust_luminosity(self.h, ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def temperature(self) -> np.ndarray:
        out = np.empty(self.sim.n_cells, dtype=np.float64)
        _check(lib().mcrt_dust_temperature(self.h, ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def close(self):
        if self.h:
            lib().mcrt_dust_destroy(self.h)
            self.h = None
        self.sim._dusts.discard(self)


def dust_params(T0: Optional[float] = None, beta: Optional[float] = None) -> DustParams:
    p = DustParams()
    lib().mcrt_dust_params_default(ctypes.byref(p))
    if T0 is not None:
        p.T0 = float(T0)
    if beta is not None:
        p.beta = float(beta)
    return p


def fits_cube_create(path, nx: int, ny: int, lambda_um) -> None:
    """Creates a FITS data cube [n_lambda][ny][nx] of zeros with a WAVELENGTHS
    extension (host only)."""
    lam = np.ascontiguousarray(lambda_um, dtype=np.float64)
    _check(lib().mcrt_fits_cube_create(os.fsencode(path), int(nx), int(ny), lam.size,
                                       ctypes.c_void_p(lam.ctypes.data)))


def fits_cube_write_slices(path, n_lambda: int, first: int, slices) -> None:
    """Writes slices[count][ny][nx] at wavelength slices [first, first + count)."""
    a = np.ascontiguousarray(slices, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("slices must be [count][ny][nx]")
    _check(lib().mcrt_fits_cube_write_slices(os.fsencode(path), a.shape[2], a.shape[1], int(n_lambda), int(first),
                                             a.shape[0], ctypes.c_void_p(a.ctypes.data)))


def sed_write_text(path, lambda_um, sed) -> None:
    lam = np.ascontiguousarray(lambda_um, dtype=np.float64)
    f = np.ascontiguousarray(sed, dtype=np.float64)
    if f.shape != lam.shape:
        raise ValueError("lambda_um and sed differ in length")
    _check(lib().mcrt_sed_write_text(os.fsencode(path), lam.size, ctypes.c_void_p(lam.ctypes.data),
                                     ctypes.c_void_p(f.ctypes.data)))


def default_options(**kw) -> Options:
    o = Options()
    lib().mcrt_options_default(ctypes.byref(o))
    names = {f[0] for f in Options._fields_}
    for k, val in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}")
        if val is None:
            continue
        if k == "brick":
            for a in range(3):
                o.brick[a] = int(val[a])
        else:
            setattr(o, k, val)
    return o


def _torch_stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A device and a stream (torch's current stream of that device by default)."""

    def __init__(self, device: int = 0, stream=None):
        if stream is None:
            stream = _torch_stream(device)
        h = ctypes.c_void_p()
        _check(lib().mcrt_context_create(int(device), stream, ctypes.byref(h)))
        self.h = h
        self.device = device
        self._deps = weakref.WeakSet()  # proposals and histories (closed first)

    def close(self):
        for d in list(getattr(self, "_deps", ())):
            d.close()
        if self.h:
            lib().mcrt_context_destroy(self.h)
            self.h = None


class Result:
    def __init__(self, sim: "Sim", h):
        self.sim = sim
        self.h = h

    def zero(self):
        _check(lib().mcrt_result_zero(self.h))

    def table(self, out=None):
        """Absorbed luminosity [n_cells, n_lambda] (cell i, wavelength j).
        out may be a float64 numpy array or a CUDA float64 torch tensor."""
        n = self.sim.n_cells * self.sim.n_lambda
        if out is None:
            out = np.empty((self.sim.n_cells, self.sim.n_lambda), dtype=np.float64)
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else out.ctypes.data
        _check(lib().mcrt_result_absorption(self.h, ctypes.c_void_p(ptr), n))
        return out

    def image(self, j: int):
        nl, ny, nx = self.sim.image_shapes[j]
        out = np.empty((nl, ny, nx), dtype=np.float64)
        _check(lib().mcrt_result_image(self.h, int(j), ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def images(self) -> List[np.ndarray]:
        return [self.image(j) for j in range(len(self.sim.image_shapes))]

    def sed(self, j: int) -> np.ndarray:
        """Total flux per wavelength of instrument j (sum of its pixels)."""
        out = np.empty(self.sim.n_lambda, dtype=np.float64)
        _check(lib().mcrt_result_sed(self.h, int(j), ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def write(self, j: int, fits_path=None, sed_path=None):
        """Writes instrument j's data cube (FITS) and/or SED (text)."""
        enc = lambda p: None if p is None else os.fsencode(p)
        _check(lib().mcrt_result_write(self.h, int(j), enc(fits_path), enc(sed_path)))

    def energy(self) -> np.ndarray:
        e = [ctypes.c_double() for _ in range(4)]
        _check(lib().mcrt_result_energy(self.h, *[ctypes.byref(x) for x in e]))
        return np.array([x.value for x in e])

    def stats(self) -> dict:
        s = Stats()
        _check(lib().mcrt_result_stats(self.h, ctypes.byref(s)))
        d = {n: int(getattr(s, n)) for n in STAT_FIELDS}
        d["kernel_ms"] = float(s.kernel_ms)
        return d

    def close(self):
        if self.h:
            lib().mcrt_result_destroy(self.h)
            self.h = None
        self.sim._results.discard(self)

    def __del__(self):
        try:
            if self.h and self.sim.h:
                self.close()
        except Exception:
            pass


class Sim:
    """A scene uploaded to the device (grid, medium, source, instruments)."""

    _SRC = {"point_iso": 0, "point_aniso": 1}

    def __init__(self, ctx: Context, scene, precision: int = FP32, **tune):
        L = lib()
        self.ctx = ctx
        self.h = None
        self._results = weakref.WeakSet()
        self._dusts = weakref.WeakSet()
        box = (ctypes.c_double * 6)(*[float(x) for x in scene.box])
        g = ctypes.c_void_p()
        if scene.grid_type == "octree":
            fc = np.ascontiguousarray(scene.first_child, dtype=np.int32)
            _check(L.mcrt_grid_create_octree(ctx.h, box, int(fc.shape[0]),
                                             fc.ctypes.data_as(IP), ctypes.byref(g)))
        else:
            n = (ctypes.c_int32 * 3)(*[int(x) for x in scene.n])
            _check(L.mcrt_grid_create_cartesian(ctx.h, box, n, ctypes.byref(g)))
        self.grid = g
        dens = np.ascontiguousarray(scene.density, dtype=np.float32)
        kap = np.ascontiguousarray(scene.kappa, dtype=np.float64)
        alb = np.ascontiguousarray(scene.albedo, dtype=np.float64)
        gg = np.ascontiguousarray(scene.hg_g, dtype=np.float64)
        lam = np.ascontiguousarray(scene.lambdas, dtype=np.float64)
        med = ctypes.c_void_p()
        _check(L.mcrt_medium_create(g, dens.ctypes.data_as(FP), int(kap.shape[0]), _dptr(lam),
                                    _dptr(kap), _dptr(alb), _dptr(gg), ctypes.byref(med)))
        self.medium = med
        lum = np.ascontiguousarray(scene.lum, dtype=np.float64)
        src = ctypes.c_void_p()
        if scene.source == "expdisk":
            _check(L.mcrt_source_create_expdisk(ctx.h, float(scene.disk_hR), float(scene.disk_zs),
                                                int(lum.shape[0]), _dptr(lum), ctypes.byref(src)))
        else:
            pos = (ctypes.c_double * 3)(*[float(x) for x in scene.src_pos])
            _check(L.mcrt_source_create_point(ctx.h, pos, self._SRC[scene.source], int(lum.shape[0]),
                                              _dptr(lum), ctypes.byref(src)))
        self.source = src
        self.instruments = []
        for ins in scene.instruments:
            h = ctypes.c_void_p()
            fov = (ctypes.c_double * 2)(float(ins.fov[0]), float(ins.fov[1]))
            npix = (ctypes.c_int32 * 2)(int(ins.npix[0]), int(ins.npix[1]))
            _check(L.mcrt_instrument_create(ctx.h, float(ins.incl_deg), float(ins.azim_deg),
                                            float(ins.distance), fov, npix, ctypes.byref(h)))
            self.instruments.append(h)
        arr = (ctypes.c_void_p * max(1, len(self.instruments)))(*[h.value for h in self.instruments])
        opt = default_options(precision=precision, w_min=scene.w_min, event_cap=scene.event_cap,
                              tau_peel_max=scene.tau_peel_max, **tune)
        s = ctypes.c_void_p()
        _check(L.mcrt_sim_create(ctx.h, med, src, arr, len(self.instruments), ctypes.byref(opt),
                                 ctypes.byref(s)))
        self.h = s
        self.n_cells = int(dens.shape[0])
        self.n_lambda = int(kap.shape[0])
        self.image_shapes = [(self.n_lambda, ins.npix[1], ins.npix[0]) for ins in scene.instruments]
        self.precision = precision

    def set_proposal(self, prop: Optional["Proposal"], alpha: float = 0.2):
        """Attach (or with None detach) a learned direction proposal."""
        _check(lib().mcrt_sim_set_proposal(self.h, prop.h if prop is not None else None, float(alpha)))
        self.proposal = prop

    def collect(self, result: Result, n_per_lambda: int, seed: int = 0, max_events: int = 16,
                first_id: int = 0, count: Optional[int] = None) -> "Histories":
        """Plain run into result that also records per-event histories."""
        if count is None:
            count = n_per_lambda - first_id
        h = ctypes.c_void_p()
        _check(lib().mcrt_proposal_collect(self.h, int(n_per_lambda), int(first_id), int(count), int(seed),
                                           int(max_events), result.h, ctypes.byref(h)), allow=(ELIMIT, ENONFINITE))
        return Histories(h, self.ctx)

    def set_tuning(self, chunk: int, waves_per_cu: int, threshold: int, chunk_shift: int = 0,
                   deposit_slots: int = 0):
        t = Tuning(chunk, waves_per_cu, threshold, 0.0, 0, 0.0, chunk_shift, deposit_slots)
        _check(lib().mcrt_sim_set_tuning(self.h, ctypes.byref(t)))

    def new_result(self) -> Result:
        r = ctypes.c_void_p()
        _check(lib().mcrt_result_create(self.h, ctypes.byref(r)))
        res = Result(self, r)
        self._results.add(res)
        return res

    def run_into(self, result: Result, n_per_lambda: int, seed: int = 0, first_id: int = 0,
                 count: Optional[int] = None) -> int:
        if count is None:
            count = n_per_lambda - first_id
        return _check(lib().mcrt_run_into(self.h, int(n_per_lambda), int(first_id), int(count),
                                          int(seed), result.h), allow=(ELIMIT, ENONFINITE))

    def run_into_noalloc(self, result: Result, n_per_lambda: int, seed: int = 0, first_id: int = 0,
                         count: Optional[int] = None) -> int:
        """run_into through the allocation-free entry point (the library's
        per-GPU scratch array; no allocation, no host copy, not timed)."""
        if count is None:
            count = n_per_lambda - first_id
        return _check(lib().mcrt_run_into_noalloc(self.h, int(n_per_lambda), int(first_id), int(count),
                                                  int(seed), result.h), allow=(ELIMIT, ENONFINITE))

    def run(self, n_per_lambda: int, seed: int = 0, first_id: int = 0,
            count: Optional[int] = None) -> Result:
        res = self.new_result()
        self.run_into(res, n_per_lambda, seed, first_id, count)
        return res

    def dust(self, absorbed: Sequence[Result], T0: Optional[float] = None, beta: Optional[float] = None) -> Dust:
        """Dust emission from the summed absorption of up to 4 results."""
        arr = (ctypes.c_void_p * len(absorbed))(*[r.h for r in absorbed])
        p = dust_params(T0, beta)
        h = ctypes.c_void_p()
        _check(lib().mcrt_dust_create(self.h, arr, len(absorbed), ctypes.byref(p), ctypes.byref(h)))
        d = Dust(self, h)
        self._dusts.add(d)
        return d

    def run_dust_into(self, dust: Dust, result: Result, n_per_lambda: int, seed: int = 0, first_id: int = 0,
                      count: Optional[int] = None) -> int:
        if count is None:
            count = n_per_lambda - first_id
        return _check(lib().mcrt_run_dust_into(self.h, dust.h, int(n_per_lambda), int(first_id), int(count),
                                               int(seed), result.h), allow=(ELIMIT, ENONFINITE))

    def run_dust(self, dust: Dust, n_per_lambda: int, seed: int = 0) -> Result:
        res = self.new_result()
        self.run_dust_into(dust, res, n_per_lambda, seed)
        return res

    def self_absorption(self, stellar: Result, n_per_lambda: int, seed: int = 0, max_cycles: int = 10,
                        tol: float = 1e-3, T0: Optional[float] = None, beta: Optional[float] = None):
        """Self-absorption cycles (mcrt_dust_self_absorption): returns the last
        cycle's (Dust, Result, cycles run)."""
        p = dust_params(T0, beta)
        d, r, k = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int32()
        _check(lib().mcrt_dust_self_absorption(self.h, stellar.h, ctypes.byref(p), int(n_per_lambda), int(seed),
                                               int(max_cycles), float(tol), ctypes.byref(d), ctypes.byref(r),
                                               ctypes.byref(k)), allow=(ELIMIT, ENONFINITE))
        dust = Dust(self, d)
        self._dusts.add(dust)
        res = Result(self, r)
        self._results.add(res)
        return dust, res, int(k.value)

    def close(self):
        """Destroys the sim's results and dust emissions first (a handle must
        outlive the handles created from it), then the sim and its scene
        objects."""
        L = lib()
        for d in list(getattr(self, "_dusts", ())):
            d.close()
        for r in list(getattr(self, "_results", ())):
            r.close()
        if getattr(self, "h", None):
            L.mcrt_sim_destroy(self.h)
            self.h = None
        for h in getattr(self, "instruments", []):
            L.mcrt_instrument_destroy(h)
        self.instruments = []
        for name, fn in (("source", L.mcrt_source_destroy), ("medium", L.mcrt_medium_destroy),
                         ("grid", L.mcrt_grid_destroy)):
            h = getattr(self, name, None)
            if h:
                fn(h)
                setattr(self, name, None)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Proposal:
    """Learned direction proposal: network parameters on the device (FP32
    master, bf16 fragments for the matrix cores, FP64 copy), Adam state."""

    def __init__(self, ctx: Context, seed: int = 0, init_scale: float = 1.0, params=None):
        self.ctx = ctx
        self.h = None
        d = MlpDesc(9, 64, 40, int(seed), float(init_scale))
        h = ctypes.c_void_p()
        _check(lib().mcrt_proposal_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        ctx._deps.add(self)
        if params is not None:
            self.set_params(params)

    def set_params(self, theta):
        t = _f32(theta)
        if t.size != MLP_PARAMS:
            raise ValueError("expected 7400 parameters")
        _check(lib().mcrt_proposal_set_params(self.h, t.ctypes.data, t.size))

    def params(self) -> np.ndarray:
        t = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().mcrt_proposal_get_params(self.h, t.ctypes.data, t.size))
        return t

    def weights_bf16(self) -> np.ndarray:
        w = np.zeros(MLP_PARAMS, dtype=np.uint16)
        _check(lib().mcrt_proposal_get_weights(self.h, w.ctypes.data, w.size))
        return w

    def forward(self, X) -> np.ndarray:
        X = _f32(X).reshape(-1, 9)
        out = np.zeros((X.shape[0], 40), dtype=np.float32)
        _check(lib().mcrt_proposal_forward(self.h, X.ctypes.data, X.shape[0], out.ctypes.data))
        return out

    def grad(self, X, KP, C):
        X, KP, C = _f32(X).reshape(-1, 9), _f32(KP).reshape(-1, 3), _f32(C).reshape(-1)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().mcrt_proposal_grad(self.h, X.ctypes.data, KP.ctypes.data, C.ctypes.data, X.shape[0],
                                        ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, hist: "Histories", epochs: int = 2, batch: int = 16384, lr: float = 1e-3,
              seed: int = 1, beta1: Optional[float] = None, beta2: Optional[float] = None,
              eps: Optional[float] = None) -> float:
        o = TrainOpts()
        lib().mcrt_train_opts_default(ctypes.byref(o))
        o.epochs, o.batch, o.lr, o.seed = int(epochs), int(batch), float(lr), int(seed)
        if beta1 is not None:
            o.beta1 = float(beta1)
        if beta2 is not None:
            o.beta2 = float(beta2)
        if eps is not None:
            o.eps = float(eps)
        loss = ctypes.c_double()
        _check(lib().mcrt_proposal_train(self.h, hist.h, ctypes.byref(o), ctypes.byref(loss)))
        return loss.value

    def eval(self, hist: "Histories") -> float:
        loss = ctypes.c_double()
        _check(lib().mcrt_proposal_eval(self.h, hist.h, ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            lib().mcrt_proposal_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Histories:
    """Per-event records of a plain run and the training samples built from them."""

    def __init__(self, h, ctx: Context):
        self.h = h
        ctx._deps.add(self)
        n, e, ns, cs = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().mcrt_histories_info(h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(ns), ctypes.byref(cs)))
        self.n_packets, self.max_events, self.n_samples, self.weight_sum = n.value, e.value, ns.value, cs.value

    def records(self):
        rec = np.zeros((self.n_packets, self.max_events, 14))
        tot = np.zeros(self.n_packets)
        _check(lib().mcrt_histories_records(self.h, rec.ctypes.data, rec.size, tot.ctypes.data, tot.size))
        return rec, tot

    def samples(self):
        n = self.n_samples
        X = np.zeros((n, 9), dtype=np.float32)
        KP = np.zeros((n, 3), dtype=np.float32)
        C = np.zeros(n, dtype=np.float32)
        if n:
            _check(lib().mcrt_histories_samples(self.h, X.ctypes.data, KP.ctypes.data, C.ctypes.data, n))
        return X, KP, C

    def close(self):
        if getattr(self, "h", None):
            lib().mcrt_histories_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handles(objs):
    return (ctypes.c_void_p * len(objs))(*[o.h.value if isinstance(o.h, ctypes.c_void_p) else o.h
                                           for o in objs])


def batch_run_into(sims: Sequence["Sim"], results: Sequence[Result], n_per_lambda: Sequence[int],
                   seed: int = 0) -> int:
    """One persistent launch over many sims (model index = position)."""
    n = len(sims)
    npl = (ctypes.c_uint64 * n)(*[int(x) for x in n_per_lambda])
    return _check(lib().mcrt_batch_run_into(_handles(sims), n, npl, int(seed), _handles(results)),
                  allow=(ELIMIT, ENONFINITE))


def autotune(sims: Sequence["Sim"], trial_packets: Sequence[int], seed: int = 0,
             cache_path: Optional[str] = None) -> dict:
    n = len(sims)
    tp = (ctypes.c_uint64 * n)(*[int(x) for x in trial_packets])
    t = Tuning()
    _check(lib().mcrt_autotune(_handles(sims), n, tp, int(seed),
                               cache_path.encode() if cache_path else None, ctypes.byref(t)))
    return {"chunk": t.chunk, "chunk_shift": t.chunk_shift, "deposit_slots": t.deposit_slots,
            "waves_per_cu": t.waves_per_cu,
            "threshold": t.threshold, "kernel_ms": t.kernel_ms, "default_ms": t.default_ms,
            "from_cache": bool(t.from_cache)}


def run_scene(scene, n_per_lambda: int, seed: int = 0, precision: int = FP32, first_id: int = 0,
              count=None, ctx: Optional[Context] = None, **tune) -> dict:
    """One-call helper: uploads the scene, runs it, returns host arrays in the
    same layout as the oracle (table [n_cells, n_lambda], images list,
    energy, stats)."""
    own = ctx is None
    if own:
        ctx = Context(0)
    sim = Sim(ctx, scene, precision, **tune)
    try:
        res = sim.run(n_per_lambda, seed, first_id, count)
        out = {"table": res.table(), "images": res.images(), "energy": res.energy(),
               "stats": res.stats()}
        res.close()
        return out
    finally:
        sim.close()
        if own:
            ctx.close()
