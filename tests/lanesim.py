"""ctypes wrapper of libmcrt_lanesim.so: the transport kernel's per-lane code
(transport_core.h) compiled for the host and run serially, packet after
packet.  Test harness only: it lets CPU tests check the kernel logic and the
scene setup against the oracle without a GPU."""
import ctypes
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PATH = os.path.join(ROOT, "paper_1705_04702_amd", "libmcrt_lanesim.so")


class _Scene(ctypes.Structure):
    _fields_ = [
        ("grid_type", ctypes.c_int32), ("box", ctypes.c_double * 6), ("n", ctypes.c_int32 * 3),
        ("n_nodes", ctypes.c_int64), ("first_child", ctypes.POINTER(ctypes.c_int32)),
        ("n_cells", ctypes.c_int64), ("density", ctypes.POINTER(ctypes.c_float)),
        ("n_lambda", ctypes.c_int32), ("kappa", ctypes.POINTER(ctypes.c_double)),
        ("albedo", ctypes.POINTER(ctypes.c_double)), ("g", ctypes.POINTER(ctypes.c_double)),
        ("L", ctypes.POINTER(ctypes.c_double)), ("src_type", ctypes.c_int32),
        ("src_pos", ctypes.c_double * 3), ("hR", ctypes.c_double), ("zs", ctypes.c_double),
        ("n_ins", ctypes.c_int32), ("ins_geom", ctypes.POINTER(ctypes.c_double)),
        ("ins_npix", ctypes.POINTER(ctypes.c_int32)), ("w_min", ctypes.c_double),
        ("event_cap", ctypes.c_int64), ("tau_peel_max", ctypes.c_double),
        ("precision", ctypes.c_int32), ("top_level", ctypes.c_int32), ("model", ctypes.c_uint32),
        ("lambda_um", ctypes.POINTER(ctypes.c_double)), ("mlp", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
    ]


class _Out(ctypes.Structure):
    _fields_ = [("table", ctypes.POINTER(ctypes.c_double)), ("images", ctypes.POINTER(ctypes.c_double)),
                ("energy", ctypes.POINTER(ctypes.c_double)), ("stats", ctypes.POINTER(ctypes.c_uint64)),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("hist_total", ctypes.POINTER(ctypes.c_double)),
                ("hist_events", ctypes.c_int32)]


STATS = ["packets", "events", "prop_cells", "locate_cells", "peel_cells", "peel_adds",
         "peel_dropped", "capped", "guard", "nonfinite"]
_SRC = {"point_iso": 0, "point_aniso": 1, "expdisk": 2}
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MCRT_LANESIM_LIB")  # the sanitizer build of the CPU tests
        if not path:
            if not os.path.exists(PATH):
                from paper_1705_04702_amd import build
                build.build_lanesim()
            path = PATH
        _lib = ctypes.CDLL(path)
        _lib.ls_run.argtypes = [ctypes.POINTER(_Scene), ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(_Out)]
        _lib.ls_run.restype = ctypes.c_int
    return _lib


def run(sc, n_per_lambda, seed=0, first_id=0, count=None, precision=1, top_level=-1, model=0,
        mlp=None, alpha=0.2, histories=0):
    """mlp: FP32 network parameters (the simulator rounds the weights to
    bf16 as the library does); histories: events recorded per packet (plain
    runs)."""
    if count is None:
        count = n_per_lambda - first_id
    keep = []

    def arr(a, dt, ct):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ct))

    s = _Scene()
    s.grid_type = 1 if sc.grid_type == "octree" else 0
    for i in range(6):
        s.box[i] = sc.box[i]
    if sc.grid_type == "octree":
        s.n_nodes = int(sc.first_child.shape[0])
        s.first_child = arr(sc.first_child, np.int32, ctypes.c_int32)
    else:
        for i in range(3):
            s.n[i] = sc.n[i]
    s.n_cells = sc.density.shape[0]
    s.density = arr(sc.density, np.float32, ctypes.c_float)
    s.n_lambda = sc.lambdas.shape[0]
    s.kappa = arr(sc.kappa, np.float64, ctypes.c_double)
    s.albedo = arr(sc.albedo, np.float64, ctypes.c_double)
    s.g = arr(sc.hg_g, np.float64, ctypes.c_double)
    s.L = arr(sc.lum, np.float64, ctypes.c_double)
    s.src_type = _SRC[sc.source]
    for i in range(3):
        s.src_pos[i] = sc.src_pos[i]
    s.hR, s.zs = sc.disk_hR, sc.disk_zs
    s.n_ins = len(sc.instruments)
    geom = np.array([[i.incl_deg, i.azim_deg, i.distance, i.fov[0], i.fov[1]] for i in sc.instruments],
                    dtype=np.float64).reshape(-1, 5)
    npix = np.array([[i.npix[0], i.npix[1]] for i in sc.instruments], dtype=np.int32).reshape(-1, 2)
    s.ins_geom = arr(geom, np.float64, ctypes.c_double)
    s.ins_npix = arr(npix, np.int32, ctypes.c_int32)
    s.w_min, s.event_cap, s.tau_peel_max = sc.w_min, sc.event_cap, sc.tau_peel_max
    s.precision = precision
    s.top_level = top_level
    s.model = model
    s.lambda_um = arr(sc.lambdas, np.float64, ctypes.c_double)
    if mlp is not None:
        s.mlp = arr(np.asarray(mlp, dtype=np.float32).astype(np.float64), np.float64, ctypes.c_double)
    s.alpha = alpha
    nl = s.n_lambda
    table = np.zeros(s.n_cells * nl)
    shapes = [(nl, i.npix[1], i.npix[0]) for i in sc.instruments]
    nimg = sum(int(np.prod(x)) for x in shapes)
    images = np.zeros(max(1, nimg))
    energy = np.zeros(4)
    stats = np.zeros(len(STATS), dtype=np.uint64)
    o = _Out(table.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             images.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             energy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             stats.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    npk = count * nl
    if histories:
        hist = np.zeros(npk * histories * 14)
        htot = np.zeros(npk)
        o.hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.hist_total = htot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.hist_events = histories
    rc = lib().ls_run(ctypes.byref(s), n_per_lambda, first_id, count, seed, ctypes.byref(o))
    if rc:
        raise RuntimeError(f"lanesim failed {rc}")
    imgs, off = [], 0
    for x in shapes:
        n = int(np.prod(x))
        imgs.append(images[off:off + n].reshape(x))
        off += n
    res = {"table": table.reshape(s.n_cells, nl), "images": imgs, "energy": energy,
           "stats": dict(zip(STATS, [int(x) for x in stats]))}
    if histories:
        res["hist"] = hist.reshape(-1, histories, 14)
        res["hist_total"] = htot
    return res
