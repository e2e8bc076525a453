"""Seeded synthetic scenes: dust grids, media, sources and instruments.

This module only builds inputs.  It holds none of the transport arithmetic
(no ray marching, sampling or tallying), so both the GPU library and the CPU
oracle can be fed from it.

The workloads stand in for the models of the hybrid-parallel SKIRT paper
(Section 7.2 spiral-galaxy test model, Section 2 clumpy AGN tori, Section 3.1
batches of small models); the paper gives no parameters for them, so the
recipes below are synthetic and seeded:

* ``sphere``   -- uniform sphere of radius 1 on a Cartesian grid in [-1, 1]^3,
  central isotropic point source (a cell is dust-filled when its centre lies
  inside the sphere, so the radial optical depth along each axis is exact).
* ``disk``     -- double-exponential dust disk (scale length 4.5 kpc, height
  0.15 kpc) with an exponential stellar disk (3 kpc, sech^2 height 0.3 kpc),
  power-law opacity and albedo over log-spaced wavelengths.
* ``torus``    -- clumpy two-phase wedge torus on an octree, central
  anisotropic source.
* ``batch``    -- many small uniform-sphere or exponential-slab models.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Instrument:
    """Distant parallel-projection observer."""

    incl_deg: float
    azim_deg: float
    distance: float
    fov: Tuple[float, float]
    npix: Tuple[int, int]


@dataclasses.dataclass
class Scene:
    grid_type: str                      # "cartesian" | "octree"
    box: Tuple[float, ...]              # xmin, ymin, zmin, xmax, ymax, zmax
    density: np.ndarray                 # float32 [n_cells]
    lambdas: np.ndarray                 # float64 [n_lambda] (micron)
    kappa: np.ndarray                   # float64 [n_lambda]
    albedo: np.ndarray                  # float64 [n_lambda]
    hg_g: np.ndarray                    # float64 [n_lambda]
    lum: np.ndarray                     # float64 [n_lambda]
    source: str                         # "point_iso" | "point_aniso" | "expdisk"
    instruments: List[Instrument]
    n: Tuple[int, int, int] = (0, 0, 0)            # Cartesian cell counts
    first_child: Optional[np.ndarray] = None       # int32 [n_nodes] (octree)
    src_pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    disk_hR: float = 0.0
    disk_zs: float = 0.0
    w_min: float = 1e-6
    event_cap: int = 10000
    tau_peel_max: float = math.inf                 # no peel-off is cut (the definition)
    name: str = ""

    @property
    def n_cells(self) -> int:
        return int(self.density.shape[0])

    @property
    def n_lambda(self) -> int:
        return int(self.lambdas.shape[0])

    def image_shapes(self) -> List[Tuple[int, int, int]]:
        return [(self.n_lambda, ins.npix[1], ins.npix[0]) for ins in self.instruments]


def _cell_centres(box: Sequence[float], n: Sequence[int]):
    axes = []
    for a in range(3):
        lo, hi = box[a], box[3 + a]
        d = (hi - lo) / n[a]
        axes.append(lo + (np.arange(n[a]) + 0.5) * d)
    # cell index m = ix + nx * (iy + ny * iz): z slowest, x fastest
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def log_lambdas(n_lambda: int, lo: float = 0.1, hi: float = 1000.0) -> np.ndarray:
    if n_lambda == 1:
        return np.array([0.55])
    return np.exp(np.linspace(math.log(lo), math.log(hi), n_lambda))


def powerlaw_optics(lambdas: np.ndarray, kappa_v: float, g: float):
    """kappa = kappa_V (lambda/0.55)^-1, albedo = min(0.7, 0.55 (lambda/0.55)^-0.25)."""
    x = lambdas / 0.55
    kappa = kappa_v * x ** -1.0
    albedo = np.minimum(0.7, 0.55 * x ** -0.25)
    return kappa.astype(np.float64), albedo.astype(np.float64), np.full_like(kappa, g)


def sphere(n: int = 32, tau: float = 1.0, albedo: float = 0.5, g: float = 0.5,
           npix: int = 64, distance: float = 100.0, incl_deg: float = 0.0,
           azim_deg: float = 0.0, w_min: float = 1e-6) -> Scene:
    """Uniform sphere (radius 1, radial optical depth tau) with a central
    isotropic unit-luminosity point source, one wavelength."""
    box = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    x, y, z = _cell_centres(box, (n, n, n))
    inside = (x * x + y * y + z * z) <= 1.0
    dens = np.where(inside, 1.0, 0.0).astype(np.float32).ravel()
    return Scene(
        grid_type="cartesian", box=box, n=(n, n, n), density=dens,
        lambdas=np.array([0.55]), kappa=np.array([float(tau)]),
        albedo=np.array([float(albedo)]), hg_g=np.array([float(g)]),
        lum=np.array([1.0]), source="point_iso",
        instruments=[Instrument(incl_deg, azim_deg, distance, (2.0, 2.0), (npix, npix))],
        w_min=w_min, name=f"sphere{n}")


def uniform_cube(n: int = 1, tau0: float = 1.0, albedo: float = 0.0, g: float = 0.0,
                 npix: int = 8, incl_deg: float = 0.0, azim_deg: float = 0.0,
                 src=(0.0, 0.0, 0.0)) -> Scene:
    """Uniform cube [-1, 1]^3 (centre-to-face optical depth tau0), point source."""
    box = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    dens = np.ones(n * n * n, dtype=np.float32)
    return Scene(
        grid_type="cartesian", box=box, n=(n, n, n), density=dens,
        lambdas=np.array([0.55]), kappa=np.array([float(tau0)]),
        albedo=np.array([float(albedo)]), hg_g=np.array([float(g)]),
        lum=np.array([1.0]), source="point_iso", src_pos=tuple(src),
        instruments=[Instrument(incl_deg, azim_deg, 100.0, (2.0, 2.0), (npix, npix))],
        name=f"cube{n}")


def disk(n: Tuple[int, int, int] = (256, 256, 256), n_lambda: int = 64, npix: int = 512,
         incl: Sequence[float] = (0.0, 60.0, 90.0), tau_v_faceon: float = 1.0) -> Scene:
    """Exponential-disk galaxy (kpc units).

    Dust: rho = rho0 exp(-R/4.5 - |z|/0.15) sampled at cell centres, with
    kappa_V rho0 chosen so that the analytic face-on optical depth through the
    centre, 2 kappa_V rho0 h_z, equals tau_v_faceon.  Stars: exponential disk,
    h_R = 3, sech^2 vertical profile with z_s = 0.3.  Box [-20, 20]^2 x [-2, 2].
    Instruments at 10 Mpc with a 40 x 40 kpc field of view.
    """
    box = (-20.0, -20.0, -2.0, 20.0, 20.0, 2.0)
    hR_d, hz_d = 4.5, 0.15
    x, y, z = _cell_centres(box, n)
    R = np.sqrt(x * x + y * y)
    rho0 = tau_v_faceon / (2.0 * hz_d)
    dens = (rho0 * np.exp(-R / hR_d - np.abs(z) / hz_d)).astype(np.float32).ravel()
    lam = log_lambdas(n_lambda)
    kappa, albedo, g = powerlaw_optics(lam, 1.0, 0.6)
    ins = [Instrument(float(i), 0.0, 1.0e4, (40.0, 40.0), (npix, npix)) for i in incl]
    return Scene(
        grid_type="cartesian", box=box, n=tuple(n), density=dens, lambdas=lam,
        kappa=kappa, albedo=albedo, hg_g=g, lum=np.ones(n_lambda), source="expdisk",
        disk_hR=3.0, disk_zs=0.3, instruments=ins, name=f"disk{n[0]}x{n[1]}x{n[2]}_l{n_lambda}")


# ----------------------------------------------------------------------------
# Octree torus
# ----------------------------------------------------------------------------

def _morton(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray, depth: int) -> np.ndarray:
    code = np.zeros(ix.shape, dtype=np.int64)
    for b in range(depth - 1, -1, -1):
        code = (code << 3) | (((ix >> b) & 1) + 2 * ((iy >> b) & 1) + 4 * ((iz >> b) & 1))
    return code


def octree_from_levels(refine_fn, max_depth: int):
    """Builds an octree top-down.  refine_fn(level, ix, iy, iz) -> bool mask of
    the nodes (lattice coordinates at that level) to subdivide.

    Returns (first_child int32 [n_nodes], leaves) where leaves is a tuple of
    arrays (level, ix, iy, iz) in depth-first leaf order (children visited in
    the order c = bx + 2 by + 4 bz).  Children of a node are contiguous.
    """
    first_child = [np.array([-1], dtype=np.int64)]
    level_nodes = [(np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(1, np.int64))]
    base = [0]
    total = 1
    leaf_parts = []
    for level in range(max_depth + 1):
        ix, iy, iz = level_nodes[level]
        if level < max_depth:
            ref = np.asarray(refine_fn(level, ix, iy, iz), dtype=bool)
        else:
            ref = np.zeros(ix.shape, dtype=bool)
        nref = int(ref.sum())
        fc = first_child[level]
        ranks = np.cumsum(ref) - 1
        fc[ref] = total + 8 * ranks[ref]
        leaf = ~ref
        leaf_parts.append((np.full(int(leaf.sum()), level, np.int64), ix[leaf], iy[leaf], iz[leaf]))
        if nref == 0:
            break
        c = np.arange(8)
        bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cx = (2 * ix[ref][:, None] + bx[None, :]).ravel()
        cy = (2 * iy[ref][:, None] + by[None, :]).ravel()
        cz = (2 * iz[ref][:, None] + bz[None, :]).ravel()
        level_nodes.append((cx, cy, cz))
        first_child.append(np.full(cx.shape[0], -1, dtype=np.int64))
        base.append(total)
        total += cx.shape[0]
    depth = len(leaf_parts) - 1
    fc_all = np.concatenate(first_child).astype(np.int32)
    lv = np.concatenate([p[0] for p in leaf_parts])
    lx = np.concatenate([p[1] for p in leaf_parts])
    ly = np.concatenate([p[2] for p in leaf_parts])
    lz = np.concatenate([p[3] for p in leaf_parts])
    sh = depth - lv
    order = np.argsort(_morton(lx << sh, ly << sh, lz << sh, depth), kind="stable")
    return fc_all, (lv[order], lx[order], ly[order], lz[order]), depth


def random_octree(max_depth: int = 3, p_refine: float = 0.5, seed: int = 0):
    """Random octree over [0,1]^3 for geometry tests: each node below
    max_depth is refined with probability p_refine (the root always)."""
    rng = np.random.default_rng(seed)

    def refine(level, ix, iy, iz):
        if level == 0:
            return np.ones(ix.shape, bool)
        return rng.random(ix.shape[0]) < p_refine

    return octree_from_levels(refine, max_depth)


def uniform_octree(depth: int):
    return octree_from_levels(lambda level, ix, iy, iz: np.ones(ix.shape, bool), depth)


def torus(max_depth: int = 9, torus_depth: int = 8, n_lambda: int = 32, npix: int = 1024,
          seed: int = 3, clump_radius: float = 0.4, fill: float = 0.03,
          contrast: float = 100.0, tau_eq: float = 50.0, r_in: float = 0.5,
          r_out: float = 15.0, half_open_deg: float = 40.0, incl_deg: float = 90.0,
          n_clumps: Optional[int] = None, min_depth: Optional[int] = None) -> Scene:
    """Clumpy two-phase wedge torus (pc units) on an octree over [-15, 15]^3.

    The medium is voxelised on the 2^max_depth lattice at voxel centres:
    outside the torus (density 0), inter-clump (rho_ic) or clump
    (contrast * rho_ic).  Clump centres are uniform in the torus volume; their
    number gives the requested volume filling factor.  A node is subdivided
    while its voxels are not all of one phase, down to max_depth when it holds
    clump voxels and to torus_depth otherwise; a leaf's density is the mean of
    its voxels.  kappa_V rho_ic is set so that kappa_V rho_mean (r_out - r_in)
    = tau_eq with rho_mean = rho_ic (1 + fill (contrast - 1)).
    """
    rng = np.random.default_rng(seed)
    if min_depth is None:
        min_depth = max_depth - 2
    half = r_out
    box = (-half, -half, -half, half, half, half)
    N = 1 << max_depth
    d = 2.0 * half / N
    sin_open = math.sin(math.radians(half_open_deg))
    rho_ic = tau_eq / ((r_out - r_in) * (1.0 + fill * (contrast - 1.0)))
    v_torus = 4.0 / 3.0 * math.pi * (r_out ** 3 - r_in ** 3) * sin_open
    if n_clumps is None:
        n_clumps = int(round(fill * v_torus / (4.0 / 3.0 * math.pi * clump_radius ** 3)))
    centres = []
    while len(centres) < n_clumps:
        p = rng.uniform(-r_out, r_out, size=(4 * n_clumps + 16, 3))
        rr = np.sqrt((p * p).sum(1))
        ok = (rr >= r_in) & (rr <= r_out) & (np.abs(p[:, 2]) <= sin_open * rr)
        centres.extend(p[ok][: n_clumps - len(centres)].tolist())
    centres = np.array(centres[:n_clumps], dtype=np.float64).reshape(-1, 3)

    coords = -half + (np.arange(N) + 0.5) * d
    phase = np.zeros((N, N, N), dtype=np.uint8)          # [iz, iy, ix]
    yy, xx = np.meshgrid(coords, coords, indexing="ij")
    for iz in range(N):
        zc = coords[iz]
        rr = np.sqrt(xx * xx + yy * yy + zc * zc)
        tor = (rr >= r_in) & (rr <= r_out) & (abs(zc) <= sin_open * rr)
        phase[iz][tor] = 1
    rc = clump_radius
    for c in centres:
        lo = np.clip(np.floor((c - rc + half) / d).astype(int), 0, N - 1)
        hi = np.clip(np.floor((c + rc + half) / d).astype(int), 0, N - 1)
        sx = coords[lo[0]:hi[0] + 1]
        sy = coords[lo[1]:hi[1] + 1]
        sz = coords[lo[2]:hi[2] + 1]
        Z, Y, X = np.meshgrid(sz, sy, sx, indexing="ij")
        inside = ((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= rc * rc
        sub = phase[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[inside & (sub >= 1)] = 2

    # min / max / sum pyramids, index [level] -> array [iz, iy, ix]
    dens_vox = np.array([0.0, rho_ic, contrast * rho_ic])
    pmin = [None] * (max_depth + 1)
    pmax = [None] * (max_depth + 1)
    psum = [None] * (max_depth + 1)
    pmin[max_depth] = phase
    pmax[max_depth] = phase
    psum[max_depth] = dens_vox[phase]
    for level in range(max_depth - 1, -1, -1):
        m = 1 << level
        pmin[level] = pmin[level + 1].reshape(m, 2, m, 2, m, 2).min(axis=(1, 3, 5))
        pmax[level] = pmax[level + 1].reshape(m, 2, m, 2, m, 2).max(axis=(1, 3, 5))
        psum[level] = psum[level + 1].reshape(m, 2, m, 2, m, 2).sum(axis=(1, 3, 5))

    def refine(level, ix, iy, iz):
        mn = pmin[level][iz, iy, ix]
        mx = pmax[level][iz, iy, ix]
        mixed = mn != mx
        lim = np.where(mx == 2, max_depth, torus_depth)
        return (mixed & (level < lim)) | ((mx >= 1) & (level < min_depth))

    first_child, (lv, lx, ly, lz), depth = octree_from_levels(refine, max_depth)
    dens = np.empty(lv.shape[0], dtype=np.float64)
    for level in np.unique(lv):
        sel = lv == level
        dens[sel] = psum[level][lz[sel], ly[sel], lx[sel]] / float(8 ** (max_depth - level))
    lam = log_lambdas(n_lambda)
    kappa, albedo, g = powerlaw_optics(lam, 1.0, 0.6)
    kappa = kappa * rho_ic  # fold rho_ic into kappa: densities become 0 .. contrast
    dens = dens / rho_ic
    return Scene(
        grid_type="octree", box=box, first_child=first_child,
        density=dens.astype(np.float32), lambdas=lam, kappa=kappa, albedo=albedo, hg_g=g,
        lum=np.ones(n_lambda), source="point_aniso",
        instruments=[Instrument(incl_deg, 0.0, 1.0e7, (2 * half, 2 * half), (npix, npix))],
        name=f"torus_d{max_depth}_l{n_lambda}")


# ----------------------------------------------------------------------------
# Initial weights of the direction-proposal network
# ----------------------------------------------------------------------------

MLP_SHAPES = [(9, 64), (64,), (64, 64), (64,), (64, 40), (40,)]


def init_mlp(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Seeded fan-in uniform initial parameters (float32, flat: W1 [9][64],
    b1, W2 [64][64], b2, W3 [64][40], b3), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            bound = scale * math.sqrt(6.0 / shape[0])
            parts.append(rng.uniform(-bound, bound, shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------
# Batch of small models
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class BatchModel:
    scene: Scene
    n_packets: int
    kind: str
    tau: float


def batch_table(n_models: int = 256, seed: int = 4, side=(16, 128), tau=(0.1, 20.0),
                packets=(1e5, 1e7)):
    """Draws the batch model table: side log-uniform, tau log-uniform,
    albedo U(0.3, 0.7), g U(0, 0.8), packets log-uniform, kind sphere/slab."""
    rng = np.random.default_rng(seed)
    rows = []
    for b in range(n_models):
        n = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
        t = float(math.exp(rng.uniform(math.log(tau[0]), math.log(tau[1]))))
        a = float(rng.uniform(0.3, 0.7))
        g = float(rng.uniform(0.0, 0.8))
        p = int(round(math.exp(rng.uniform(math.log(packets[0]), math.log(packets[1])))))
        kind = "sphere" if rng.random() < 0.5 else "slab"
        rows.append(dict(n=n, tau=t, albedo=a, g=g, packets=p, kind=kind))
    return rows


def batch_model(row, npix: int = 128) -> Scene:
    n = row["n"]
    box = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    x, y, z = _cell_centres(box, (n, n, n))
    if row["kind"] == "sphere":
        dens = np.where(x * x + y * y + z * z <= 1.0, 1.0, 0.0)
        kappa = row["tau"]  # radial optical depth, radius 1
    else:
        hz = 0.2
        dens = np.exp(-np.abs(z) / hz)
        kappa = row["tau"] / (hz * (1.0 - math.exp(-1.0 / hz)))  # midplane to z = 1
    return Scene(
        grid_type="cartesian", box=box, n=(n, n, n), density=dens.astype(np.float32).ravel(),
        lambdas=np.array([0.55]), kappa=np.array([kappa]), albedo=np.array([row["albedo"]]),
        hg_g=np.array([row["g"]]), lum=np.array([1.0]), source="point_iso",
        instruments=[Instrument(60.0, 0.0, 100.0, (2.0, 2.0), (npix, npix))],
        name=f"batch_{row['kind']}{n}")


def batch(n_models: int = 256, seed: int = 4, packet_scale: float = 1.0, **kw) -> List[BatchModel]:
    out = []
    for row in batch_table(n_models, seed, **kw):
        out.append(BatchModel(batch_model(row), max(1, int(round(row["packets"] * packet_scale))),
                              row["kind"], row["tau"]))
    return out
