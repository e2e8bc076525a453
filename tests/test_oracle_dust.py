"""Pins of the oracle's dust emission phase (Section 3.2, dust emission and
self-absorption phases; a modified blackbody stands in for the paper's dust
model files): the Planck function against the Stefan-Boltzmann law, Wien's
displacement law and the Rayleigh-Jeans limit; bin widths of a log grid in
closed form; per-cell energy conservation and the temperature scaling law;
the peak of the emitted spectrum against the textbook modified-blackbody
peak; the launch positions of dust packets."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_1705_04702_amd import scenes

SIGMA = 5.670374419e-8        # W m^-2 K^-4 (CODATA)
WIEN_B = 2897.771955          # micron K (CODATA)
C2 = 14387.76877              # h c / k in micron K


def test_planck_stefan_boltzmann():
    for T in (15.0, 40.0, 300.0):
        lam = np.geomspace(1e-2, 1e6, 40001)
        B = np.array([oracle.planck(x, T) for x in lam])
        integral = np.trapezoid(B * lam * 1e-6, np.log(lam))  # d lambda = lambda d ln lambda (metres)
        assert integral == pytest.approx(SIGMA * T ** 4 / np.pi, rel=1e-6)


def test_planck_wien_and_rayleigh_jeans():
    T = 50.0
    lam = np.linspace(40.0, 80.0, 400001)
    B = np.array([oracle.planck(x, T) for x in lam])
    assert lam[np.argmax(B)] * T == pytest.approx(WIEN_B, abs=(lam[1] - lam[0]) * T)
    x = 1e5  # micron: h c / (lambda k T) = 2.9e-3
    rj = 2.0 * 2.99792458e8 * 1.380649e-23 * T / (x * 1e-6) ** 4
    assert oracle.planck(x, T) == pytest.approx(rj, rel=2e-3)


def test_bin_widths_log_grid():
    lam = np.geomspace(0.1, 1000.0, 33)
    q = lam[1] / lam[0]
    w = oracle.bin_widths(lam)
    assert np.allclose(w, lam * (np.sqrt(q) - 1.0 / np.sqrt(q)), rtol=1e-12)


def _two_cell_scene(n_lambda=200, lo=1.0, hi=1e4, beta=0.0):
    sc = scenes.uniform_cube(n=2, tau0=1.0)
    lam = np.geomspace(lo, hi, n_lambda)
    sc.lambdas = lam
    sc.kappa = lam ** -beta
    sc.albedo = np.zeros(n_lambda)
    sc.hg_g = np.zeros(n_lambda)
    sc.lum = np.ones(n_lambda)
    return sc


def test_energy_conservation_and_temperature_law():
    sc = _two_cell_scene(40)
    rng = np.random.default_rng(3)
    table = rng.random((8, 40)) * 10.0 ** rng.integers(-3, 3, (8, 1))
    table[5] = 0.0  # a cell that absorbed nothing emits nothing
    T, em = oracle.dust_emission(sc, table, T0=25.0, beta=1.5)
    assert np.allclose(em.sum(axis=1), table.sum(axis=1), rtol=1e-12, atol=0)
    assert T[5] == 0.0 and not em[5].any()
    # uniform density: T / T0 = (absorbed / mean absorbed)^(1 / (4 + beta))
    u = table.sum(axis=1)
    ratio = (T[u > 0] / T[u > 0][0]) ** (4 + 1.5)
    assert np.allclose(ratio, u[u > 0] / u[u > 0][0], rtol=1e-12)
    uni = np.ones((8, 40))
    T, _ = oracle.dust_emission(sc, uni, T0=25.0, beta=1.5)
    assert np.allclose(T, 25.0, rtol=1e-14)


@pytest.mark.parametrize("beta", [0.0, 2.0])
def test_emission_peak_modified_blackbody(beta):
    """Emission per unit ln(lambda) of kappa ~ lambda^-beta grains peaks where
    x = h c / (lambda k T) solves x = (4 + beta)(1 - e^-x)."""
    sc = _two_cell_scene(2000, 10.0, 2000.0, beta)
    T, em = oracle.dust_emission(sc, np.ones((8, 2000)), T0=20.0, beta=beta)
    lam = np.asarray(sc.lambdas)
    per_lnlam = em[0] / np.log(lam[1] / lam[0])
    x = brentq(lambda x: x - (4 + beta) * (1 - np.exp(-x)), 1.0, 20.0)
    step = np.log(lam[1] / lam[0])
    assert np.log(lam[np.argmax(per_lnlam)] * 20.0 / (C2 / x)) == pytest.approx(0.0, abs=1.5 * step)


def test_dust_packets_start_in_emitting_cells():
    """Optically thin 4^3 grid, face-on instrument with one pixel per cell
    column: only the columns of the two emitting cells receive flux, in the
    ratio of their emission (3 : 1) within the Monte Carlo error."""
    sc = scenes.uniform_cube(n=4, tau0=1e-9, npix=4)
    emis = np.zeros((64, 1))
    emis[1 + 4 * 2 + 16 * 1, 0] = 3.0   # cell (1, 2, 1)
    emis[3 + 4 * 0 + 16 * 3, 0] = 1.0   # cell (3, 0, 3)
    ds = oracle.dust_scene(sc, emis)
    r = oracle.run(ds, 20000, seed=7)
    img = r["images"][0][0]
    on = np.zeros((4, 4), bool)
    # face-on at azimuth 0: image x along world y, image y along -world x
    on[2, 2] = on[0, 0] = True
    assert not img[~on].any()
    a, b = img[2, 2], img[0, 0]
    assert a / b == pytest.approx(3.0, rel=0.05)
    e = r["energy"]
    assert e[0] == pytest.approx(4.0, rel=1e-12)
    assert abs(e[0] - e[1] - e[2] - e[3]) <= 1e-12 * e[0]


def test_self_absorption_cycles_conserve_energy():
    sc = scenes.disk(n=(12, 12, 8), n_lambda=6, npix=12, tau_v_faceon=5.0)
    st = oracle.run(sc, 150, seed=1)
    cyc = oracle.self_absorption(sc, st["table"], 100, seed=3, cycles=3)
    for L, r in cyc:
        e = r["energy"]
        assert e[0] == pytest.approx(L.sum(), rel=1e-12)
        assert abs(e[0] - e[1] - e[2] - e[3]) <= 1e-12 * e[0]
    # the dust emits the stellar absorption plus its own: more after cycle 1
    assert cyc[1][0].sum() > cyc[0][0].sum()
    assert cyc[0][0].sum() == pytest.approx(st["table"].sum(), rel=1e-12)


def _oct_scene(seed=3, depth=3, npix=8):
    fc, leaves, D = scenes.random_octree(depth, 0.5, seed)
    nl = leaves[0].shape[0]
    sc = scenes.Scene(grid_type="octree", box=(-1.0, -1.0, -1.0, 1.0, 1.0, 1.0), first_child=fc,
                      density=np.full(nl, 1e-9, np.float32), lambdas=np.array([1.0]), kappa=np.array([1.0]),
                      albedo=np.array([0.0]), hg_g=np.array([0.0]), lum=np.array([1.0]), source="point_iso",
                      instruments=[scenes.Instrument(0.0, 0.0, 100.0, (2.0, 2.0), (npix, npix))])
    return sc, leaves, D


def test_octree_temperature_weights_leaf_volume():
    """Absorption proportional to leaf volume at uniform density is uniform
    heating per unit mass: every leaf sits at T0."""
    sc, (lv, lx, ly, lz), D = _oct_scene()
    sc.lambdas = np.array([200.0])  # where an 18 K grain emits
    assert len(set(lv.tolist())) > 1
    table = (8.0 ** -lv.astype(np.float64))[:, None] * np.array([[3.0]])
    T, em = oracle.dust_emission(sc, table, T0=18.0, beta=2.0)
    assert np.allclose(T, 18.0, rtol=1e-13)
    assert np.allclose(em[:, 0], table[:, 0], rtol=1e-13)


def test_octree_dust_packets_start_in_their_leaf():
    """Two emitting leaves of different size: the face-on image (one pixel
    per finest lattice column) has flux only over their footprints, in the
    ratio of their emission."""
    sc, (lv, lx, ly, lz), D = _oct_scene(npix=8)
    N = 1 << D
    big = int(np.argmin(lv))
    small = [m for m in range(lv.size) if lv[m] == lv.max()]
    def foot(m):
        size = 1 << (D - lv[m])
        x0, y0 = lx[m] * size, ly[m] * size
        px = np.zeros((N, N), bool)
        # image x along world y, image y along -world x
        for ix in range(x0, x0 + size):
            for iy in range(y0, y0 + size):
                px[N - 1 - ix, iy] = True
        return px
    fb = foot(big)
    small = next(m for m in small if not (foot(m) & fb).any())
    fs = foot(small)
    emis = np.zeros((lv.size, 1))
    emis[big, 0], emis[small, 0] = 1.0, 2.0
    r = oracle.run(oracle.dust_scene(sc, emis), 20000, seed=11)
    img = r["images"][0][0]
    assert not img[~(fb | fs)].any()
    assert img[fs].sum() / img[fb].sum() == pytest.approx(2.0, rel=0.05)
    # within the big leaf's footprint the flux is spread over all its columns
    assert (img[fb] > 0).all()
