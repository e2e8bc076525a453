"""Pins of the oracle's transport estimator against closed forms, invariants
and an independent analog Monte Carlo.

* energy: emitted = absorbed + escaped + truncated to 1e-12 (FP64), for every
  scene family;
* direct image: a non-scattering medium with a point source gives exactly one
  lit pixel, N L0 exp(-tau_los) / (4 pi d^2), with tau_los from brute-force
  chords;
* uniform cube, no scattering: the escaped fraction equals the quadrature of
  exp(-tau0 / max|k_i|) over the sphere (within the Monte Carlo error);
* optically thin limit: absorbed / ((1 - albedo) mean tau) -> 1 within O(tau);
* Henyey-Greenstein: normalisation by quadrature, sampled moments and a KS
  test against the closed-form CDF; rotation invariants;
* whole estimator (continuous absorption + forced scattering + peel-off) vs an
  analog Monte Carlo with delta tracking, rejection-sampled HG and binned
  escape directions, written independently below;
* split-run additivity (the tables of disjoint packet ranges add up).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_1705_04702_amd import scenes

from test_oracle_geometry import chord


def balance(res):
    e = res["energy"]
    return abs(e[0] - e[1] - e[2] - e[3]) / e[0]


@pytest.mark.parametrize("make", [
    lambda: scenes.sphere(),
    lambda: scenes.sphere(tau=5.0, albedo=0.9, g=-0.3),
    lambda: scenes.uniform_cube(2, 2.0, 0.7, 0.8),
    lambda: scenes.disk((16, 16, 8), 4, 32),
    lambda: scenes.torus(5, 4, 3, 32, n_clumps=30),
])
def test_energy_conservation(make):
    sc = make()
    res = oracle.run(sc, 400, seed=3)
    assert balance(res) < 1e-12
    assert res["energy"][0] == pytest.approx(sc.lum.sum(), rel=1e-12)
    assert np.all(res["table"] >= 0.0)
    assert res["table"].sum() == pytest.approx(res["energy"][1], rel=1e-12)


@pytest.mark.parametrize("incl,azim", [(0.0, 0.0), (60.0, 30.0), (90.0, 0.0)])
def test_direct_image_exact(incl, azim):
    # odd n puts the source at a cell centre, so no ray lies on a cell face and
    # every brute-force chord is unique
    n = 31
    sc = scenes.sphere(n=n, tau=1.0, albedo=0.0, incl_deg=incl, azim_deg=azim)
    N = 500
    res = oracle.run(sc, N, seed=0)
    img = res["images"][0][0]
    nz = np.argwhere(img != 0.0)
    # the central source projects onto a pixel corner and lands in (npix/2, npix/2)
    assert nz.tolist() == [[32, 32]]
    i, a = math.radians(incl), math.radians(azim)
    kobs = np.array([math.sin(i) * math.cos(a), math.sin(i) * math.sin(a), math.cos(i)])
    # tau along kobs from the centre by brute-force chords through every cell
    d = 2.0 / n
    tau = 0.0
    for m in np.flatnonzero(sc.density):
        ix, iy, iz = m % n, (m // n) % n, m // (n * n)
        lo = [-1 + ix * d, -1 + iy * d, -1 + iz * d]
        hi = [lo[0] + d, lo[1] + d, lo[2] + d]
        tau += sc.kappa[0] * sc.density[m] * chord(lo, hi, [0.0, 0.0, 0.0], kobs)
    expect = N * (1.0 / N) * math.exp(-tau) / (4 * math.pi * 100.0 ** 2)
    assert img[32, 32] == pytest.approx(expect, rel=1e-12)


def _cube_escape_moments(tau0):
    """E[exp(-tau0/max|k|)] and E[exp(-2 tau0/max|k|)] over isotropic k, by the
    48-fold symmetry of the cube: phi in [0, pi/4], polar cosine c from
    cos(phi)/sqrt(1+cos^2 phi) to 1 on the +z face."""
    def m(t):
        val, err = integrate.quad(
            lambda phi: integrate.quad(lambda c: math.exp(-t / c),
                                       math.cos(phi) / math.sqrt(1 + math.cos(phi) ** 2), 1.0,
                                       epsabs=1e-14, epsrel=1e-13)[0],
            0.0, math.pi / 4, epsabs=1e-14, epsrel=1e-13)
        return 48.0 / (4.0 * math.pi) * val
    return m(tau0), m(2 * tau0)


def test_cube_escape_quadrature():
    # the quadrature itself: tau0 = 0 must give exactly the whole sphere
    assert _cube_escape_moments(0.0)[0] == pytest.approx(1.0, rel=1e-12)
    tau0 = 1.0
    sc = scenes.uniform_cube(1, tau0, 0.0, 0.0)
    N = 100000
    res = oracle.run(sc, N, seed=11)
    m1, m2 = _cube_escape_moments(tau0)
    sigma = math.sqrt((m2 - m1 * m1) / N)
    assert abs(res["energy"][2] - m1) < 4 * sigma
    assert res["energy"][1] == pytest.approx(1.0 - res["energy"][2], abs=1e-12)


def test_optically_thin_limit():
    tau0, albedo = 1e-3, 0.5
    sc = scenes.uniform_cube(1, tau0, albedo, 0.3)
    N = 50000
    res = oracle.run(sc, N, seed=5)
    # mean tau over the sphere: d/dt of E[exp(-t tau0/max|k|)] at t = 0, by
    # the quadrature of 1/max|k| over the +z face region
    val, _ = integrate.quad(
        lambda phi: integrate.quad(lambda c: 1.0 / c,
                                   math.cos(phi) / math.sqrt(1 + math.cos(phi) ** 2), 1.0)[0],
        0.0, math.pi / 4)
    taubar = tau0 * 48.0 / (4.0 * math.pi) * val
    ratio = res["energy"][1] / ((1.0 - albedo) * taubar)
    assert abs(ratio - 1.0) < 3 * taubar + 0.01


@pytest.mark.parametrize("g", [-0.7, 0.0, 0.3, 0.5, 0.9])
def test_hg_normalisation_and_sampling(g):
    val, _ = integrate.quad(lambda mu: oracle.hg_phase(g, mu), -1.0, 1.0, epsabs=1e-13,
                            epsrel=1e-12, limit=200)
    assert 0.5 * val == pytest.approx(1.0, rel=1e-10)
    rng = np.random.default_rng(7)
    u = rng.random(40000)
    mu = np.array([oracle.hg_sample(g, x) for x in u])
    n = mu.size
    assert abs(mu.mean() - g) < 4 * mu.std() / math.sqrt(n) + 1e-12
    m2 = (1 + 2 * g * g) / 3
    assert abs((mu * mu).mean() - m2) < 4 * (mu * mu).std() / math.sqrt(n) + 1e-12

    def cdf(x):
        if abs(g) < 1e-6:
            return (x + 1) / 2
        return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * x) ** -0.5 - 1 / (1 + g))
    assert stats.kstest(mu, np.vectorize(cdf)).pvalue > 1e-4


def test_rotation_invariants():
    rng = np.random.default_rng(3)
    ks = [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
          np.array([1e-4, 0, math.sqrt(1 - 1e-8)]), np.array([1.0, 0, 0])]
    for _ in range(200):
        k = rng.normal(size=3)
        ks.append(k / np.linalg.norm(k))
    for k in ks:
        for mu in (-1.0, -0.3, 0.0, 0.77, 1.0):
            phi = 2 * math.pi * rng.random()
            kn = np.array(oracle.rotate(list(k), mu, phi))
            assert abs(np.linalg.norm(kn) - 1.0) < 1e-14
            assert abs(kn @ k - mu) < 1e-12
    # azimuth: uniform phi gives a mean direction of mu * k
    k = np.array([0.3, -0.5, 0.81])
    k /= np.linalg.norm(k)
    acc = np.zeros(3)
    for j in range(720):
        acc += np.array(oracle.rotate(list(k), 0.4, 2 * math.pi * (j + 0.5) / 720))
    assert np.allclose(acc / 720, 0.4 * k, atol=1e-12)


# --------------------------------------------------------------------------
# Independent analog Monte Carlo (delta tracking)
# --------------------------------------------------------------------------

def _perp_basis(k):
    a = np.where(np.abs(k[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(k, a)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(k, u)
    return u, v


def _hg_rejection(rng, g, n):
    out = np.empty(n)
    todo = np.arange(n)
    fmax = (1 + abs(g)) / (1 - abs(g)) ** 2
    while todo.size:
        mu = rng.uniform(-1, 1, todo.size)
        f = (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5
        ok = rng.random(todo.size) * fmax < f
        out[todo[ok]] = mu[ok]
        todo = todo[~ok]
    return out


def analog_mc(sc, N, rng, kobs_list, cos_cone):
    """Analog photons: unit weight, free paths by delta tracking against the
    majorant, absorption or HG scattering at real collisions; escapes are
    binned in cones around each observer direction."""
    box = np.array(sc.box)
    n = np.array(sc.n)
    d = (box[3:] - box[:3]) / n
    ext = sc.kappa[0] * sc.density.astype(np.float64)
    emax = ext.max()
    alb, g = sc.albedo[0], sc.hg_g[0]
    pos = np.tile(np.array(sc.src_pos, float), (N, 1))
    mu = rng.uniform(-1, 1, N)
    ph = rng.uniform(0, 2 * math.pi, N)
    st = np.sqrt(1 - mu * mu)
    k = np.stack([st * np.cos(ph), st * np.sin(ph), mu], 1)
    absorbed = np.zeros(sc.n_cells)
    cone = np.zeros(len(kobs_list))
    alive = np.arange(N)
    while alive.size:
        s = -np.log(rng.random(alive.size)) / emax
        pos[alive] += s[:, None] * k[alive]
        p = pos[alive]
        out = np.any((p < box[:3]) | (p > box[3:]), axis=1)
        esc = alive[out]
        for j, ko in enumerate(kobs_list):
            cone[j] += np.count_nonzero(k[esc] @ ko >= cos_cone)
        alive = alive[~out]
        p = pos[alive]
        idx = np.clip(np.floor((p - box[:3]) / d).astype(int), 0, n - 1)
        m = idx[:, 0] + n[0] * (idx[:, 1] + n[1] * idx[:, 2])
        real = rng.random(alive.size) * emax < ext[m]
        u = rng.random(alive.size)
        absb = real & (u >= alb)
        np.add.at(absorbed, m[absb], 1.0)
        scat = real & (u < alb)
        who = alive[scat]
        if who.size:
            mus = _hg_rejection(rng, g, who.size)
            phs = rng.uniform(0, 2 * math.pi, who.size)
            kk = k[who]
            uu, vv = _perp_basis(kk)
            sts = np.sqrt(np.maximum(0, 1 - mus * mus))
            k[who] = (mus[:, None] * kk + (sts * np.cos(phs))[:, None] * uu
                      + (sts * np.sin(phs))[:, None] * vv)
        alive = alive[~absb]
    return absorbed / N, cone / N


@pytest.mark.parametrize("dens,src,alb,g", [
    ((1.0,), (0.0, 0.0, 0.0), 0.6, 0.5),
    ((1.0, 3.0), (0.25, 0.1, -0.2), 0.6, 0.5),
])
def test_whole_estimator_vs_analog_mc(dens, src, alb, g):
    nx = len(dens)
    incls = [(0.0, 0.0), (90.0, 0.0), (90.0, 90.0), (45.0, 200.0)]
    sc = scenes.Scene(
        grid_type="cartesian", box=(-1, -1, -1, 1, 1, 1), n=(nx, 1, 1),
        density=np.array(dens, np.float32), lambdas=np.array([0.55]), kappa=np.array([0.7]),
        albedo=np.array([alb]), hg_g=np.array([g]), lum=np.array([1.0]), source="point_iso",
        src_pos=src, instruments=[scenes.Instrument(i, a, 100.0, (4.0, 4.0), (4, 4))
                                  for i, a in incls], w_min=1e-9)
    # oracle: K independent batches give the spread of the image totals
    K, Nb = 8, 5000
    tables, radiance = [], []
    for b in range(K):
        r = oracle.run(sc, Nb, seed=100 + b)
        assert balance(r) < 1e-12
        tables.append(r["table"][:, 0])
        radiance.append([img.sum() * 100.0 ** 2 for img in r["images"]])
    tables = np.array(tables)
    radiance = np.array(radiance)
    t_mean, t_err = tables.mean(0), tables.std(0, ddof=1) / math.sqrt(K)
    r_mean, r_err = radiance.mean(0), radiance.std(0, ddof=1) / math.sqrt(K)
    # analog
    rng = np.random.default_rng(2024)
    Na = 400000
    kobs = []
    for i, a in incls:
        i, a = math.radians(i), math.radians(a)
        kobs.append(np.array([math.sin(i) * math.cos(a), math.sin(i) * math.sin(a), math.cos(i)]))
    cosc = math.cos(0.12)
    domega = 2 * math.pi * (1 - cosc)
    a_abs, a_cone = analog_mc(sc, Na, rng, kobs, cosc)
    a_abs_err = np.sqrt(a_abs * (1 - a_abs) / Na)
    a_rad = a_cone / domega
    a_rad_err = np.sqrt(a_cone * (1 - a_cone) / Na) / domega
    z_abs = (t_mean - a_abs) / np.sqrt(t_err ** 2 + a_abs_err ** 2)
    z_rad = (r_mean - a_rad) / np.sqrt(r_err ** 2 + a_rad_err ** 2)
    assert np.all(np.abs(z_abs) < 4.0), (t_mean, a_abs, z_abs)
    assert np.all(np.abs(z_rad) < 4.0), (r_mean, a_rad, z_rad)


def test_split_runs_add_up():
    sc = scenes.sphere(n=16, tau=2.0)
    full = oracle.run(sc, 2000, seed=9)
    a = oracle.run(sc, 2000, seed=9, first_id=0, count=1200)
    b = oracle.run(sc, 2000, seed=9, first_id=1200, count=800)
    np.testing.assert_allclose(a["table"] + b["table"], full["table"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(a["images"][0] + b["images"][0], full["images"][0], rtol=1e-12,
                               atol=1e-300)
    np.testing.assert_allclose(a["energy"] + b["energy"], full["energy"], rtol=1e-12)


def test_event_cap_and_termination():
    sc = scenes.sphere(n=16, tau=3.0, albedo=0.9)
    sc.event_cap = 1
    res = oracle.run(sc, 500, seed=1)
    assert res["stats"]["capped"] > 0
    assert res["stats"]["events"] <= 500
    assert balance(res) < 1e-12
    sc.event_cap = 10000
    sc.w_min = 1e-2
    r2 = oracle.run(sc, 500, seed=1)
    assert r2["stats"]["capped"] == 0
    assert r2["energy"][3] > 0 and balance(r2) < 1e-12
    sc.w_min = 1e-9
    r3 = oracle.run(sc, 500, seed=1)
    assert r3["energy"][3] < r2["energy"][3]
    assert r3["energy"][3] / r3["energy"][0] < 1e-8


def test_moments_match_batch_spread():
    """Per-packet second moments give the same standard error as the spread
    of independent runs (checks the O12 bookkeeping)."""
    sc = scenes.sphere(n=8, tau=1.0)
    N = 4000
    r = oracle.run(sc, N, seed=21, moments=True)
    T = r["table"][:, 0]
    var = r["table_m2"][:, 0] - T * T / N
    assert np.all(var >= -1e-15)
    reps = np.array([oracle.run(sc, N, seed=1000 + s)["table"][:, 0] for s in range(30)])
    sd = reps.std(0, ddof=1)
    big = T > 0.2 * T.max()
    ratio = np.sqrt(np.maximum(var[big], 0)) / sd[big]
    assert 0.6 < np.median(ratio) < 1.6


def test_threaded_id_ranges_equal_one_run():
    """The test harness's threaded oracle (disjoint id ranges, summed) equals
    one serial run, second moments included."""
    import oracle_par
    sc = scenes.disk((16, 16, 8), 3, 24)
    a = oracle.run(sc, 900, seed=4, first_id=17, count=613, moments=True)
    b = oracle_par.run(sc, 900, seed=4, first_id=17, count=613, moments=True, threads=5)
    for k in ("table", "table_m2"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=0)
    for x, y in zip(b["images"] + b["image_m2"], a["images"] + a["image_m2"]):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=0)
    np.testing.assert_allclose(b["energy"], a["energy"], rtol=1e-12)
    assert b["stats"] == a["stats"]
