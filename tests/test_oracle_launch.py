"""Pins of the oracle's launch step (Section 3.2: the launch position and
direction are determined by Monte Carlo sampling from the source).

The oracle's own launch is read back through its history records: event 0 of
every packet holds the launch position (as r / r_out, r_out = half the
largest box side) and the emission direction.  The samples are compared with
the closed-form laws of the sources, written out here from their densities:

* exponential disk, surface density ~ exp(-R/h_R): the radius of a point
  drawn from the disk follows p(R) = R exp(-R/h_R) / h_R^2, a Gamma(2) law
  with scale h_R; the azimuth is uniform; the height follows the sech^2 law
  p(z) = sech^2(z/z_s) / (2 z_s), the logistic law with scale z_s / 2;
  radius, azimuth and height are independent;
* anisotropic point source, angular distribution S(k) = 2|k_z| (normalised
  to average 1 over the sphere): mu = k_z has density |mu| on [-1, 1], CDF
  (1 - mu^2)/2 below 0 and (1 + mu^2)/2 above; the azimuth is uniform;
* isotropic point source: mu uniform on [-1, 1].

The emission peel-off of the anisotropic source is pinned by its direct image
in a transparent medium, one pixel of value N L0 S(k_obs) / (4 pi d^2), and
by Gauss-Legendre quadrature of those values over the observer's inclination,
which must give the sphere average of S, 1.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1705_04702_amd import scenes

P_MIN = 1e-4     # the seeds are fixed, so each p-value is a fixed number


def _launch_records(sc, n, seed):
    """Launch positions [n, 3] and directions [n, 3] of packets 0 .. n-1."""
    res = oracle.run(sc, n, seed=seed, histories=1)
    rec = res["hist"][:, 0, :]
    r_out = 0.5 * max(sc.box[3 + a] - sc.box[a] for a in range(3))
    return rec[:, 0:3] * r_out, rec[:, 9:12]


def _transparent(sc):
    sc.density[:] = 0.0
    return sc


def _disk_scene():
    sc = _transparent(scenes.disk((8, 8, 4), 1, 8))
    sc.instruments = sc.instruments[:1]
    return sc


def test_disk_launch_radius_azimuth_height():
    sc = _disk_scene()
    N = 200_000
    r, k = _launch_records(sc, N, seed=11)
    R = np.hypot(r[:, 0], r[:, 1])
    phi = np.arctan2(r[:, 1], r[:, 0])
    z = r[:, 2]
    # radius: Gamma(2) with scale h_R, CDF 1 - (1 + R/h) exp(-R/h)
    hR, zs = sc.disk_hR, sc.disk_zs
    cdf_R = lambda x: 1.0 - (1.0 + x / hR) * np.exp(-x / hR)
    assert stats.kstest(R, cdf_R).pvalue > P_MIN
    # the radius law's first two moments: E[R] = 2 h, E[R^2] = 6 h^2
    assert abs(R.mean() - 2 * hR) < 4 * math.sqrt(2) * hR / math.sqrt(N)
    # azimuth: uniform on (-pi, pi]
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > P_MIN
    # height: sech^2(z/z_s) / (2 z_s), CDF (1 + tanh(z/z_s)) / 2
    cdf_z = lambda x: 0.5 * (1.0 + np.tanh(x / zs))
    assert stats.kstest(z, cdf_z).pvalue > P_MIN
    assert stats.kstest(z, stats.logistic(scale=zs / 2).cdf).pvalue > P_MIN
    # independence: rank correlations vanish within 5 / sqrt(N)
    for a, b in ((R, np.abs(z)), (R, phi), (phi, z), (R, z)):
        assert abs(stats.spearmanr(a, b).statistic) < 5.0 / math.sqrt(N)
    # the direction of a disk packet is isotropic
    assert np.allclose(np.linalg.norm(k, axis=1), 1.0, atol=1e-12)
    assert stats.kstest(k[:, 2], stats.uniform(-1, 2).cdf).pvalue > P_MIN


def test_disk_launch_face_on_image_follows_surface_density():
    """Transparent disk: the face-on emission image is the projected launch
    density; the flux inside radius R over the total is the Gamma(2) CDF."""
    sc = _disk_scene()
    sc.instruments = [scenes.Instrument(0.0, 0.0, 1.0e4, (40.0, 40.0), (64, 64))]
    N = 100_000
    img = oracle.run(sc, N, seed=3)["images"][0][0]
    # pixel centres on the sky: x along e_x = (0, 1, 0), y along e_y = (-1, 0, 0)
    c = (np.arange(64) + 0.5) * (40.0 / 64) - 20.0
    yy, xx = np.meshgrid(c, c, indexing="ij")
    Rpix = np.hypot(xx, yy)
    tot = img.sum()
    # the disk's packets that launch outside the 40 kpc field are not imaged
    hR = sc.disk_hR
    for Rc in (2.0, 4.0, 8.0, 12.0):
        # pixel-centre binning smears R by at most half a pixel diagonal
        lo = 1.0 - (1.0 + (Rc - 0.45) / hR) * math.exp(-(Rc - 0.45) / hR)
        hi = 1.0 - (1.0 + (Rc + 0.45) / hR) * math.exp(-(Rc + 0.45) / hR)
        frac = img[Rpix < Rc].sum() / (N * (1.0 / N)) * (4 * math.pi * 1.0e4 ** 2)
        sig = math.sqrt(hi * (1 - hi) / N)
        assert lo - 5 * sig <= frac <= hi + 5 * sig
    assert tot > 0


def _point_scene(aniso, incl=(0.0,)):
    sc = _transparent(scenes.sphere(n=4, tau=1.0, albedo=0.0))
    sc.source = "point_aniso" if aniso else "point_iso"
    sc.instruments = [scenes.Instrument(float(i), 0.0, 100.0, (2.0, 2.0), (8, 8)) for i in incl]
    return sc


def test_anisotropic_direction_law():
    sc = _point_scene(True)
    N = 200_000
    _, k = _launch_records(sc, N, seed=7)
    assert np.allclose(np.linalg.norm(k, axis=1), 1.0, atol=1e-12)
    mu = k[:, 2]
    cdf = lambda m: np.where(m < 0.0, 0.5 * (1.0 - m * m), 0.5 * (1.0 + m * m))
    assert stats.kstest(mu, cdf).pvalue > P_MIN
    # |mu| has density 2|mu| on [0, 1]: E|mu| = 2/3, E mu^2 = 1/2; P(mu > 0) = 1/2
    assert abs(np.abs(mu).mean() - 2.0 / 3.0) < 4 * math.sqrt(1.0 / 18.0 / N)
    assert abs((mu > 0).mean() - 0.5) < 4 * 0.5 / math.sqrt(N)
    phi = np.arctan2(k[:, 1], k[:, 0])
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > P_MIN
    assert abs(stats.spearmanr(np.abs(mu), phi).statistic) < 5.0 / math.sqrt(N)


def test_isotropic_direction_law():
    sc = _point_scene(False)
    N = 100_000
    _, k = _launch_records(sc, N, seed=8)
    assert stats.kstest(k[:, 2], stats.uniform(-1, 2).cdf).pvalue > P_MIN
    phi = np.arctan2(k[:, 1], k[:, 0])
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > P_MIN


@pytest.mark.parametrize("incl", [0.0, 60.0, 90.0, 120.0, 180.0])
def test_anisotropic_direct_image_exact(incl):
    """Transparent medium: the emission peel-off of the 2|mu| source is one
    pixel of N L0 2|cos i| / (4 pi d^2)."""
    sc = _point_scene(True, (incl,))
    N = 300
    img = oracle.run(sc, N, seed=0)["images"][0][0]
    expect = N * (1.0 / N) * 2.0 * abs(math.cos(math.radians(incl))) / (4 * math.pi * 100.0 ** 2)
    nz = np.argwhere(img != 0.0).tolist()
    if expect == 0.0:
        assert nz == []
    else:
        assert nz == [[4, 4]]
        assert img[4, 4] == pytest.approx(expect, rel=1e-13)


def test_anisotropic_source_phase_averages_to_one():
    """Gauss-Legendre quadrature over cos(i) of the direct-image values
    (separately on each half, where S is a polynomial): the sphere average of
    the source's angular distribution is 1, as for every normalised source."""
    nodes, w = np.polynomial.legendre.leggauss(6)
    mus = np.concatenate([0.5 * (nodes - 1.0), 0.5 * (nodes + 1.0)])
    ws = np.concatenate([0.5 * w, 0.5 * w])
    incl = np.degrees(np.arccos(mus))
    sc = _point_scene(True, incl)
    N = 50
    imgs = oracle.run(sc, N, seed=1)["images"]
    S = np.array([im[0].sum() for im in imgs]) * (4 * math.pi * 100.0 ** 2)
    assert np.allclose(S, 2.0 * np.abs(mus), rtol=1e-12, atol=1e-15)
    # (1/4pi) int S dOmega = (1/2) int S dmu
    assert 0.5 * float(np.dot(ws, S)) == pytest.approx(1.0, rel=1e-12)
