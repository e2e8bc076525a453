"""Pins of the learned-proposal oracle (oracle/learned.py).

* backward propagation vs central finite differences (FP64, smooth variant
  without activation rounding): relative error <= 1e-6;
* vMF: normalisation by quadrature, mean resultant length coth(k) - 1/k by
  sampling with the inverse-CDF cosine, tail behaviour;
* the proposal mixture integrates to 1 (quadrature over the sphere) and the
  weights p_phys/q have expectation 1 under q (sampling);
* bfloat16 rounding: nearest-even on exact halfway cases, idempotent;
* the FP64 Adam step: against torch.optim.Adam (an independent
  implementation, run on the CPU in float64) over several steps and
  hyperparameters, and against its closed forms (the first step and every
  step under a constant gradient move each parameter by lr g / (|g| + eps),
  because the bias correction makes both moment estimates exact there).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import learned as L


def _batch(n=48, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 9))
    kp = rng.normal(size=(n, 3))
    kp /= np.linalg.norm(kp, axis=1, keepdims=True)
    C = rng.exponential(size=n)
    return X, kp, C


def test_backward_matches_finite_differences():
    theta = L.init_params(1, scale=0.8)
    theta = theta + 0.01 * np.random.default_rng(2).normal(size=theta.size)  # non-zero biases
    X, kp, C = _batch()
    loss, g = L.loss_and_grad(theta, X, kp, C, round_act=False)
    assert loss == pytest.approx(L.loss_only(theta, X, kp, C, round_act=False), rel=1e-12)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(L.N_PARAMS, 300, replace=False),
                          np.arange(L.N_PARAMS - 40, L.N_PARAMS)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L.loss_only(tp, X, kp, C, round_act=False) - L.loss_only(tm, X, kp, C, round_act=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 2e-9, (i, fd, g[i])


def test_vmf_normalisation_and_mean_resultant():
    for kappa in (0.01, 0.5, 3.0, 40.0, 900.0):
        val, _ = integrate.quad(lambda w: 2 * math.pi * L.vmf_pdf(np.array([0, 0, w]),
                                                                   np.array([0, 0, 1.0]), kappa),
                                -1.0, 1.0, epsabs=1e-13, epsrel=1e-12, limit=200, points=[1 - 1 / kappa])
        assert val == pytest.approx(1.0, rel=1e-9)
        u = (np.arange(200000) + 0.5) / 200000
        w = L.sample_vmf_w(u, kappa)
        want = 1.0 / math.tanh(kappa) - 1.0 / kappa
        assert w.mean() == pytest.approx(want, rel=1e-4, abs=1e-6)


def _sphere_quadrature(fun, n_mu=400, n_phi=400):
    x, wx = np.polynomial.legendre.leggauss(n_mu)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    M, P = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - M * M)
    k = np.stack([st * np.cos(P), st * np.sin(P), M], -1).reshape(-1, 3)
    vals = fun(k).reshape(n_mu, n_phi)
    return (vals * wx[:, None]).sum() * (2 * math.pi / n_phi)


def test_mixture_integrates_to_one_and_weights_are_unbiased():
    theta = L.init_params(4)
    X, _, _ = _batch(3, seed=5)
    o = L.forward(theta, X)
    pi, mu, kappa = L.mixture_params(o)
    g = 0.6
    kin = np.array([0.3, -0.2, 0.93])
    kin /= np.linalg.norm(kin)
    for i in range(3):
        def q(k):
            n = k.shape[0]
            pphys = L.hg_pdf(g, k @ kin)
            return L.proposal_pdf(k, pphys, np.repeat(pi[i:i + 1], n, 0), np.repeat(mu[i:i + 1], n, 0),
                                  np.repeat(kappa[i:i + 1], n, 0))
        assert _sphere_quadrature(q) == pytest.approx(1.0, rel=1e-6)
        assert _sphere_quadrature(lambda k: L.hg_pdf(g, k @ kin)) == pytest.approx(1.0, rel=1e-6)
        # E_q[p/q] = 1: the integral of p over the sphere, evaluated through q
        ratio = _sphere_quadrature(lambda k: q(k) * (L.hg_pdf(g, k @ kin) / q(k)))
        assert ratio == pytest.approx(1.0, rel=1e-6)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 1e-30])
    got = L.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                     # halfway: to even (mantissa ...0)
    assert got[2] == 1.0 + 2 ** -7           # above halfway rounds up
    assert got[3] == 1.0 + 2 ** -6           # halfway between ..01 and ..10: to even
    assert got[4] == -2.5 and got[5] == 0.0
    assert np.array_equal(L.bf16(got), got)
    assert L.N_PARAMS == 7400


# --------------------------------------------------------------------------
# The learned proposal inside the C oracle's transport
# --------------------------------------------------------------------------

import oracle  # noqa: E402
from paper_1705_04702_amd import scenes  # noqa: E402


def test_c_and_numpy_networks_agree_bitwise():
    theta = L.round_weights(scenes.init_mlp(7).astype(np.float64))
    rng = np.random.default_rng(8)
    for _ in range(20):
        f = rng.normal(size=9)
        assert np.array_equal(oracle.mlp_forward(theta, f), L.forward(theta, f[None, :])[0])


def _small_torus():
    return scenes.torus(5, 4, 2, 32, n_clumps=25, tau_eq=8.0)


@pytest.mark.parametrize("make", [_small_torus, lambda: scenes.sphere(n=12, tau=2.0, albedo=0.7)])
def test_learned_transport_is_unbiased(make):
    """Weighted transport with an (untrained) proposal has the plain
    estimator's expectation: totals agree within 4 sigma."""
    sc = make()
    N = 3000
    theta = scenes.init_mlp(11)
    plain = oracle.run(sc, N, seed=4, moments=True)
    learn = oracle.run(sc, N, seed=5, mlp=theta, moments=True)
    for key in ("table",):
        a, b = plain[key], learn[key]
        va = np.maximum(plain[key + "_m2"] - a * a / N, 0).sum()
        vb = np.maximum(learn[key + "_m2"] - b * b / N, 0).sum()
        assert abs(a.sum() - b.sum()) < 4 * math.sqrt(va + vb)
    ia, ib = plain["images"][0], learn["images"][0]
    va = np.maximum(plain["image_m2"][0] - ia * ia / N, 0).sum()
    vb = np.maximum(learn["image_m2"][0] - ib * ib / N, 0).sum()
    assert abs(ia.sum() - ib.sum()) < 4 * math.sqrt(va + vb)
    e = learn["energy"]
    assert e[0] == pytest.approx(plain["energy"][0], rel=1e-12)
    assert abs(e[1] + e[2] + e[3] - e[0]) / e[0] < 0.05   # balance holds in expectation only


def test_histories_bookkeeping():
    sc = _small_torus()
    N, E = 200, 12
    r = oracle.run(sc, N, seed=2, histories=E)
    h, tot = r["hist"], r["hist_total"]
    assert h.shape == (N * sc.n_lambda, E, 14)
    L_e = h[:, :, 12]
    # emission always recorded, with the launch luminosity and event flag 0
    assert np.all(L_e[:, 0] == 1.0 / N)
    assert np.all(h[:, 0, 8] == 0.0) and np.all(h[:, 0, 3:6] == 0.0)
    # recorded scattering events carry flag 1 and unit directions
    rec = L_e > 0
    assert np.all(h[:, 1:, 8][rec[:, 1:]] == 1.0)
    nk = np.linalg.norm(h[:, :, 9:12], axis=2)
    assert np.allclose(nk[rec], 1.0, atol=1e-12)
    # cumulative flux never decreases and never exceeds the packet total
    cf = np.where(rec, h[:, :, 13], np.nan)
    d = np.diff(cf, axis=1)
    assert np.all(d[~np.isnan(d)] >= 0)
    assert np.all(cf[rec] <= np.repeat(tot[:, None], E, 1)[rec] * (1 + 1e-12))
    # the image holds exactly the recorded fluxes
    assert tot.sum() == pytest.approx(r["images"][0].sum(), rel=1e-12)
    # luminosity after an event shrinks by at most the albedo
    assert np.all(L_e[:, 1:][rec[:, 1:]] <= L_e[:, :-1][rec[:, 1:]] * (1 + 1e-12))


ADAM_CASES = [dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8),
              dict(lr=1e-2, beta1=0.8, beta2=0.99, eps=1e-3),
              dict(lr=3e-4, beta1=0.0, beta2=0.5, eps=1e-6)]


@pytest.mark.parametrize("hp", ADAM_CASES)
def test_adam_matches_torch(hp):
    import torch
    rng = np.random.default_rng(5)
    theta0 = rng.normal(size=257)
    grads = [rng.normal(size=257) * 10.0 ** rng.uniform(-4, 1, size=257) for _ in range(7)]
    grads[3][:20] = 0.0
    p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=hp["lr"], betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    th, m, v = theta0.copy(), np.zeros(257), np.zeros(257)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = L.adam_step(th, m, v, g, t, **hp)
        assert np.allclose(th, p.detach().numpy(), rtol=1e-14, atol=1e-16)
        st = opt.state[p]
        # the moments differ by rounding order only (torch interpolates)
        assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-15 * np.abs(m).max())
        assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-15 * np.abs(v).max())


@pytest.mark.parametrize("hp", ADAM_CASES)
def test_adam_closed_forms(hp):
    rng = np.random.default_rng(6)
    theta0 = rng.normal(size=64)
    g = rng.normal(size=64) * 10.0 ** rng.uniform(-3, 1, size=64)
    step = hp["lr"] * g / (np.abs(g) + hp["eps"])
    th, m, v = theta0, np.zeros(64), np.zeros(64)
    for t in range(1, 6):
        th, m, v = L.adam_step(th, m, v, g, t, **hp)
        assert np.allclose(th, theta0 - t * step, rtol=1e-12, atol=1e-15)
    # a zero gradient from a zero state leaves the parameters where they are
    th0, _, _ = L.adam_step(theta0, np.zeros(64), np.zeros(64), np.zeros(64), 1, **hp)
    assert np.array_equal(th0, theta0)
