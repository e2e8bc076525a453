"""GPU parity of the learned direction proposal, through the C-ABI.

* Network on the matrix cores vs the FP64 oracle network (bf16 weights,
  inputs and hidden activations in both): FP32 summation order only, plus the
  rare hidden activation that rounds to the neighbouring bf16 value.
* Gradient of the weighted likelihood (MFMA forward and backward with bf16
  high + low gradient parts) vs the oracle's hand-written FP64 backward.
* FP64 validation transport with the proposal (scalar FP64 network): per
  cell and pixel within 1e-9 of the oracle, identical counters.
* Plain-run histories in FP64: records and packet totals as the oracle's;
  the training samples as the oracle's records compacted.
* FP32 transport with the proposal (MFMA network): same expectation as the
  plain estimator (4 sigma); training lowers the loss.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import learned as L
from paper_1705_04702_amd import mcrt, scenes

from test_gpu_parity import assert_fp64_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = mcrt.Context(0)
    yield c
    c.close()


def _features(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 9)).astype(np.float32)
    X[:, 8] = rng.integers(0, 2, n)
    kp = rng.normal(size=(n, 3))
    kp = (kp / np.linalg.norm(kp, axis=1, keepdims=True)).astype(np.float32)
    C = rng.exponential(size=n).astype(np.float32)
    return X, kp, C


def _params(seed, scale=1.0, bias=0.05):
    th = scenes.init_mlp(seed, scale=scale).astype(np.float64)
    p = L.unpack(th)
    rng = np.random.default_rng(seed + 100)
    for b in ("b1", "b2", "b3"):
        p[b] = rng.normal(scale=bias, size=p[b].shape)
    return L.pack(p).astype(np.float32)


@pytest.mark.parametrize("n", [1, 16, 1000, 4099])
def test_mfma_forward_matches_oracle(ctx, n):
    theta = _params(3, scale=1.5)
    X, _, _ = _features(n, 5)
    prop = mcrt.Proposal(ctx, params=theta)
    say(f"forward n={n}")
    got = prop.forward(X).astype(np.float64)
    ref = L.forward(L.round_weights(theta.astype(np.float64)), X.astype(np.float64))
    err = np.abs(got - ref)
    scale = np.abs(ref).max()
    say(f"forward n={n}: max abs err {err.max():.3e}, median {np.median(err):.3e}, scale {scale:.3e}")
    assert np.median(err) <= 1e-5 * scale
    assert err.max() <= 5e-3 * scale
    assert (err > 1e-4 * scale).mean() <= 0.01
    prop.close()


def test_params_roundtrip_and_bf16_weights(ctx):
    theta = _params(4)
    prop = mcrt.Proposal(ctx, params=theta)
    np.testing.assert_array_equal(prop.params(), theta)
    w = prop.weights_bf16()
    want = (L.bf16(theta.astype(np.float64)).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    np.testing.assert_array_equal(w, want)
    prop.close()


@pytest.mark.parametrize("n", [64, 333, 5000])
def test_gradient_matches_oracle(ctx, n):
    theta = _params(7, scale=1.0)
    X, kp, C = _features(n, 11)
    prop = mcrt.Proposal(ctx, params=theta)
    say(f"grad n={n}")
    loss, g = prop.grad(X, kp, C)
    th64 = L.round_weights(theta.astype(np.float64))
    lref, gref = L.loss_and_grad(th64, X.astype(np.float64), kp.astype(np.float64), C.astype(np.float64))
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say(f"grad n={n}: loss {loss:.6f} vs {lref:.6f}, rel-norm err {rel:.3e}")
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    assert rel <= 2e-3
    # every block of the parameter vector, not just the dominant one
    off = 0
    for name, shape in L.SHAPES:
        k = int(np.prod(shape))
        a, b = g[off:off + k], gref[off:off + k]
        assert np.linalg.norm(a - b) <= 5e-3 * np.linalg.norm(b) + 1e-7, name
        off += k
    prop.close()


LEARNED = {
    "torus": (lambda: scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0), 400),
    "sphere": (lambda: scenes.sphere(n=12, tau=2.0, albedo=0.7, npix=24), 800),
    "disk": (lambda: scenes.disk((16, 16, 8), 3, 24), 300),
}


def _run(ctx, sc, N, precision, seed, theta=None, **kw):
    sim = mcrt.Sim(ctx, sc, precision)
    prop = None
    if theta is not None:
        prop = mcrt.Proposal(ctx, params=theta)
        sim.set_proposal(prop, 0.2)
    res = sim.run(N, seed=seed, **kw)
    out = {"table": res.table(), "images": res.images(), "energy": res.energy(), "stats": res.stats()}
    sim.close()
    if prop is not None:
        prop.close()
    return out


@pytest.mark.parametrize("name", list(LEARNED))
def test_learned_transport_fp64_parity(ctx, name):
    make, N = LEARNED[name]
    sc = make()
    theta = _params(11, scale=1.5, bias=0.1)
    say(f"learned fp64 {name} N={N}")
    g = _run(ctx, sc, N, mcrt.FP64_VALIDATE, 9, theta)
    o = oracle.run(sc, N, seed=9, mlp=theta)
    assert_fp64_parity(g, o)


def test_learned_full_size_torus_fp64(ctx):
    """The learned proposal on the full clumpy torus (2.24e6 leaves to depth
    9, 1024^2 edge-on instrument, anisotropic source): FP64 validation per
    cell and pixel on 3 of the 32 wavelengths for a packet-id range inside
    the full run's 3.125e6 ids per wavelength."""
    sc = scenes.torus()
    sub = type(sc)(**{**sc.__dict__})
    keep = [0, 15, 31]
    for f in ("lambdas", "kappa", "albedo", "hg_g", "lum"):
        setattr(sub, f, np.ascontiguousarray(getattr(sc, f)[keep]))
    sub.name = "torus_full_3l"
    N, first, count = 3_125_000, 1_234_567, 400
    theta = _params(11, scale=1.5, bias=0.1)
    say(f"learned fp64 full torus ids [{first}, +{count}) x 3 wavelengths")
    g = _run(ctx, sub, N, mcrt.FP64_VALIDATE, 4, theta, first_id=first, count=count)
    o = oracle.run(sub, N, seed=4, first_id=first, count=count, mlp=theta)
    assert g["stats"]["packets"] == 3 * count
    assert_fp64_parity(g, o)


@pytest.mark.parametrize("name", ["torus", "disk"])
def test_histories_fp64_match_oracle(ctx, name):
    make, N = LEARNED[name]
    sc = make()
    E = 10
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    res = sim.new_result()
    say(f"histories fp64 {name} N={N}")
    h = sim.collect(res, N, seed=5, max_events=E, first_id=7, count=N - 20)
    rec, tot = h.records()
    X, KP, C = h.samples()
    table = res.table()
    h.close()
    sim.close()
    o = oracle.run(sc, N, seed=5, histories=E, first_id=7, count=N - 20)
    np.testing.assert_allclose(rec, o["hist"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(tot, o["hist_total"], rtol=1e-12, atol=0)
    assert np.array_equal(rec == 0, o["hist"] == 0)
    nz = o["table"] != 0
    assert np.max(np.abs(table[nz] - o["table"][nz]) / o["table"][nz]) <= 1e-9
    # training samples: recorded events with positive weight, in (packet, event) order
    hr, ht = o["hist"], o["hist_total"]
    Lr = hr[:, :, 12]
    with np.errstate(divide="ignore", invalid="ignore"):
        Cr = np.where(Lr > 0, (ht[:, None] - hr[:, :, 13]) / np.where(Lr > 0, Lr, 1.0), 0.0).astype(np.float32)
    keep = Cr > 0
    np.testing.assert_allclose(C, Cr[keep], rtol=1e-6, atol=0)  # flux sums to rounding
    np.testing.assert_array_equal(X, hr[:, :, :9][keep].astype(np.float32))
    np.testing.assert_array_equal(KP, hr[:, :, 9:12][keep].astype(np.float32))


@pytest.mark.parametrize("name", ["torus", "sphere"])
def test_learned_fp32_unbiased(ctx, name):
    make, _ = LEARNED[name]
    sc = make()
    N = 4000
    theta = _params(11, scale=1.5, bias=0.1)
    say(f"learned fp32 {name} N={N}")
    g = _run(ctx, sc, N, mcrt.FP32, 21, theta)
    # the plain estimator (other random numbers) in K independent batches: the
    # spread of the batch totals gives the standard deviation of the total
    K = 8
    parts = [oracle.run(sc, N, seed=4, first_id=k * (N // K), count=N // K) for k in range(K)]
    e = g["energy"]
    assert e[0] == pytest.approx(sum(p["energy"][0] for p in parts), rel=1e-6)
    assert abs(e[1] + e[2] + e[3] - e[0]) / e[0] < 0.05
    for name_, get in (("table", lambda r: r["table"].sum()), ("image", lambda r: r["images"][0].sum())):
        tot = np.array([get(p) for p in parts])
        sd_plain = math.sqrt(K * tot.var(ddof=1))
        # the learned run's own spread is not known here: allow three times the plain variance
        diff = get(g) - tot.sum()
        say(f"{name_}: learned {get(g):.6e} plain {tot.sum():.6e} sd {sd_plain:.2e}")
        assert abs(diff) <= 4 * math.sqrt(4.0) * sd_plain
    assert g["stats"]["packets"] == N * sc.n_lambda


def test_training_lowers_the_loss(ctx):
    sc = scenes.torus(5, 4, 3, 32, n_clumps=25, tau_eq=8.0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    res = sim.new_result()
    say("collect fp32 torus 20000/lambda")
    h = sim.collect(res, 20000, seed=1, max_events=16)
    assert h.n_samples > 1000
    prop = mcrt.Proposal(ctx, seed=3, init_scale=1.0)
    l0 = prop.eval(h)
    # the device loss over all samples equals the oracle's at the same parameters
    X, KP, C = h.samples()
    th = L.round_weights(prop.params().astype(np.float64))
    lref = L.loss_only(th, X.astype(np.float64), KP.astype(np.float64), C.astype(np.float64))
    say(f"loss before training {l0:.5f} (oracle {lref:.5f}), {h.n_samples} samples")
    assert abs(l0 - lref) <= 1e-4 * abs(lref)
    lf = prop.train(h, epochs=3, batch=4096, lr=3e-3, seed=2)
    l1 = prop.eval(h)
    say(f"loss after training {l1:.5f} (last batch {lf:.5f})")
    assert l1 < l0 - 0.05
    # training is deterministic: fixed minibatch draws, fixed-order gradient sums
    again = mcrt.Proposal(ctx, seed=3, init_scale=1.0)
    again.train(h, epochs=3, batch=4096, lr=3e-3, seed=2)
    np.testing.assert_array_equal(again.params(), prop.params())
    again.close()
    h.close()
    prop.close()
    sim.close()


@pytest.mark.parametrize("hp", [dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8),
                                dict(lr=1e-2, beta1=0.8, beta2=0.99, eps=1e-4)])
def test_adam_steps_match_fp64_reference(ctx, hp):
    """k Adam steps of mcrt_proposal_train against the FP64 Adam step.

    The histories hold exactly one training sample, so every minibatch of a
    step is that sample drawn batch times and the step's gradient is the
    sample's normalised gradient at the current parameters, which
    mcrt_proposal_grad gives for the same parameters.  Each training call
    makes one step; the Adam state persists across calls.  The FP64
    reference tracks m and v from those gradients and takes each step from
    the device's previous parameters."""
    sc = scenes.sphere(n=8, tau=1.0, albedo=0.5, g=0.5, npix=16)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    res = sim.new_result()
    say(f"adam steps {hp}")
    h = sim.collect(res, 1, seed=3, max_events=1)
    assert h.n_samples == 1
    X, KP, C = h.samples()
    theta0 = _params(5, scale=1.0, bias=0.05)
    prop = mcrt.Proposal(ctx, params=theta0)
    probe = mcrt.Proposal(ctx, params=theta0)
    m = np.zeros(L.N_PARAMS)
    v = np.zeros(L.N_PARAMS)
    prev = prop.params()
    lr = hp["lr"]
    for t in range(1, 6):
        probe.set_params(prev)
        _, g = probe.grad(X, KP, C)
        assert np.count_nonzero(g) > 1000
        prop.train(h, epochs=1, batch=64, seed=t, **hp)
        cur = prop.params()
        ref, m, v = L.adam_step(prev.astype(np.float64), m, v, g.astype(np.float64), t, **hp)
        # FP32 moments and update, FP32 parameters; the minibatch gradient
        # (64 copies of the sample, scaled by 1/64) differs from the single
        # sample's by the rounding of its bf16 high + low parts
        tol = 3e-5 * lr + 2.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        err = np.abs(cur - ref)
        step = np.abs(ref - prev)
        say(f"adam t={t}: max err {err.max():.3e} (tol min {tol.min():.1e}), step median "
            f"{np.median(step):.3e}")
        assert np.all(err <= tol)
        prev = cur
    probe.close()
    prop.close()
    h.close()
    sim.close()


def test_proposal_errors(ctx):
    a = mcrt.Sim(ctx, scenes.sphere(n=8), mcrt.FP32)
    prop = mcrt.Proposal(ctx, seed=1)
    try:
        with pytest.raises(mcrt.MCRTError) as ei:
            a.set_proposal(prop, 0.0)
        assert ei.value.code == mcrt.EINVAL
        a.set_proposal(prop, 0.2)
        r = a.new_result()
        with pytest.raises(mcrt.MCRTError) as ei:  # histories come from plain runs
            a.collect(r, 10, max_events=4)
        assert ei.value.code == mcrt.EINVAL
        with pytest.raises(mcrt.MCRTError) as ei:  # batched runs are plain
            mcrt.batch_run_into([a], [r], [10])
        assert ei.value.code == mcrt.EINVAL
        a.set_proposal(None)
        with pytest.raises(mcrt.MCRTError) as ei:
            a.collect(r, 10, max_events=0)
        assert ei.value.code == mcrt.EINVAL
        with pytest.raises(mcrt.MCRTError) as ei:
            prop.grad(np.zeros((4, 9)), np.tile([0, 0, 1.0], (4, 1)), np.zeros(4))
        assert ei.value.code == mcrt.EINVAL
    finally:
        prop.close()
        a.close()


def test_learned_event_cap_fp64(ctx):
    """The event cap with the learned proposal: the capped packet's weighted
    luminosity goes to truncated and the run reports ELIMIT, as in the oracle."""
    sc = scenes.sphere(n=12, tau=4.0, albedo=0.95, npix=16)
    sc.event_cap = 2
    N = 600
    theta = _params(5, scale=1.2)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    prop = mcrt.Proposal(ctx, params=theta)
    try:
        sim.set_proposal(prop, 0.2)
        res = sim.new_result()
        say("learned fp64 event cap 2")
        rc = sim.run_into(res, N, 3)
        assert rc == mcrt.ELIMIT
        g = {"table": res.table(), "images": res.images(), "energy": res.energy(), "stats": res.stats()}
        o = oracle.run(sc, N, seed=3, mlp=theta)
        assert g["stats"]["capped"] == o["stats"]["capped"] > 0
        assert_fp64_parity(g, o)
        res.close()
    finally:
        sim.close()
        prop.close()


def test_trained_proposal_reduces_image_variance(ctx):
    """What the trained network gains: on a small clumpy torus, after training
    on plain histories, the learned estimator's image has a smaller variance
    than the plain estimator's at the same number of packets.  The variances
    come from the spread of 8 independent runs of each (no reference image)."""
    sc = scenes.torus(6, 5, 4, 48, n_clumps=60, tau_eq=20.0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    prop = mcrt.Proposal(ctx, seed=5, init_scale=1.0)
    try:
        say("train on 40000/lambda plain histories")
        h = sim.collect(sim.new_result(), 40000, seed=1, max_events=16)
        prop.train(h, epochs=4, batch=8192, lr=2e-3, seed=1)
        h.close()
        K, n = 8, 8000
        var = {}
        for learned in (False, True):
            sim.set_proposal(prop if learned else None, 0.2)
            imgs = []
            for k in range(K):
                r = sim.new_result()
                sim.run_into(r, K * n, seed=11 + learned, first_id=k * n, count=n)
                imgs.append(r.image(0) * K)  # one batch as an estimate of the whole image
                r.close()
            imgs = np.array(imgs)
            var[learned] = imgs.var(axis=0, ddof=1).sum()
            say(f"{'learned' if learned else 'plain'}: image total {imgs.sum(axis=(1, 2, 3)).mean():.4e}, "
                f"summed pixel variance {var[learned]:.4e}")
        assert var[True] < 0.7 * var[False]
    finally:
        sim.set_proposal(None)
        prop.close()
        sim.close()
