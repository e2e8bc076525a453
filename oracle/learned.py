"""FP64 oracle of the learned direction proposal (test infrastructure only).

A small MLP maps the features of an emission or scattering event to an
8-lobe von Mises-Fisher (vMF) mixture over new directions; the proposal
mixes it with the physical distribution, q = alpha p_phys + (1 - alpha)
sum_j pi_j vMF_j, and the packet carries the weight W = p_phys / q so that
the estimator of the stellar emission phase (Section 3.2 of the hybrid-
parallel SKIRT paper) keeps its expectation.  Training maximises the
likelihood of the vMF part on plain-method events weighted by the flux the
packet still produced afterwards, so that the optimum is proportional to
p_phys times the expected future contribution.

Everything here is numpy FP64, written from the definitions; the weights
and the hidden activations are rounded to bfloat16 exactly where the device
stores them (features and hidden layers), the sums themselves are FP64.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID, N_OUT, N_LOBES = 9, 64, 40, 8
ALPHA = 0.2
KAPPA_MIN, KAPPA_MAX = 1e-3, 1e3

# flat parameter layout: W1 [9][64], b1 [64], W2 [64][64], b2 [64], W3 [64][40], b3 [40]
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to float32 (nearest even), then to bfloat16 (nearest even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_weights(theta):
    """Weights to bfloat16, biases unchanged."""
    p = unpack(theta)
    for name in ("W1", "W2", "W3"):
        p[name] = bf16(p[name])
    return pack(p)


def forward(theta, X, keep=False, round_act=True):
    """X [n, 9] -> outputs [n, 40].  theta must hold bf16-representable weights.
    Sums run over the inputs in order, then the bias is added.  With
    round_act=False the features and hidden activations stay FP64 (a smooth
    function of the parameters, for finite-difference checks)."""
    p = unpack(theta)
    rnd = bf16 if round_act else (lambda a: np.asarray(a, dtype=np.float64))
    x = rnd(X)
    z1 = _affine(x, p["W1"], p["b1"])
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = _affine(h1, p["W2"], p["b2"])
    h2 = rnd(np.maximum(z2, 0.0))
    o = _affine(h2, p["W3"], p["b3"])
    if keep:
        return o, (x, z1, h1, z2, h2)
    return o


def _affine(x, W, b):
    acc = np.zeros((x.shape[0], W.shape[1]))
    for k in range(W.shape[0]):
        acc = acc + x[:, k:k + 1] * W[k][None, :]
    return acc + b[None, :]


def softplus(x):
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def mixture_params(o):
    """o [n, 40] -> pi [n, 8], mu [n, 8, 3], kappa [n, 8]."""
    lg = o[:, :8]
    e = np.exp(lg - lg.max(axis=1, keepdims=True))
    pi = e / e.sum(axis=1, keepdims=True)
    m = o[:, 8:32].reshape(-1, 8, 3)
    nrm = np.sqrt((m * m).sum(axis=2, keepdims=True))
    mu = np.where(nrm > 0, m / np.where(nrm > 0, nrm, 1.0), np.array([0.0, 0.0, 1.0]))
    kappa = np.clip(softplus(o[:, 32:40]) + 1e-3, KAPPA_MIN, KAPPA_MAX)
    return pi, mu, kappa


def vmf_pdf(kp, mu, kappa):
    """Density on the unit sphere of vMF(mu, kappa) at directions kp."""
    dot = (mu * kp).sum(axis=-1)
    return kappa / (2.0 * math.pi * -np.expm1(-2.0 * kappa)) * np.exp(kappa * (dot - 1.0))


def vmf_mixture_pdf(kp, pi, mu, kappa):
    """kp [n, 3]; pi, kappa [n, 8]; mu [n, 8, 3]."""
    return (pi * vmf_pdf(kp[:, None, :], mu, kappa)).sum(axis=1)


def hg_pdf(g, cosang):
    """Henyey-Greenstein density on the sphere (phase / 4 pi)."""
    return (1.0 - g * g) / (1.0 + g * g - 2.0 * g * cosang) ** 1.5 / (4.0 * math.pi)


def proposal_pdf(kp, pphys, pi, mu, kappa, alpha=ALPHA):
    return alpha * pphys + (1.0 - alpha) * vmf_mixture_pdf(kp, pi, mu, kappa)


def sample_vmf_w(u, kappa):
    """Cosine to the mean direction: inverse CDF of p(w) ~ exp(kappa w)."""
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    return np.clip(w, -1.0, 1.0)


def loss_and_grad(theta, X, kp, C, round_act=True):
    """Weighted negative log-likelihood of the vMF mixture,
    -sum_e C_e log q_vMF(k'_e | f_e) / sum_e C_e, and its gradient with
    respect to the (bf16) weights and biases, by hand-written backward
    propagation in FP64 (the bf16-rounded activations are the ones used)."""
    p = unpack(theta)
    o, (x, z1, h1, z2, h2) = forward(theta, X, keep=True, round_act=round_act)
    n = X.shape[0]
    csum = C.sum()
    lg = o[:, :8]
    e = np.exp(lg - lg.max(axis=1, keepdims=True))
    pi = e / e.sum(axis=1, keepdims=True)
    m = o[:, 8:32].reshape(n, 8, 3)
    nrm = np.sqrt((m * m).sum(axis=2))
    mu = m / nrm[:, :, None]
    s = o[:, 32:40]
    sp = softplus(s) + 1e-3
    kappa = np.clip(sp, KAPPA_MIN, KAPPA_MAX)
    dk_ds = np.where((sp > KAPPA_MIN) & (sp < KAPPA_MAX), 1.0 / (1.0 + np.exp(-s)), 0.0)
    f = vmf_pdf(kp[:, None, :], mu, kappa)                    # [n, 8]
    q = (pi * f).sum(axis=1)
    loss = -(C * np.log(q)).sum() / csum
    r = pi * f / q[:, None]                                    # responsibilities
    dot = (mu * kp[:, None, :]).sum(axis=2)
    # d log q / d outputs
    d_logit = r - pi
    g_mu = (r * kappa)[:, :, None] * (kp[:, None, :] - dot[:, :, None] * mu) / nrm[:, :, None]
    e2 = np.exp(-2.0 * kappa)
    dlogf_dk = 1.0 / kappa - 2.0 * e2 / (-np.expm1(-2.0 * kappa)) + (dot - 1.0)
    d_s = r * dlogf_dk * dk_ds
    dlogq = np.concatenate([d_logit, g_mu.reshape(n, 24), d_s], axis=1)
    dO = -(C / csum)[:, None] * dlogq                           # [n, 40]
    grads = {}
    grads["W3"] = h2.T @ dO
    grads["b3"] = dO.sum(axis=0)
    dh2 = dO @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    grads["W2"] = h1.T @ dz2
    grads["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    grads["W1"] = x.T @ dz1
    grads["b1"] = dz1.sum(axis=0)
    return loss, pack(grads)


def loss_only(theta, X, kp, C, round_act=True):
    o = forward(theta, X, round_act=round_act)
    pi, mu, kappa = mixture_params(o)
    q = vmf_mixture_pdf(kp, pi, mu, kappa)
    return -(C * np.log(q)).sum() / C.sum()


def init_params(seed=0, scale=1.0):
    """Uniform fan-in initialisation (seeded), weights already bf16."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = scale * math.sqrt(6.0 / shape[0])
            p[name] = bf16(rng.uniform(-bound, bound, shape))
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def adam_step(theta, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, ICLR 2015, Algorithm 1) in FP64.

    The moment estimates are exponential averages of the gradient and of its
    square; dividing them by 1 - beta^t removes the bias of their zero start;
    the parameters move by lr times the corrected first moment over the
    square root of the corrected second moment plus eps.  t >= 1 is the step
    number.  Returns the new (theta, m, v).
    """
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    theta = np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v
