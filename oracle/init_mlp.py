"""CPU FP64 oracle of the learned particle proposal -- TEST INFRASTRUCTURE ONLY.

Plain numpy, written from the definitions (not from the HIP code): the
feature summary of a sequence step, the 64-256-256-120 ReLU network, the
8-component diagonal Gaussian mixture it outputs, the mixture negative
log-likelihood of a particle set and the gradients of both (hand-derived
backpropagation), and the Adam update that trains the network.  The paper
gives no initialisation of the particles of a new step (Algorithm 2 starts
SVGD from them without saying how they are drawn); this proposal is an
addition whose arithmetic is fixed here.

``bf16=True`` rounds what the GPU kernels feed to their BF16 products (the
input features, the weights, the hidden activations and the back-propagated
gradients) to bfloat16 with round-to-nearest-even; everything else stays
FP64.  Pins (tests/test_oracle_init.py): backward against central finite
differences of forward, the NLL gradient against finite differences of the
NLL, the one-component one-dimensional NLL against scipy's normal log-pdf,
features of a set of identical particles in closed form, the mixture
moments against a hand-solved two-component mixture (law of total variance),
Adam against a hand-worked two-step example and its closed-form first step.
"""
from __future__ import annotations

import numpy as np

from . import grad_loglik, loglik, transition_mean

FEAT, HID, K, COMP = 64, 256, 8, 15
OUT = K * COMP
RHO_MIN, RHO_MAX = -7.0, 3.0

# flattened parameter layout
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * FEAT
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + OUT * HID
N_PARAMS = OFF_B3 + OUT


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    W1 = P[OFF_W1:OFF_B1].reshape(HID, FEAT)
    b1 = P[OFF_B1:OFF_W2]
    W2 = P[OFF_W2:OFF_B2].reshape(HID, HID)
    b2 = P[OFF_B2:OFF_W3]
    W3 = P[OFF_W3:OFF_B3].reshape(OUT, HID)
    b3 = P[OFF_B3:N_PARAMS]
    return W1, b1, W2, b2, W3, b3


def features(desc, t, x_prev, phi_prev, z, mask, n):
    """(F [64], anchor a [8], scale s [8]) of the step-t proposal.

    best = lowest index of max phi_prev; a = f_t(x_prev[best]); M_j =
    f_t(x_prev[j]); population mean and variance of M over j; g and ll the
    observation log-likelihood gradient and value at a.  No feature holds
    the absolute position (only offsets from a, spreads and the likelihood
    around a), so the proposal, placed relative to a, does not depend on
    how far a sequence has moved."""
    d = desc.d
    x_prev = np.asarray(x_prev, dtype=np.float64).reshape(-1, d)
    phi = np.asarray(phi_prev, dtype=np.float64)
    best = int(np.argmax(phi))            # first maximum
    a = transition_mean(desc, t, x_prev[best])
    M = np.stack([transition_mean(desc, t, xj) for xj in x_prev])
    mu = M.mean(axis=0)
    var = ((M - mu) ** 2).mean(axis=0)
    s = np.sqrt(np.asarray(desc.q_var[:d], dtype=np.float64))
    g = grad_loglik(desc, z, mask, a)
    ll = loglik(desc, z, mask, a)
    F = np.zeros(FEAT)
    F[int(desc.kind)] = 1.0
    F[4] = np.log(n) / 7.0
    F[5:5 + d] = (mu - a) / s
    F[12:12 + d] = np.log(var / s ** 2 + 1e-6) / 8.0
    F[19:19 + d] = np.arcsinh(s * g) / 4.0
    F[26] = np.arcsinh(ll) / 8.0
    av = np.zeros(8)
    sv = np.ones(8)
    av[:d] = a
    sv[:d] = s
    return F, av, sv


def forward(P, F, bf16=True):
    """Outputs [B, 120] for features F [B, 64], and the cache for backward."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    X = r(np.atleast_2d(F))
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    pre1 = X @ W1r.T + b1
    h1 = r(np.maximum(pre1, 0.0))
    pre2 = h1 @ W2r.T + b2
    h2 = r(np.maximum(pre2, 0.0))
    out = h2 @ W3r.T + b3
    return out, (X, pre1, h1, pre2, h2, W1r, W2r, W3r)


def backward(cache, dout, bf16=True):
    """Gradient [N_PARAMS] of sum(dout * out) with respect to the parameters."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    X, pre1, h1, pre2, h2, W1r, W2r, W3r = cache
    dout = np.atleast_2d(np.asarray(dout, dtype=np.float64))
    do = r(dout)
    G = np.zeros(N_PARAMS)
    G[OFF_W3:OFF_B3] = (do.T @ h2).ravel()
    G[OFF_B3:N_PARAMS] = dout.sum(axis=0)
    d2 = (do @ W3r) * (pre2 > 0)
    d2r = r(d2)
    G[OFF_W2:OFF_B2] = (d2r.T @ h1).ravel()
    G[OFF_B2:OFF_W3] = d2.sum(axis=0)
    d1 = (d2r @ W2r) * (pre1 > 0)
    d1r = r(d1)
    G[OFF_W1:OFF_B1] = (d1r.T @ X).ravel()
    G[OFF_B1:OFF_W2] = d1.sum(axis=0)
    return G


def mixture(out, a, s, d):
    """(log pi [8], means [8, d], standard deviations [8, d], in-clamp mask)."""
    o = np.asarray(out, dtype=np.float64).reshape(K, COMP)
    logits = o[:, 0]
    lp = logits - (logits.max() + np.log(np.exp(logits - logits.max()).sum()))
    rho = o[:, 8:8 + d]
    rin = (rho >= RHO_MIN) & (rho <= RHO_MAX)
    rc = np.clip(rho, RHO_MIN, RHO_MAX)
    mean = a[:d] + s[:d] * o[:, 1:1 + d]
    sd = s[:d] * np.exp(rc)
    return lp, mean, sd, rin


def mixture_nll(out, a, s, X):
    """Mean over the rows of X [n, d] of -log sum_c pi_c N(x; mean_c, diag sd_c^2),
    and its gradient [120] with respect to the outputs."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    n, d = X.shape
    lp, mean, sd, rin = mixture(out, a, s, d)
    pc = np.exp(lp)
    u = (X[:, None, :] - mean[None, :, :]) / sd[None, :, :]              # [n, K, d]
    lc = lp[None, :] + (-0.5 * u ** 2 - np.log(sd)[None] - 0.5 * np.log(2 * np.pi)).sum(axis=2)
    m = lc.max(axis=1, keepdims=True)
    lse = (m + np.log(np.exp(lc - m).sum(axis=1, keepdims=True)))[:, 0]
    loss = -lse.mean()
    resp = np.exp(lc - lse[:, None])                                      # [n, K]
    g = np.zeros((K, COMP))
    g[:, 0] = -(resp - pc[None, :]).sum(axis=0)
    g[:, 1:1 + d] = -(resp[:, :, None] * u / sd[None] * s[None, None, :d]).sum(axis=0)
    g[:, 8:8 + d] = -(resp[:, :, None] * (u ** 2 - 1.0)).sum(axis=0) * rin
    return loss, g.ravel() / n


def mixture_moments(out, a, s, d):
    """Mean [d] and variance [d] of the proposal (per dimension)."""
    lp, mean, sd, _ = mixture(out, a, s, d)
    p = np.exp(lp)[:, None]
    m = (p * mean).sum(axis=0)
    v = (p * (sd ** 2 + mean ** 2)).sum(axis=0) - m ** 2
    return m, v


def adam_step(P, G, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015, Algorithm 1) at step t >= 1:
    first and second moment estimates m <- b1 m + (1 - b1) g and
    v <- b2 v + (1 - b2) g^2, their bias-corrected values m / (1 - b1^t) and
    v / (1 - b2^t), and P <- P - lr m_hat / (sqrt(v_hat) + eps), with eps
    added outside the square root.  Returns (P, m, v) as new arrays."""
    P = np.asarray(P, dtype=np.float64)
    g = np.asarray(G, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return P - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
