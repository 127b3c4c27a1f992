"""Reference (FP64, numpy) for the surrogate and the two-stage unweighting.

The paper has no surrogate; this is the CPU counterpart of the learned part
of the path: a multilayer perceptron on phase-space invariants that predicts
log|M|^2, trained by mean-squared error with Adam, and the two-stage
unweighting that uses it (Danziger, Janssen, Schumann, Siegert, SciPost
Phys. 12 (2022) 164): stage 1 accepts on the surrogate weight, stage 2
corrects the accepted events with the exact matrix element.

Everything here is written from the textbook definitions, slowly:
  features   f_ij = log(2 p_i.p_j / s) for the particle pairs i < j
  layer      z = W h + b, h' = silu(z) = z / (1 + exp(-z))  (last layer linear)
  loss       L = mean_b (y_b - t_b)^2
  Adam       m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
             w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np


def features(mom):
    """log(2 p_i.p_j / s) for all pairs i < j; momenta [nevt][npar][4]."""
    mom = np.asarray(mom, dtype=np.float64)
    p = mom
    s = (p[:, 0, 0] + p[:, 1, 0]) ** 2 - ((p[:, 0, 1:] + p[:, 1, 1:]) ** 2).sum(axis=1)
    out = []
    n = p.shape[1]
    for i in range(n):
        for j in range(i + 1, n):
            d = p[:, i, 0] * p[:, j, 0] - (p[:, i, 1:] * p[:, j, 1:]).sum(axis=1)
            out.append(np.log(2.0 * d / s))
    return np.stack(out, axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def forward(params, x):
    """params = [(W, b), ...] with W [out][in]; returns (y, cache)."""
    h = x
    cache = []
    for li, (w, b) in enumerate(params):
        z = h @ w.T + b
        cache.append((h, z))
        h = silu(z) if li < len(params) - 1 else z
    return h[:, 0], cache


def loss_and_grads(params, x, t):
    """MSE loss and its gradients with respect to every W and b (backpropagation)."""
    y, cache = forward(params, x)
    nb = x.shape[0]
    loss = np.mean((y - t) ** 2)
    g = (2.0 / nb) * (y - t)[:, None]            # dL/dy
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        h, z = cache[li]
        if li < len(params) - 1:
            g = g * dsilu(z)                       # through the activation
        w, _ = params[li]
        grads[li] = (g.T @ h, g.sum(axis=0))
        g = g @ w
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = {'t': int, 'm': [...], 'v': [...]}."""
    state['t'] += 1
    t = state['t']
    for k, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        for which, (p, g) in enumerate(((w, gw), (b, gb))):
            key = 2 * k + which
            m = state['m'][key] = b1 * state['m'][key] + (1 - b1) * g
            v = state['v'][key] = b2 * state['v'][key] + (1 - b2) * g * g
            p -= lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)


def adam_state(params):
    z = []
    for w, b in params:
        z += [np.zeros_like(w), np.zeros_like(b)]
    return {'t': 0, 'm': [a.copy() for a in z], 'v': [a.copy() for a in z]}


def two_stage(w_hat, w_exact_fn, r1, r2, what_max, x_max):
    """Two-stage unweighting.

    Stage 1 accepts event i with probability min(1, w_hat_i / what_max); stage 2
    evaluates the exact weight w_i only for stage-1 events and accepts with
    probability min(1, x_i / x_max), x_i = w_i / w_hat_i.  Returns (accepted
    mask, residual weights max(1, w_hat/what_max) max(1, x/x_max) of accepted
    events, indices of the stage-1 events whose exact weight was needed).
    """
    s1 = r1 < np.minimum(1.0, w_hat / what_max)
    idx = np.nonzero(s1)[0]
    w = w_exact_fn(idx)
    x = w / w_hat[idx]
    s2 = r2[idx] < np.minimum(1.0, x / x_max)
    acc = np.zeros_like(s1)
    acc[idx[s2]] = True
    resid = (np.maximum(1.0, w_hat[idx[s2]] / what_max) * np.maximum(1.0, x[s2] / x_max))
    return acc, resid, idx


def one_stage(w, r, w_max):
    """Plain hit-or-miss unweighting on the exact weights."""
    acc = r < np.minimum(1.0, w / w_max)
    return acc, np.maximum(1.0, w[acc] / w_max)
