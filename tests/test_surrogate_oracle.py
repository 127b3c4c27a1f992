"""Pins of the CPU surrogate reference: features, backpropagation, Adam and
the two-stage unweighting, each against a definition it does not reuse."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_2510_05392_amd import rambo


def _params(rng, sizes):
    return [(rng.normal(size=(o, i)) / np.sqrt(i), rng.normal(size=o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_features_are_pair_invariants():
    mom = rambo.generate(6, 5, 3)
    f = S.features(mom)
    assert f.shape == (5, 15)
    # pair (0,1): 2 p1.p2 = s exactly, so its feature is log 1 = 0
    assert np.allclose(f[:, 0], 0.0, atol=1e-14)
    # Lorentz invariance under a boost along x
    b = 0.4
    g = 1 / np.sqrt(1 - b * b)
    bm = mom.copy()
    bm[..., 0] = g * (mom[..., 0] + b * mom[..., 1])
    bm[..., 1] = g * (mom[..., 1] + b * mom[..., 0])
    assert np.allclose(S.features(bm), f, atol=1e-11)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = _params(rng, [15, 7, 5, 1])
    x = rng.normal(size=(9, 15))
    t = rng.normal(size=9)
    loss, grads = S.loss_and_grads(params, x, t)
    h = 1e-6
    for li, (w, b) in enumerate(params):
        for arr, g in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[k]
                flat[k] = old + h
                lp, _ = S.loss_and_grads(params, x, t)
                flat[k] = old - h
                lm, _ = S.loss_and_grads(params, x, t)
                flat[k] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[k]) <= 1e-6 * max(1.0, abs(fd))


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (S.silu(z + h) - S.silu(z - h)) / (2 * h)
    assert np.allclose(S.dsilu(z), fd, atol=1e-8)


def test_adam_first_step_is_signed_learning_rate():
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps)
    rng = np.random.default_rng(1)
    params = _params(rng, [4, 3, 1])
    before = [(w.copy(), b.copy()) for w, b in params]
    grads = [(rng.normal(size=w.shape), rng.normal(size=b.shape)) for w, b in params]
    st = S.adam_state(params)
    S.adam_step(params, grads, st, lr=0.01)
    for (w0, b0), (w1, b1), (gw, gb) in zip(before, params, grads):
        assert np.allclose(w0 - w1, 0.01 * gw / (np.abs(gw) + 1e-8))
        assert np.allclose(b0 - b1, 0.01 * gb / (np.abs(gb) + 1e-8))


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(2)
    params = _params(rng, [3, 16, 16, 1])
    x = rng.normal(size=(256, 3))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    st = S.adam_state(params)
    l0, _ = S.loss_and_grads(params, x, t)
    for _ in range(300):
        _, g = S.loss_and_grads(params, x, t)
        S.adam_step(params, g, st, lr=0.01)
    l1, _ = S.loss_and_grads(params, x, t)
    assert l1 < 0.1 * l0


def test_two_stage_unweighting_is_unbiased():
    # toy weights w(x) on x ~ U(0,1); an imperfect surrogate w_hat.  The
    # accepted events, weighted by their residual weights, reproduce the
    # w-weighted distribution of x (chi^2 within statistics).
    rng = np.random.default_rng(3)
    n = 400000
    x = rng.random(n)
    w = 1.0 + 4.0 * x ** 3
    w_hat = 1.0 + 3.0 * x ** 2                      # wrong shape on purpose
    acc, resid, idx = S.two_stage(w_hat, lambda i: w[i], rng.random(n), rng.random(n),
                                  what_max=w_hat.max(), x_max=(w / w_hat).max())
    edges = np.linspace(0, 1, 11)
    expect = np.histogram(x, edges, weights=w)[0]
    expect = expect / expect.sum()
    got = np.histogram(x[acc], edges, weights=resid)[0]
    ntot = got.sum()
    chi2 = (((got / ntot - expect) ** 2) / (expect / ntot)).sum()
    assert chi2 < 30                                  # 10 bins
    assert len(idx) < n                               # the exact weight is not needed everywhere
    # the one-stage method on the exact weights agrees
    acc1, res1 = S.one_stage(w, rng.random(n), w.max())
    got1 = np.histogram(x[acc1], edges, weights=res1)[0]
    chi2b = (((got1 / got1.sum() - expect) ** 2) / (expect / got1.sum())).sum()
    assert chi2b < 30
