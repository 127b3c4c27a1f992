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


def test_adam_three_steps_against_unrolled_sums():
    """Three Adam steps against the textbook moments written as explicit sums
    over the gradient history, m_t = (1-b1) sum_s b1^(t-s) g_s and likewise v_t
    with g^2, bias-corrected with the step count t = 1, 2, 3.

    Mutations caught: a step counter that never advances (bias correction of
    step 1 reused), moments that are overwritten instead of decayed, and b1/b2
    swapped between the two moments."""
    rng = np.random.default_rng(11)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 0.05
    params = _params(rng, [3, 2, 1])
    p0 = [(w.copy(), b.copy()) for w, b in params]
    hist = [[(rng.normal(size=w.shape), rng.normal(size=b.shape)) for w, b in params]
            for _ in range(3)]
    st = S.adam_state(params)
    expect = [[w.copy(), b.copy()] for w, b in p0]
    for t in (1, 2, 3):
        S.adam_step(params, hist[t - 1], st, lr=lr, b1=b1, b2=b2, eps=eps)
        for li in range(len(params)):
            for which in (0, 1):
                gs = [hist[s - 1][li][which] for s in range(1, t + 1)]
                m = (1 - b1) * sum(b1 ** (t - s) * g for s, g in zip(range(1, t + 1), gs))
                v = (1 - b2) * sum(b2 ** (t - s) * g * g for s, g in zip(range(1, t + 1), gs))
                mh = m / (1 - b1 ** t)
                vh = v / (1 - b2 ** t)
                expect[li][which] = expect[li][which] - lr * mh / (np.sqrt(vh) + eps)
        for (w, b), (ew, eb) in zip(params, expect):
            assert np.allclose(w, ew, rtol=1e-13, atol=1e-15)
            assert np.allclose(b, eb, rtol=1e-13, atol=1e-15)
    assert st['t'] == 3


def test_two_stage_overweights_with_quantile_maxima():
    """Two-stage unweighting with maxima below the largest weights (as the
    calibration quantiles do), on a toy where every probability is a multiple
    of 1/8 and each event meets the 8 x 8 grid of random numbers
    ((i + 1/2)/8, (j + 1/2)/8): event e is then accepted exactly
    64 p1(e) p2(e) times, p1 = min(1, w_hat/w_hat_max), p2 = min(1, x/x_max),
    x = w/w_hat.  Known exactly:
      * the number of accepted events,
      * the overweights (residual > 1): the accepts of the events with
        w_hat > w_hat_max or x > x_max,
      * the residual-weight sum, 64 sum_e w_e / (w_hat_max x_max): each accept
        carries max(1, w_hat/w_hat_max) max(1, x/x_max), so accept count times
        residual is 64 (w_hat/w_hat_max)(x/x_max) for every event (unbiased).

    Mutations caught: dropping either max(1, .) factor of the residual weight
    (the sum then falls short), using min instead of max, or forgetting to
    divide the exact weight by the surrogate weight in stage 2."""
    w_hat = np.array([1.0, 2.0, 3.0, 6.0, 2.0, 6.0])
    x = np.array([0.5, 1.0, 2.0, 3.0, 3.0, 0.5])
    w = w_hat * x
    what_max, x_max = 4.0, 2.0                  # below max(w_hat) = 6, max(x) = 3
    grid = (np.arange(8) + 0.5) / 8
    r1 = np.repeat(np.tile(grid, 8)[None, :], len(w), 0).reshape(-1)
    r2 = np.repeat(np.repeat(grid, 8)[None, :], len(w), 0).reshape(-1)
    ev = np.repeat(np.arange(len(w)), 64)
    acc, resid, idx = S.two_stage(w_hat[ev], lambda i: w[ev[i]], r1, r2, what_max, x_max)
    p1 = np.minimum(1, w_hat / what_max)
    p2 = np.minimum(1, x / x_max)
    n_acc = 64 * p1 * p2
    assert acc.sum() == int(round(n_acc.sum()))
    # stage 1 needs the exact weight only for its own accepts
    assert len(idx) == int(round(8 * (8 * p1).sum()))
    over = (w_hat > what_max) | (x > x_max)
    assert (resid > 1).sum() == int(round(n_acc[over].sum()))
    assert np.isclose(resid.sum(), 64 * w.sum() / (what_max * x_max), rtol=1e-14)
    # per event: every accepted copy carries the same residual
    for e in range(len(w)):
        r = resid[ev[acc] == e]
        assert np.allclose(r, max(1, w_hat[e] / what_max) * max(1, x[e] / x_max))


def test_one_stage_overweights_with_a_quantile_maximum():
    """One-stage unweighting with w_max below the largest weight (the calibration
    quantile of the baseline): on a toy where min(1, w/w_max) is a multiple of 1/8
    and each event meets the grid of 8 random numbers (i + 1/2)/8, event e is
    accepted exactly 8 min(1, w_e/w_max) times, each accept carrying
    max(1, w_e/w_max); the accepted residual weights then sum to 8 sum_e w_e/w_max
    (unbiased), and the overweights are the accepts of the events above w_max.

    Mutations caught: dropping the max(1, .) of the residual weight (the sum falls
    short by the overweights' excess), min instead of max, or accepting on
    w_max/w."""
    w = np.array([0.5, 1.0, 2.0, 3.0, 4.0, 6.0])
    w_max = 2.0
    grid = (np.arange(8) + 0.5) / 8
    ev = np.repeat(np.arange(len(w)), 8)
    acc, resid = S.one_stage(w[ev], np.tile(grid, len(w)), w_max)
    p = np.minimum(1.0, w / w_max)
    assert acc.sum() == int(round(8 * p.sum()))
    assert np.isclose(resid.sum(), 8 * w.sum() / w_max, rtol=1e-14)
    assert (resid > 1).sum() == int(round(8 * p[w > w_max].sum()))
    for e in range(len(w)):
        assert np.allclose(resid[ev[acc] == e], max(1.0, w[e] / w_max))
