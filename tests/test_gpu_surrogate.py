"""Surrogate kernels on the GPU vs the FP64 CPU reference, and what the
trained network gains in two-stage unweighting.

Tolerances: the GPU keeps weights and activations in BF16 (8 significant
bits, unit roundoff 2^-8) with FP32 accumulation; gradients through a few
layers therefore agree with the FP64 reference (fed the same BF16-rounded
weights and inputs) to a few times 2^-8 in norm and direction.
"""
import numpy as np
import pytest

from oracle import me as ome, surrogate as S
from paper_2510_05392_amd import rambo

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

AS = 0.118


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2510_05392_amd import binding as b
    b.load()
    return b


def _bf16(x):
    return torch.from_numpy(np.asarray(x, dtype=np.float32)).bfloat16().float().numpy().astype(np.float64)


def _unflatten(flat, sizes):
    out, off = [], 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        w = flat[off:off + o * i].reshape(o, i)
        off += o * i
        b = flat[off:off + o]
        off += o
        out.append((w.astype(np.float64), b.astype(np.float64)))
    return out


def test_surrogate_forward_and_gradients_vs_cpu(binding):
    _say('case surrogate gradients vs cpu (15-64-64-1, 300 rows)')
    nfeat, width, depth, nb = 15, 64, 2, 300
    sur = binding.Surrogate(nfeat, width, depth, seed=7)
    sizes = [nfeat] + [width] * depth + [1]
    params = _unflatten(sur.me_sur_get_params(), sizes)
    mom = rambo.generate(6, nb, 5)
    raw = S.features(mom)
    # the (g1, g2) invariant is 2 p1.p2 / s = 1 for every event: a constant feature
    mean, std = raw.mean(axis=0), np.maximum(raw.std(axis=0), 1e-6)
    sur.me_sur_set_normalisation(mean.astype(np.float32), (1 / std).astype(np.float32))
    dmom = torch.from_numpy(mom).cuda()
    feat = torch.empty((nb, sur.kpad), dtype=torch.int16, device='cuda')
    sur.me_sur_features(dmom, nb, 6, feat)
    rng = np.random.default_rng(1)
    target = rng.normal(size=nb).astype(np.float32)
    y = torch.empty(nb, dtype=torch.float32, device='cuda')
    sur.me_sur_predict(feat, nb, y)
    tg = torch.from_numpy(target).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device='cuda')
    sur.me_sur_grads(feat, tg, nb, loss)
    torch.cuda.synchronize()
    # the GPU features (BF16) against the FP64 ones, except the constant (g1, g2)
    # column whose normalised value is rounding noise amplified by 1 / std
    xg = feat.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)[:, :nfeat]
    xc = (raw - mean) / std
    assert np.all(np.abs(xg[:, 1:] - xc[:, 1:]) <= 2.0 ** -7 * np.abs(xc[:, 1:]) + 1e-3)
    # CPU FP64 reference of the network on the same BF16 inputs and weights
    x = xg
    pb = [(_bf16(w), b) for w, b in params]
    yref, _ = S.forward(pb, x)
    ygpu = y.cpu().numpy()
    assert np.max(np.abs(ygpu - yref)) < 0.05 * max(1.0, np.abs(yref).max())
    lref, gref = S.loss_and_grads(pb, x, target)
    assert abs(float(loss.item()) / nb - lref) < 0.03 * lref
    ggpu = _unflatten(sur.me_sur_get_grads(), sizes)
    for (gw, gb), (rw, rb) in zip(ggpu, gref):
        for a, b in ((gw, rw), (gb, rb)):
            cos = float((a * b).sum() / (np.linalg.norm(a) * np.linalg.norm(b)))
            assert cos > 0.995, cos
            assert abs(np.linalg.norm(a) / np.linalg.norm(b) - 1) < 0.05


def test_adam_step_matches_reference(binding):
    _say('case adam step')
    nfeat, width, depth = 15, 32, 1
    sur = binding.Surrogate(nfeat, width, depth, seed=3)
    sizes = [nfeat, width, 1]
    before = sur.me_sur_get_params().astype(np.float64)
    mom = rambo.generate(6, 128, 9)
    dmom = torch.from_numpy(mom).cuda()
    feat = torch.empty((128, sur.kpad), dtype=torch.int16, device='cuda')
    sur.me_sur_features(dmom, 128, 6, feat)
    tg = torch.zeros(128, dtype=torch.float32, device='cuda') + 0.5
    sur.me_sur_grads(feat, tg, 128)
    g = sur.me_sur_get_grads().astype(np.float64)
    sur.me_sur_adam(1e-3)
    after = sur.me_sur_get_params().astype(np.float64)
    # first step: w -= lr * g / (|g| + eps)
    expect = before - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(after, expect, rtol=0, atol=2e-6)


@pytest.fixture(scope='module')
def trained(binding):
    from paper_2510_05392_amd.surrogate import SurrogatePipeline
    _say('case train surrogate gg_ttxgg (131072 events, 12 epochs)')
    pipe = SurrogatePipeline('gg_ttxgg', width=256, depth=4, seed=11)
    mom = torch.from_numpy(rambo.generate(6, 131072, 2001)).cuda()
    hist = pipe.fit(mom, epochs=12, batch=4096, lr=2e-3, lr_final=1e-4, log=_say)
    return pipe, hist


def test_training_reduces_loss_and_predicts(trained):
    pipe, hist = trained
    assert hist[-1] < 0.25 * hist[0]
    val = torch.from_numpy(rambo.generate(6, 32768, 2003)).cuda()
    err = pipe.log_error(val)
    rms = float(np.sqrt(np.mean(err ** 2)))
    _say(f'  validation RMS log-error {rms:.3f} (target spread {pipe.ystd:.3f})')
    assert rms < 0.5 * pipe.ystd


def test_unweighting_kernels_match_cpu_reference(trained, binding):
    _say('case unweighting kernels vs cpu reference')
    pipe = trained[0]
    n = 4000
    mom, wps = rambo.generate(6, n, 2004, return_weights=True)
    dmom = torch.from_numpy(mom).cuda()
    dw = torch.from_numpy(wps).cuda()
    rng = np.random.default_rng(5)
    r1, r2 = rng.random(n), rng.random(n)
    what_max, x_max = pipe.calibrate(dmom, dw)
    res = pipe.unweight(dmom, dw, torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda(), what_max, x_max)
    # the same decisions from the CPU reference given the network output
    y = pipe.predict(dmom).double().cpu().numpy()
    w_hat = np.exp(y * pipe.ystd + pipe.ymean) * wps
    exact = ome.matrix_element(ome.process(6), mom, AS) * wps
    acc, resid, idx = S.two_stage(w_hat, lambda i: exact[i], r1, r2, what_max, x_max)
    assert res['stage1'] == len(idx)
    got = res['index'].cpu().numpy()
    assert np.array_equal(np.sort(got), np.nonzero(acc)[0])
    assert np.allclose(res['resid'].cpu().numpy(), resid, rtol=1e-9)


def test_surrogate_gain_and_unbiasedness(trained, binding):
    # the trained network lets stage 1 discard most events without their exact
    # matrix element, while the accepted sample reproduces the exact-weighted
    # distribution of an observable (chi^2 against the one-stage method)
    _say('case surrogate gain (262144 events)')
    pipe = trained[0]
    n = 262144
    mom, wps = rambo.generate(6, n, 2002, return_weights=True)
    dmom = torch.from_numpy(mom).cuda()
    dw = torch.from_numpy(wps).cuda()
    cal = torch.from_numpy(rambo.generate(6, 65536, 2005)).cuda()
    cw = torch.from_numpy(rambo.generate(6, 65536, 2005, return_weights=True)[1]).cuda()
    # flat phase space without cuts gives heavy-tailed weights: the maxima are
    # taken as high quantiles of a calibration sample, and events above them keep
    # residual weights > 1 (overweights), which keeps the sample unbiased
    what_max, x_max = pipe.calibrate(cal, cw, quantile=0.99)
    g = torch.Generator(device='cuda').manual_seed(9)
    r1 = torch.rand(n, dtype=torch.float64, device='cuda', generator=g)
    r2 = torch.rand(n, dtype=torch.float64, device='cuda', generator=g)
    two = pipe.unweight(dmom, dw, r1, r2, what_max, x_max)
    w_exact = pipe.exact(dmom) * dw
    w_cal = pipe.exact(cal) * cw
    one = pipe.unweight_exact(dmom, dw, r2, float(torch.quantile(w_cal, 0.99)))
    saved = 1 - two['stage1'] / n
    _say(f"  stage-1 events {two['stage1']} of {n} (exact calls saved {saved:.1%}); accepted two-stage "
         f"{two['accepted']}, one-stage {one['accepted']}; overweights {two['overweight']}")
    assert saved > 0.5
    assert two['accepted'] > 0.3 * one['accepted']
    # observable: rapidity-like log(E_t + pz_t) / (E_t - pz_t) of the top, 8 bins
    obs = 0.5 * np.log((mom[:, 2, 0] + mom[:, 2, 3]) / (mom[:, 2, 0] - mom[:, 2, 3]))
    edges = np.quantile(obs, np.linspace(0, 1, 9))
    wt = (w_exact.cpu().numpy())
    expect = np.histogram(obs, edges, weights=wt)[0]
    expect = expect / expect.sum()
    sel, res = obs[two['index'].cpu().numpy()], two['resid'].cpu().numpy()
    got = np.histogram(sel, edges, weights=res)[0]
    # variance of a bin filled with weights r_k is sum r_k^2 (overweights count more)
    var = np.histogram(sel, edges, weights=res ** 2)[0]
    ntot = got.sum()
    chi2 = float((((got - ntot * expect) ** 2) / np.maximum(var, 1.0)).sum())
    _say(f'  chi2 of the two-stage sample vs exact-weighted distribution: {chi2:.1f} (8 bins)')
    assert chi2 < 30
