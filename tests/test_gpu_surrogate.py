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


def _bf16_bits_ulp(x):
    """One BF16 unit in the last place of each value (2^(e-7) for |x| in [2^e, 2^(e+1)))."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(x, 1e-38)))
    return 2.0 ** (e - 7)


def _silu64(z):
    return z / (1.0 + np.exp(-z))


def _dsilu64(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


GAMMA_FP32 = 2.0 ** -24   # unit roundoff of the FP32 accumulation


@pytest.mark.parametrize('width,depth,nb', [(256, 4, 300), (96, 3, 130), (48, 2, 70), (32, 1, 33)])
def test_surrogate_layers_and_gradients_elementwise(binding, width, depth, nb):
    """Every layer of the GPU network element by element against an FP64 reference
    that takes the GPU's own BF16 inputs and BF16 weights: pre-activations within
    the FP32 accumulation bound gamma_K sum|h||w| (K terms, any order), activations
    equal to bf16(silu(z)) up to one BF16 ulp where the FP32 exponential sits on a
    rounding boundary; gradients of every weight and bias element by element
    against the same reference with dZ rounded to BF16 where the kernels round it
    (bound: four BF16 ulps of each product term plus the FP32 accumulation)."""
    _say(f'case surrogate layers and gradients elementwise (15-{width}x{depth}-1, {nb} rows)')
    nfeat = 15
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
    tg = torch.from_numpy(target).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device='cuda')
    sur.me_sur_grads(feat, tg, nb, loss)
    torch.cuda.synchronize()
    # features: the GPU's BF16 rows against the FP64 ones, except the constant
    # (g1, g2) column whose normalised value is rounding noise amplified by 1 / std
    xg = feat.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)[:, :nfeat]
    xc = (raw - mean) / std
    assert np.all(np.abs(xg[:, 1:] - xc[:, 1:]) <= _bf16_bits_ulp(xc[:, 1:]) + 1e-3)
    L = depth + 1
    H = [sur.me_sur_activations(l, 0, nb).astype(np.float64) for l in range(L)]
    Z = [sur.me_sur_activations(l, 1, nb).astype(np.float64) for l in range(L)]
    assert np.array_equal(H[0], xg)
    w16 = [_bf16(w) for w, _ in params]
    flips = 0
    for l in range(L):
        ref = H[l] @ w16[l].T + params[l][1]
        K = H[l].shape[1]
        bound = K * GAMMA_FP32 * (np.abs(H[l]) @ np.abs(w16[l]).T + np.abs(params[l][1])) + GAMMA_FP32 * np.abs(ref)
        assert np.all(np.abs(Z[l] - ref) <= bound), (l, np.max(np.abs(Z[l] - ref) / np.maximum(bound, 1e-300)))
        if l + 1 < L:
            want = _bf16(_silu64(Z[l]))
            diff = np.abs(H[l + 1] - want)
            assert np.all(diff <= _bf16_bits_ulp(want) * 1.0001), l
            flips += int((diff > 0).sum())
    assert flips <= 0.01 * nb * width * depth
    # gradients: FP64 backward on the GPU's forward activations, dZ rounded to BF16 as
    # the kernels round it (the bias gradients sum the FP32 dZ).  Alongside, a
    # first-order bound on the GPU's deviation: e_f bounds |dZ_gpu - dZ| before the
    # BF16 rounding, e_h after it (a rounding of a perturbed value can land one BF16
    # ulp away, <= 2^-7 |dZ|); every product adds the FP32 accumulation bound and
    # the FP32 SiLU derivative is taken good to 1e-6.
    y = Z[L - 1][:, 0]
    dzf = (2.0 / nb) * (y - target.astype(np.float64))[:, None]
    e_f = 4 * GAMMA_FP32 * np.abs(dzf)
    dzh = _bf16(dzf)
    e_h = e_f + 2.0 ** -7 * np.abs(dzf)
    gref = [None] * L
    bnd = [None] * L
    for l in range(L - 1, -1, -1):
        gref[l] = (dzh.T @ H[l], dzf.sum(axis=0))
        bnd[l] = (e_h.T @ np.abs(H[l]) + nb * GAMMA_FP32 * (np.abs(dzh).T @ np.abs(H[l])),
                  e_f.sum(axis=0) + nb * GAMMA_FP32 * np.abs(dzf).sum(axis=0))
        if l == 0:
            break
        K = dzh.shape[1]
        dh = dzh @ w16[l]
        e_dh = e_h @ np.abs(w16[l]) + K * GAMMA_FP32 * (np.abs(dzh) @ np.abs(w16[l]))
        ds = _dsilu64(Z[l - 1])
        dzf = dh * ds
        e_f = e_dh * np.abs(ds) + np.abs(dh) * 1e-6 + 2 * GAMMA_FP32 * np.abs(dzf)
        dzh = _bf16(dzf)
        e_h = e_f + 2.0 ** -7 * np.abs(dzf)
    ggpu = _unflatten(sur.me_sur_get_grads(), sizes)
    for l, ((gw, gb), (rw, rb), (bw, bb)) in enumerate(zip(ggpu, gref, bnd)):
        for name, a, b, t in (('W', gw, rw, bw), ('b', gb, rb, bb)):
            err = np.abs(a - b)
            assert np.all(err <= t + 1e-30), (l, name, float(np.max(err / np.maximum(t, 1e-300))))
    lref = float(np.mean((y - target) ** 2))
    assert abs(float(loss.item()) / nb - lref) <= 1e-5 * lref
    # end to end against the FP64 reference with its own BF16 rounding (no GPU
    # activations): the same network within a few BF16 ulps of the output
    pb = [(w16[l], params[l][1]) for l in range(L)]
    h = xg
    for l in range(L):
        z = h @ pb[l][0].T + pb[l][1]
        h = _bf16(_silu64(z)) if l + 1 < L else z
    assert np.max(np.abs(Z[L - 1][:, 0] - h[:, 0])) <= 1e-2 * max(1.0, np.abs(h).max())
    # inference (for widths 32 MB <= 256 the whole network in one kernel, with the
    # same products summed in the same order) against the forward pass just run
    yp = torch.empty(nb, dtype=torch.float32, device='cuda')
    sur.me_sur_predict(feat, nb, yp)
    yp = yp.cpu().numpy().astype(np.float64)
    d = np.abs(yp - Z[L - 1][:, 0])
    _say(f'  predict vs forward pass: {int((d == 0).sum())} of {nb} identical, max abs diff {d.max():.3e}')
    assert d.max() <= 1e-3 * max(1.0, np.abs(Z[L - 1][:, 0]).max())


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
    rms, worst = pipe.log_error(val)
    _say(f'  validation RMS log-error {rms:.3f}, largest {worst:.3f} (target spread {pipe.ystd:.3f})')
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
    assert np.array_equal(res['index'].cpu().numpy(), idx)
    gres = res['resid'].cpu().numpy()
    assert np.array_equal(idx[gres > 0], np.nonzero(acc)[0])
    assert np.allclose(gres[gres > 0], resid, rtol=1e-9)
    # the summary kernel against the GPU's own residual weights (an event at the
    # calibration maximum sits on the overweight boundary, where the CPU's exp can
    # land one ulp above 1)
    acc_g = gres[gres > 0]
    assert res['accepted'] == int(acc.sum()) and res['overweight'] == int((acc_g > 1).sum())
    assert np.isclose(res['sum_w'], acc_g.sum(), rtol=1e-13) and np.isclose(res['sum_w2'], (acc_g ** 2).sum(),
                                                                             rtol=1e-13)


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
    one = pipe.unweight_exact(dmom, dw, r2, pipe.exact_weight_max(cal, cw, 0.99))
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


def test_statistics_targets_and_row_gather_vs_numpy(binding):
    """Normalisation statistics, training targets and the per-epoch row gather of the
    library against numpy on the same device data."""
    _say('case surrogate statistics / targets / gather (70001 events)')
    n = 70001
    mom = rambo.generate(6, n, 21)
    dmom = torch.from_numpy(mom).cuda()
    me = binding.MatrixElement('gg_ttxgg')
    me2 = me.compute(dmom, AS)
    sur = binding.Surrogate(15, 64, 1, seed=2)
    raw = torch.empty((n, 15), dtype=torch.float32, device='cuda')
    feat = torch.empty((n, sur.kpad), dtype=torch.int16, device='cuda')
    sur.me_sur_features(dmom, n, 6, feat, raw)
    ymean, ystd = sur.me_sur_fit_normalisation(raw, n, me2)
    torch.cuda.synchronize()
    rh = raw.cpu().numpy().astype(np.float64)
    lm = np.log(me2.cpu().numpy())
    assert abs(ymean - lm.mean()) <= 1e-12 * abs(lm.mean()) and abs(ystd / lm.std() - 1) <= 1e-10
    # the handle now normalises with the fitted statistics: features recomputed
    sur.me_sur_features(dmom, n, 6, feat)
    xg = feat.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)[:, :15]
    mu, sd = rh.mean(axis=0), np.maximum(rh.std(axis=0), 1e-6)
    xc = ((rh - mu.astype(np.float32)) * (1 / sd).astype(np.float32))
    assert np.all(np.abs(xg[:, 1:] - xc[:, 1:]) <= _bf16_bits_ulp(xc[:, 1:]) * 1.0001 + 1e-6)
    tgt = torch.empty(n, dtype=torch.float32, device='cuda')
    binding.me_sur_targets(me2, n, ymean, ystd, tgt)
    want = ((lm - ymean) / ystd).astype(np.float32)
    got = tgt.cpu().numpy()
    assert np.all(np.abs(got - want) <= np.spacing(np.abs(want)))
    perm = np.random.default_rng(4).permutation(n).astype(np.int64)
    fo = torch.empty_like(feat)
    to = torch.empty_like(tgt)
    binding.me_sur_gather_rows(feat, tgt, torch.from_numpy(perm).cuda(), n, sur.kpad, fo, to)
    torch.cuda.synchronize()
    assert np.array_equal(fo.cpu().numpy(), feat.cpu().numpy()[perm])
    assert np.array_equal(to.cpu().numpy(), got[perm])


@pytest.mark.parametrize('n,q', [(1, 0.99), (2, 0.5), (1000, 1.0), (65537, 0.99), (65536, 0.5), (4097, 0.001)])
def test_maxima_quantiles_onestage_summary_vs_numpy(binding, n, q):
    """Quantiles by device radix selection (linear interpolation between order
    statistics, numpy's default), one-stage unweighting, residual-weight summary
    and log error against numpy on the same inputs."""
    _say(f'case unweighting maxima n={n} q={q}')
    rng = np.random.default_rng(n)
    y = rng.normal(size=n).astype(np.float32)
    wps = rng.lognormal(size=n)
    me2 = rng.lognormal(mean=-20, sigma=3, size=n)
    # ties: a block of equal weights
    me2[: n // 3] = me2[0]
    wps[: n // 3] = wps[0]
    r = rng.random(n)
    ymean, ystd = -20.0, 3.0
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    what_max, x_max = binding.me_unweight_maxima(d(y), d(wps), d(me2), n, ymean, ystd, q)
    what = np.exp(y.astype(np.float64) * ystd + ymean) * wps
    x = me2 * wps / what
    ref = (lambda v: v.max()) if q >= 1 else (lambda v: np.quantile(v, q))
    assert abs(what_max / ref(what) - 1) < 1e-14 and abs(x_max / ref(x) - 1) < 1e-14
    w = me2 * wps
    w_max = binding.me_unweight_quantile(d(me2), d(wps), n, q)
    assert abs(w_max / ref(w) - 1) < 1e-14
    resid = torch.empty(n, dtype=torch.float64, device='cuda')
    binding.me_unweight_onestage(d(me2), d(wps), d(r), n, w_max, resid)
    acc = r < np.minimum(1.0, w / w_max)
    want = np.where(acc, np.maximum(1.0, w / w_max), 0.0)
    got = resid.cpu().numpy()
    assert np.array_equal(got > 0, acc) and np.allclose(got, want, rtol=1e-15, atol=0)
    na, no, sw, sw2 = binding.me_unweight_summary(resid, n)
    assert na == int(acc.sum()) and no == int((want > 1).sum())
    assert np.isclose(sw, want.sum(), rtol=1e-13) and np.isclose(sw2, (want ** 2).sum(), rtol=1e-13)
    rms, worst = binding.me_sur_log_error(d(y), d(me2), n, ymean, ystd)
    dl = y.astype(np.float64) * ystd + ymean - np.log(me2)
    assert abs(rms / np.sqrt(np.mean(dl ** 2)) - 1) < 1e-12 and abs(worst / np.abs(dl).max() - 1) < 1e-14


def test_surrogate_at_configured_size(binding):
    """The surrogate configuration on gg -> t tbar g g at its full size: training
    on 2^21 events (seed 2001) labelled by the exact path (split-BF16 colour sum),
    the first 4096 labels against the oracle within that mode's stated bound, and
    two-stage unweighting of 2^20 events (seed 2002), unbiased against the exact
    weights of the same events (chi^2 of an observable) with most exact calls
    saved."""
    import os

    from paper_2510_05392_amd.surrogate import SurrogatePipeline
    from test_gpu_parity import GOLDEN
    _say('case surrogate at its configured size: 2097152 training events, 1048576 unweighted')
    pipe = SurrogatePipeline('gg_ttxgg', width=256, depth=4, seed=11, colorsum_mode=binding.ME_CS_BF16X2)
    train = torch.from_numpy(rambo.generate(6, 2097152, 2001)).cuda()
    labels = pipe.exact(train[:4096]).cpu().numpy()
    g = np.load(os.path.join(GOLDEN, 'gg_ttxgg_seed2001_first4096.npz'))
    rel = np.abs(labels / g['me'] - 1)
    _say(f'  labels vs oracle (first 4096): max rel {rel.max():.2e}')
    assert rel.max() < 2e-4
    hist = pipe.fit(train, epochs=4, batch=4096, lr=2e-3, lr_final=1e-4)
    del train
    _say(f'  training mse per epoch: {[round(h, 5) for h in hist]}')
    assert hist[-1] < hist[0]
    val = torch.from_numpy(rambo.generate(6, 65536, 2003)).cuda()
    rms, worst = pipe.log_error(val)
    _say(f'  validation RMS log-error {rms:.3f} (target spread {pipe.ystd:.3f})')
    assert rms < 0.25 * pipe.ystd
    n = 1048576
    mom, wps = rambo.generate(6, n, 2002, return_weights=True)
    dmom, dw = torch.from_numpy(mom).cuda(), torch.from_numpy(wps).cuda()
    calm, calw = rambo.generate(6, 65536, 2005, return_weights=True)
    dcal, dcw = torch.from_numpy(calm).cuda(), torch.from_numpy(calw).cuda()
    what_max, x_max = pipe.calibrate(dcal, dcw, quantile=0.99)
    gen = torch.Generator(device='cuda').manual_seed(21)
    r1 = torch.rand(n, dtype=torch.float64, device='cuda', generator=gen)
    r2 = torch.rand(n, dtype=torch.float64, device='cuda', generator=gen)
    two = pipe.unweight(dmom, dw, r1, r2, what_max, x_max)
    saved = 1 - two['stage1'] / n
    _say(f"  stage-1 events {two['stage1']} (exact calls saved {saved:.1%}), accepted {two['accepted']}, "
         f"overweights {two['overweight']}, ESS {two['ess']:.1f}")
    assert saved > 0.9
    w_exact = (pipe.exact(dmom) * dw).cpu().numpy()
    obs = 0.5 * np.log((mom[:, 2, 0] + mom[:, 2, 3]) / (mom[:, 2, 0] - mom[:, 2, 3]))
    edges = np.quantile(obs, np.linspace(0, 1, 9))
    expect = np.histogram(obs, edges, weights=w_exact)[0]
    expect = expect / expect.sum()
    sel, res = obs[two['index'].cpu().numpy()], two['resid'].cpu().numpy()
    got = np.histogram(sel, edges, weights=res)[0]
    var = np.histogram(sel, edges, weights=res ** 2)[0]
    chi2 = float((((got - got.sum() * expect) ** 2) / np.maximum(var, 1.0)).sum())
    _say(f'  chi2 of the two-stage sample vs exact-weighted distribution: {chi2:.1f} (8 bins)')
    assert chi2 < 30
