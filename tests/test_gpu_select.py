"""Helicity / colour selection (me_select) and running alpha_s (me_compute_alphas)
on the GPU vs the oracle.

Selections are integers decided by floating-point cumulative sums: they must
agree with the oracle's draw exactly, except where r * total lies within
1e-9 relative of a boundary between two running sums (there both sides'
rounding may legitimately decide differently); such events are counted and
the GPU's choice is checked to be one of the two neighbours.
"""
import numpy as np
import pytest

from oracle import me as ome, select as osel
from paper_2510_05392_amd import rambo
from test_gpu_parity import AS, NPAR, _say, assert_parity

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2510_05392_amd import binding as b
    b.load()
    return b


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _near_boundary(weights, r, tol=1e-9):
    """Per event: True when r * total is within tol * total of a running sum."""
    w = np.asarray(weights)
    cum = np.cumsum(w, axis=0)
    tot = cum[-1]
    t = r * tot
    return np.any(np.abs(cum - t[None, :]) <= tol * tot[None, :], axis=0)


def _gpu_select(binding, name, mom, rh, rc):
    m = binding.MatrixElement(name)
    n = len(mom)
    out = torch.empty(n, dtype=torch.float64, device='cuda')
    sh = torch.full((n,), -1, dtype=torch.int32, device='cuda')
    sc = torch.full((n,), -1, dtype=torch.int32, device='cuda')
    m.me_select(_dev(mom), n, AS, _dev(rh), _dev(rc), out, sh, sc)
    torch.cuda.synchronize()
    return m, out.cpu().numpy(), sh.cpu().numpy(), sc.cpu().numpy()


@pytest.mark.parametrize('name,nevt,seed', [('gg_ttx', 200, 21), ('gg_ttxg', 133, 22), ('gg_ttxgg', 67, 23)])
def test_select_vs_oracle(binding, name, nevt, seed):
    _say(f'case me_select {name} nevt={nevt}')
    npar = NPAR[name]
    mom = rambo.generate(npar, nevt, seed)
    rng = np.random.default_rng(seed)
    rh, rc = rng.random(nevt), rng.random(nevt)
    m, me2, sh, sc = _gpu_select(binding, name, mom, rh, rc)
    good = m.me_good_helicities()
    proc = ome.process(npar)
    ref_me, ref_h, ref_c = osel.select(proc, mom, AS, rh, rc, good)
    assert_parity(me2, mom, npar, me64=ref_me)
    meh = ome.me_helicities(proc, mom, AS, good)
    amb_h = _near_boundary(meh, rh)
    assert np.isin(sh, good).all()
    agree = sh == ref_h
    assert np.all(agree | amb_h), np.nonzero(~agree & ~amb_h)
    # colour: compare where the helicities agree; elsewhere check validity
    ncol = m.ncolor
    assert np.all((sc >= 0) & (sc < ncol))
    namb_c = 0
    for e in np.nonzero(agree)[0]:
        if sc[e] == ref_c[e]:
            continue
        jam = ome.jamps(proc, mom[e:e + 1], int(sh[e]), AS)[0]
        w = (np.abs(jam) ** 2)[:, None]
        assert _near_boundary(w, rc[e:e + 1])[0], (e, sc[e], ref_c[e])
        namb_c += 1
    _say(f'  helicity agreement {agree.mean():.3f} (boundary cases {int(amb_h.sum())}), '
         f'colour boundary cases {namb_c}')


def test_select_frequencies_one_event(binding):
    # one gg->ttg event repeated with stratified r: helicity counts follow the
    # GPU's own per-helicity sums to within one
    _say('case me_select stratified frequencies')
    n = 8192
    mom = np.repeat(rambo.generate(5, 1, 31), n, axis=0)
    r = (np.arange(n) + 0.5) / n
    m, me2, sh, sc = _gpu_select(binding, 'gg_ttxg', mom, r, r[::-1].copy())
    good = m.me_good_helicities()
    meh = torch.empty((len(good), 1), dtype=torch.float64, device='cuda')
    m.me_helicity_sums(_dev(mom[:1]), 1, AS, good, meh)
    torch.cuda.synchronize()
    w = meh.cpu().numpy()[:, 0]
    counts = np.array([(sh == h).sum() for h in good])
    assert np.all(np.abs(counts - n * w / w.sum()) <= 1.0 + 1e-6)
    assert np.all(me2 == me2[0])


@pytest.mark.parametrize('name,mode', [('gg_ttxg', 0), ('gg_ttxgg', 0), ('gg_ttxgg', 1)])
def test_running_alpha_s(binding, name, mode):
    _say(f'case me_compute_alphas {name} mode={mode}')
    npar = NPAR[name]
    nevt = 200
    mom = rambo.generate(npar, nevt, 41)
    alphas = np.random.default_rng(5).uniform(0.08, 0.2, nevt)
    m = binding.MatrixElement(name, colorsum_mode=mode)
    out = torch.empty(nevt, dtype=torch.float64, device='cuda')
    m.me_compute_alphas(_dev(mom), nevt, _dev(alphas), out)
    torch.cuda.synchronize()
    gpu = out.cpu().numpy()
    proc = ome.process(npar)
    ref = np.array([ome.matrix_element(proc, mom[e:e + 1], alphas[e])[0] for e in range(nevt)])
    if mode == 0:
        assert_parity(gpu, mom, npar, me64=ref)
    else:
        assert np.max(np.abs(gpu / ref - 1)) < 1e-5
    # |M|^2 scales as alpha_s^(npar - 2) against the fixed-coupling path
    fixed = m.compute(_dev(mom), AS).cpu().numpy()
    assert np.allclose(gpu, fixed * (alphas / AS) ** (npar - 2), rtol=1e-12 if mode == 0 else 1e-5)
