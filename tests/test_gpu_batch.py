"""Uneven multi-process batches in one persistent launch (me_compute_batch).

Each segment must equal what me_compute gives for that process alone (same
FP64 arithmetic; only the rounding order of the helicity sum may differ) and,
on sampled events, the oracle to 1e-12 relative.
"""
import numpy as np
import pytest

from paper_2510_05392_amd import rambo
from test_gpu_parity import AS, NPAR, _golden, _say, assert_parity

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2510_05392_amd import binding as b
    b.load()
    return b


def _run_batch(binding, names, moms):
    hs = [binding.MatrixElement(n) for n in names]
    dm = [torch.from_numpy(m).cuda() if len(m) else None for m in moms]
    outs = [torch.full((max(1, len(m)),), -1.0, dtype=torch.float64, device='cuda') for m in moms]
    binding.me_compute_batch(hs, dm, [len(m) for m in moms], AS, outs)
    torch.cuda.synchronize()
    return hs, [o.cpu().numpy()[:len(m)] for o, m in zip(outs, moms)]


def _single(binding, name, mom):
    m = binding.MatrixElement(name)
    out = m.compute(torch.from_numpy(mom).cuda(), AS)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_uneven_batch_three_processes(binding):
    # gg->ttg 8192 + gg->ttgg 65536 + gg->ttggg 16384 events in one launch
    _say('case batch ggttg 8192 + ggttgg 65536 + ggttggg 16384')
    names = ['gg_ttxg', 'gg_ttxgg', 'gg_ttxggg']
    sizes = [8192, 65536, 16384]
    seeds = [1004, 1002, 1003]
    moms = [rambo.generate(NPAR[n], k, s) for n, k, s in zip(names, sizes, seeds)]
    _, outs = _run_batch(binding, names, moms)
    for n, mom, out in zip(names, moms, outs):
        ref = _single(binding, n, mom)
        rel = np.abs(out / ref - 1)
        _say(f'  {n}: max rel diff vs single-process launch {rel.max():.2e}')
        assert np.all(np.isfinite(out)) and rel.max() < 1e-13
    # against the oracle: sampled events of the two smaller processes, and the
    # first 197 gg->ttggg events against the stored oracle values
    for n, mom, out in zip(names[:2], moms[:2], outs[:2]):
        idx = np.linspace(0, len(mom) - 1, 67).astype(int)
        assert_parity(out[idx], mom[idx], NPAR[n])
    g = _golden('gg_ttxggg_seed1003_first197.npz')
    assert np.array_equal(moms[2][:197], g['momenta'])
    assert_parity(outs[2][:197], moms[2][:197], 7, me64=g['me'], me_ext=g['me_ext'])


def test_ragged_batch_with_empty_segment(binding):
    _say('case batch ragged: ggtt 1, ggttg 0, ggttgg 37, ggttggg 70')
    names = ['gg_ttx', 'gg_ttxg', 'gg_ttxgg', 'gg_ttxggg']
    moms = [rambo.generate(4, 1, 11), np.zeros((0, 5, 4)), rambo.generate(6, 37, 12),
            rambo.generate(7, 70, 13)]
    _, outs = _run_batch(binding, names, moms)
    assert len(outs[1]) == 0
    for n, mom, out in zip(names, moms, outs):
        if len(mom):
            rel = np.abs(out / _single(binding, n, mom) - 1)
            assert rel.max() < 1e-13, (n, rel.max())
    for n, mom, out in zip(names[:3], moms[:3], outs[:3]):
        if len(mom):
            assert_parity(out, mom, NPAR[n])


def test_batch_errors(binding):
    _say('case batch argument errors')
    a = binding.MatrixElement('gg_ttx')
    mom = torch.from_numpy(rambo.generate(4, 64, 3)).cuda()
    out = torch.empty(64, dtype=torch.float64, device='cuda')
    with pytest.raises(binding.MeError):
        binding.me_compute_batch([a, a], [mom, mom], [64, 64], AS, [out, out])
    with pytest.raises(binding.MeError):
        binding.me_compute_batch([a], [mom], [-1], AS, [out])
    with pytest.raises(binding.MeError):
        binding.me_compute_batch([a] * 9, [mom] * 9, [64] * 9, AS, [out] * 9)
    with pytest.raises(binding.MeError):
        binding.me_compute_batch([a], [None], [64], AS, [out])
    # a valid call afterwards still works
    binding.me_compute_batch([a], [mom], [64], AS, [out])
    torch.cuda.synchronize()
    assert torch.all(out > 0)
