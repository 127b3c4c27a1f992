"""The autotuner's candidates on the GPU: every launch configuration, executor and
split-executor variant it can pick gives the oracle's |M|^2 (stored golden
values, 1e-12 per event with adjudication); the result cache and the autotune
parameter."""
import json
import os

import numpy as np
import pytest

from paper_2510_05392_amd import rambo
from test_gpu_parity import AS, GOLDEN, _say, assert_parity

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def binding():
    if not torch.cuda.is_available():
        pytest.fail('GPU tests need a GPU')
    from paper_2510_05392_amd import binding as b
    b.load()
    return b


def _golden197():
    g = np.load(os.path.join(GOLDEN, 'gg_ttxggg_seed1003_first197.npz'))
    return g['momenta'], g['me'], g['me_ext']


def test_every_candidate_matches_the_oracle(binding):
    _say('case autotune candidates gg_ttxggg 197 golden events')
    mom, me64, ext = _golden197()
    d = torch.from_numpy(mom).cuda()
    lane = [(0, 1, 0, 1024), (0, 1, 0, 4096), (0, 1, 0, 16384), (1, 1, 0, 4096), (1, 1, 8, 4096), (1, 2, 8, 4096),
            (1, 1, 1, 4096), (1, 2, 1, 4096)]
    cases = [('lane',) + c for c in lane] + [('team', 0, 1, 0, tw) for tw in (1024, 262144, 1048576)]
    cases += [('split', w, f, r) for w in (1, 2) for f in (8, 16, 32) for r in (0, 2)]
    cases += [('bg', v) for v in (0, 1, 2, 3, 4, 5)]
    for c in cases:
        m = binding.MatrixElement('gg_ttxggg')
        if c[0] == 'lane':
            m.me_set_launch(*c[1:])
        elif c[0] == 'team':
            m.me_set_executor(binding.ME_EXEC_TEAM)
            m.me_set_launch(*c[1:])
        elif c[0] == 'split':
            m.me_set_executor(binding.ME_EXEC_SPLIT)
            m.me_set_split(c[1], c[2], c[3], 0)
        else:
            m.me_set_executor(binding.ME_EXEC_BG)
            m.me_set_bg(c[1])
        gpu = m.compute(d, AS).cpu().numpy()
        assert_parity(gpu, mom, 7, me64=me64, me_ext=ext)
    # the split variants in a matrix-core mode agree with each other to rounding
    outs = []
    for w in (1, 2):
        for f in (8, 16, 32):
            m = binding.MatrixElement('gg_ttxggg', colorsum_mode=binding.ME_CS_FP16X2)
            m.me_set_executor(binding.ME_EXEC_SPLIT)
            m.me_set_split(w, f, 0, 0)
            outs.append(m.compute(d, AS).cpu().numpy())
    for o in outs:
        assert np.max(np.abs(o / me64 - 1)) < 1e-5
    with pytest.raises(binding.MeError):
        binding.MatrixElement('gg_ttxggg').me_set_split(3, 0, 0, 0)
    with pytest.raises(binding.MeError):
        binding.MatrixElement('gg_ttxgggg').me_set_split(1, 16, 0, 0)
    with pytest.raises(binding.MeError):
        binding.MatrixElement('gg_ttxggg').me_set_bg(6)
    for v in (3, 4, 5):
        with pytest.raises(binding.MeError):
            binding.MatrixElement('gg_ttxgggg').me_set_bg(v)   # helicity recycling: four and five gluons


def test_autotune_cache_and_parameter(binding, tmp_path, monkeypatch):
    _say('case autotune cache gg_ttxgg 8192 events')
    cache = tmp_path / 'tune.json'
    monkeypatch.setenv('ME_TUNE_CACHE', str(cache))
    mom = torch.from_numpy(rambo.generate(6, 8192, 41)).cuda()
    out = torch.empty(8192, dtype=torch.float64, device='cuda')
    ref = binding.MatrixElement('gg_ttxgg').compute(mom, AS).cpu().numpy()
    fp64_best = None
    for mode in (binding.ME_CS_FP64, binding.ME_CS_BF16X2):
        a = binding.MatrixElement('gg_ttxgg', colorsum_mode=mode)
        best = a.me_autotune(mom, 8192, AS, out)
        _say(f'  mode {mode}: chosen {best}')
        lines = cache.read_text().splitlines()
        entry = json.loads(lines[-1])
        assert entry['config'] == [best[k] for k in binding.MatrixElement.TUNE_FIELDS]
        # a second handle takes the stored configuration without timing anything
        b = binding.MatrixElement('gg_ttxgg', colorsum_mode=mode)
        assert b.me_autotune(mom, 8192, AS, out) == best
        assert len(cache.read_text().splitlines()) == len(lines)
        got = b.compute(mom, AS).cpu().numpy()
        # the chosen executor may be another algorithm than the default one (each
        # candidate is held to the oracle in the test above): agreement to rounding
        tol = 1e-12 if mode == binding.ME_CS_FP64 else 1e-4
        assert np.max(np.abs(got / ref - 1)) < tol
        fp64_best = best if mode == binding.ME_CS_FP64 else fp64_best
    # the autotune parameter tunes on the first call (found in the cache here): the
    # same configuration and the same numbers as the handle configured by hand
    c = binding.MatrixElement('gg_ttxgg', autotune=True)
    got = c.compute(mom, AS).cpu().numpy()
    d = binding.MatrixElement('gg_ttxgg')
    assert d.me_autotune(mom, 8192, AS, out) == fp64_best
    assert np.array_equal(got, d.compute(mom, AS).cpu().numpy())
    assert len(cache.read_text().splitlines()) == 2
