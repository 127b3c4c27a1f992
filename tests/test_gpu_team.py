"""Team executor (one team of lanes per (event, helicity), currents in LDS)
vs the oracle and vs the one-lane-per-(event, helicity) executor.

Same FP64 arithmetic per routine; only the rounding order of the colour-flow
accumulation and of the colour sum differ, so the two executors agree to
~1e-13 relative and both meet the 1e-12 bar against the oracle.
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


def _run(binding, name, mom, executor, target_waves=4096, alphas=None):
    m = binding.MatrixElement(name)
    m.me_set_launch(0, 1, 0, target_waves)
    m.me_set_executor(executor)
    d = torch.from_numpy(np.ascontiguousarray(mom)).cuda()
    out = torch.empty(len(mom), dtype=torch.float64, device='cuda')
    if alphas is None:
        m.me_compute(d, len(mom), AS, out)
    else:
        m.me_compute_alphas(d, len(mom), torch.from_numpy(alphas).cuda(), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize('name,nevt,seed', [('gg_ttx', 257, 1001), ('gg_ttxg', 133, 22), ('gg_ttxgg', 67, 23),
                                            ('gg_ttxg', 1, 5), ('gg_ttxgg', 3, 6)])
def test_team_vs_oracle_and_lane(binding, name, nevt, seed):
    _say(f'case team {name} nevt={nevt}')
    npar = NPAR[name]
    mom = rambo.generate(npar, nevt, seed)
    team = _run(binding, name, mom, binding.ME_EXEC_TEAM)
    lane = _run(binding, name, mom, binding.ME_EXEC_LANE)
    rel = np.abs(team / lane - 1)
    _say(f'  team vs lane max rel {rel.max():.2e}')
    assert rel.max() < 1e-13
    assert_parity(team, mom, npar)


def test_team_ggttggg_golden(binding):
    _say('case team ggttggg golden 197 events')
    g = _golden('gg_ttxggg_seed1003_first197.npz')
    mom = rambo.generate(7, 197, 1003)
    team = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_TEAM)
    assert_parity(team, mom, 7, me64=g['me'], me_ext=g['me_ext'])


@pytest.mark.parametrize('tw', [64, 1 << 20])
def test_team_helicity_chunking(binding, tw):
    # one chunk with every helicity, or one helicity per chunk: same result up to rounding order
    _say(f'case team chunking target_waves={tw}')
    mom = rambo.generate(6, 100, 24)
    a = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_TEAM, target_waves=tw)
    b = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_LANE)
    assert np.max(np.abs(a / b - 1)) < 1e-13


def test_team_deterministic_and_alphas(binding):
    _say('case team determinism and running alpha_s')
    mom = rambo.generate(6, 130, 25)
    a = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_TEAM)
    b = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_TEAM)
    assert np.array_equal(a, b)
    alphas = np.random.default_rng(2).uniform(0.08, 0.2, 130)
    c = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_TEAM, alphas=alphas)
    assert np.allclose(c, a * (alphas / AS) ** 4, rtol=1e-12)


def test_team_full_size_ggttggg_sampled(binding):
    # the benchmark workload in the team executor, sampled events against the oracle
    _say('case team full size ggttggg 262144')
    mom = rambo.generate(7, 262144, 1003)
    team = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_TEAM)
    assert np.all(np.isfinite(team)) and np.all(team > 0)
    g = _golden('gg_ttxggg_seed1003_n262144_sampled.npz')
    idx = g['index']
    assert_parity(team[idx], mom[idx], 7, me64=g['me'], me_ext=g['me_ext'])


def test_team_only_process_ggttgggg(binding):
    # g g -> t tbar g g g g (15495 diagrams, 720 colour flows) has only the team
    # program; the stored oracle values cover 24 events of its 32768-event workload
    _say('case team ggttgggg full size 32768, 24 sampled events against the oracle')
    g = _golden('gg_ttxgggg_seed1005_n32768_sampled.npz')
    full = rambo.generate(8, 32768, 1005)
    idx = g['index']
    assert np.array_equal(full[idx], g['momenta'])
    m = binding.MatrixElement('gg_ttxgggg')
    assert m.ncolor == 720 and m.ndiag == 15495
    with pytest.raises(binding.MeError):
        m.me_set_executor(binding.ME_EXEC_LANE)
    out = m.compute(torch.from_numpy(full).cuda(), AS)
    torch.cuda.synchronize()
    gpu = out.cpu().numpy()
    assert len(m.me_good_helicities()) == 256
    assert np.all(np.isfinite(gpu)) and np.all(gpu > 0)
    assert_parity(gpu[idx], full[idx], 8, me64=g['me'], me_ext=g['me_ext'])


def test_ggttgggg_mixed_colour_sum(binding):
    # team program writing the 720 colour flows, split-FP16 colour sum on the
    # matrix cores (the integer colour matrix, entries up to 32768, is exact in FP16)
    _say('case ggttgggg split-FP16 colour sum, 24 sampled events')
    g = _golden('gg_ttxgggg_seed1005_n32768_sampled.npz')
    mom = g['momenta']
    m = binding.MatrixElement('gg_ttxgggg', colorsum_mode=binding.ME_CS_FP16X2)
    out = m.compute(torch.from_numpy(np.ascontiguousarray(mom)).cuda(), AS)
    torch.cuda.synchronize()
    rel = np.abs(out.cpu().numpy() / g['me_ext'] - 1)
    _say(f'  max rel err {rel.max():.3e}')
    assert rel.max() < 1e-5


def test_team_graph_replay_matches_eager(binding):
    # the captured launch sequence of the team executor, replayed with new
    # buffer contents and eager work in between, equals eager evaluation
    _say('case team graph replay gg_ttxgg')
    mom = rambo.generate(6, 130, 51)
    mom2 = rambo.generate(6, 130, 52)
    eager = binding.MatrixElement('gg_ttxgg')
    eager.me_set_executor(binding.ME_EXEC_TEAM)
    graph = binding.MatrixElement('gg_ttxgg', use_graph=True)
    graph.me_set_executor(binding.ME_EXEC_TEAM)
    d = torch.from_numpy(mom).cuda()
    out = torch.empty(130, dtype=torch.float64, device='cuda')
    ref = eager.compute(d, AS).cpu().numpy()
    ref2 = eager.compute(torch.from_numpy(mom2).cuda(), AS).cpu().numpy()
    s = torch.cuda.current_stream()
    for rep in range(4):
        d.copy_(torch.from_numpy(mom if rep % 2 == 0 else mom2))
        torch.cuda.synchronize()
        graph.me_compute(d, 130, AS, out, s)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref if rep % 2 == 0 else ref2), rep
        _ = eager.compute(d, AS)
