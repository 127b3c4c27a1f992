"""Split executor (colour-group sums stored per (event, helicity), then the
colour flows and the colour form in a second kernel) vs the oracle and vs the
one-lane executor.

Same FP64 routines; only the rounding order of the flow accumulation differs,
so the executors agree to ~1e-13 relative and meet the 1e-12 bar against the
oracle.  The full-size workloads span several event chunks of the group-sum
scratch.
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


def _run(binding, name, mom, executor, alphas=None, graph=False, mode=0):
    m = binding.MatrixElement(name, use_graph=graph, colorsum_mode=mode)
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
def test_split_vs_oracle_and_lane(binding, name, nevt, seed):
    _say(f'case split {name} nevt={nevt}')
    npar = NPAR[name]
    mom = rambo.generate(npar, nevt, seed)
    split = _run(binding, name, mom, binding.ME_EXEC_SPLIT)
    lane = _run(binding, name, mom, binding.ME_EXEC_LANE)
    rel = np.abs(split / lane - 1)
    _say(f'  split vs lane max rel {rel.max():.2e}')
    assert rel.max() < 1e-13
    assert_parity(split, mom, npar)


def test_split_ggttggg_golden(binding):
    _say('case split ggttggg golden 197 events')
    g = _golden('gg_ttxggg_seed1003_first197.npz')
    mom = rambo.generate(7, 197, 1003)
    assert_parity(_run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_SPLIT), mom, 7, me64=g['me'], me_ext=g['me_ext'])


def test_split_full_size_multi_chunk(binding):
    # the benchmark workload (several event chunks of the group-sum scratch), sampled
    # events against the oracle, and gg->ttgg at 524288 events against the lane executor
    _say('case split full size ggttggg 262144')
    mom = rambo.generate(7, 262144, 1003)
    split = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_SPLIT, graph=True)
    assert np.all(np.isfinite(split)) and np.all(split > 0)
    g = _golden('gg_ttxggg_seed1003_n262144_sampled.npz')
    idx = g['index']
    assert_parity(split[idx], mom[idx], 7, me64=g['me'], me_ext=g['me_ext'])
    _say('case split full size ggttgg 524288 vs lane')
    mom = rambo.generate(6, 524288, 1002)
    a = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_SPLIT)
    b = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_LANE)
    assert np.max(np.abs(a / b - 1)) < 1e-13


def test_split_deterministic_alphas_and_graph(binding):
    _say('case split determinism, running alpha_s, graph replay')
    mom = rambo.generate(6, 130, 25)
    a = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_SPLIT)
    b = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_SPLIT, graph=True)
    assert np.array_equal(a, b)
    alphas = np.random.default_rng(2).uniform(0.08, 0.2, 130)
    c = _run(binding, 'gg_ttxgg', mom, binding.ME_EXEC_SPLIT, alphas=alphas)
    assert np.allclose(c, a * (alphas / AS) ** 4, rtol=1e-12)
    with pytest.raises(binding.MeError):
        binding.MatrixElement('gg_ttxgggg').me_set_executor(binding.ME_EXEC_SPLIT)


@pytest.mark.parametrize('executor,mode,expect', [(2, 0, [1, 1, 1, 1]), (0, 0, [1, 0, 0, 1]), (1, 0, [1, 0, 0, 1]),
                                                  (0, 1, [1, 0, 1, 1]), (2, 1, [1, 1, 1, 1])])
def test_kernel_timing(binding, executor, mode, expect):
    # per-kernel events: one launch per kernel class of a one-chunk call, durations
    # positive, results equal to an untimed call (also on a graph handle, which runs
    # eagerly while timing is on), counters reset on reading
    _say(f'case kernel timing executor={executor} mode={mode}')
    mom = rambo.generate(6, 130, 26)
    d = torch.from_numpy(mom).cuda()
    m = binding.MatrixElement('gg_ttxgg', colorsum_mode=mode, use_graph=True)
    m.me_set_executor(executor)
    ref = m.compute(d, AS).cpu().numpy()
    m.me_set_kernel_timing(True)
    got = m.compute(d, AS).cpu().numpy()
    ms, n = m.me_kernel_times()
    assert n == expect
    assert all((t > 0) == (c > 0) for t, c in zip(ms, n))
    assert np.array_equal(got, ref)
    ms, n = m.me_kernel_times()
    assert n == [0, 0, 0, 0]
    m.compute(d, AS)
    m.me_set_kernel_timing(False)
    assert np.array_equal(m.compute(d, AS).cpu().numpy(), ref)
    assert m.me_kernel_times()[1] == [0, 0, 0, 0]


@pytest.mark.parametrize('mode', [1, 2])
def test_split_flows_into_matrix_core_colour_sum(binding, mode):
    # the split executor's flows ([2 ncol][rows] layout) into the split-FP16 / BF16
    # matrix-core colour sum: within 1e-5 of the oracle, and equal to the one-lane
    # kernel's matrix-core result up to the rounding of the flows
    _say(f'case split flows into matrix-core colour sum, mode {mode}')
    g = _golden('gg_ttxggg_seed1003_first197.npz')
    mom = rambo.generate(7, 197, 1003)
    split = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_SPLIT, mode=mode)
    lane = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_LANE, mode=mode)
    rel = np.abs(split / g['me_ext'] - 1)
    _say(f'  max rel err vs oracle {rel.max():.2e}; vs lane {np.max(np.abs(split / lane - 1)):.2e}')
    assert rel.max() < 1e-5
    assert np.max(np.abs(split / lane - 1)) < 1e-6
    for name, npar, n in (('gg_ttx', 4, 77), ('gg_ttxgg', 6, 131)):
        mom = rambo.generate(npar, n, 31)
        a = _run(binding, name, mom, binding.ME_EXEC_SPLIT, mode=mode)
        b = _run(binding, name, mom, binding.ME_EXEC_SPLIT)
        assert np.max(np.abs(a / b - 1)) < 1e-5


def test_split_matrix_core_full_size(binding):
    # the benchmark workload through the split executor with the split-FP16 colour sum
    # (many event chunks, graph replay) against the FP64 split executor
    _say('case split + FP16 colour sum, full size ggttggg 262144')
    mom = rambo.generate(7, 262144, 1003)
    a = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_SPLIT, mode=1, graph=True)
    b = _run(binding, 'gg_ttxggg', mom, binding.ME_EXEC_SPLIT)
    rel = np.abs(a / b - 1)
    _say(f'  max rel {rel.max():.2e}')
    assert rel.max() < 1e-5
