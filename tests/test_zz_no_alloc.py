"""me_compute_noalloc (no device allocation: scratch in a static device array)
against me_compute with the same launch, through the C ABI: two calls in a row,
the second with fewer events, results identical; sizes beyond the static array
and unfiltered handles are refused."""
import numpy as np
import pytest

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


@pytest.mark.parametrize('name,npar,n1,n2,seed', [('gg_ttxgg', 6, 5000, 777, 61), ('gg_ttxggg', 7, 1500, 200, 62),
                                                   ('gg_ttxgggg', 8, 130, 67, 63)])
def test_noalloc_matches_compute(binding, name, npar, n1, n2, seed):
    _say(f'case noalloc {name} n1={n1} n2={n2} seed={seed}')
    ref = binding.MatrixElement(name)
    m = binding.MatrixElement(name)
    s = torch.cuda.current_stream()
    for call, n in enumerate((n1, n2)):
        mom = torch.from_numpy(rambo.generate(npar, n, seed + call)).cuda()
        if call == 0:
            m.me_filter_helicities(mom, n, AS, s)
        out = torch.full((n,), -1.0, dtype=torch.float64, device='cuda')
        m.me_compute_noalloc(mom, n, AS, out, s)
        want = ref.compute(mom, AS)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want.cpu().numpy()), (call, np.max(np.abs(got / want.cpu().numpy() - 1)))


def test_noalloc_refuses_oversize_and_unfiltered(binding):
    _say('case noalloc refusals')
    from paper_2510_05392_amd.binding import ME_EINVAL, MeError
    m = binding.MatrixElement('gg_ttxgg')
    mom = torch.from_numpy(rambo.generate(6, 64, 5)).cuda()
    out = torch.empty(64, dtype=torch.float64, device='cuda')
    with pytest.raises(MeError) as ei:
        m.me_compute_noalloc(mom, 64, AS, out)          # helicity filter not yet run
    assert ei.value.code == ME_EINVAL
    m.me_filter_helicities(mom, 64, AS)
    big = 800000                                       # 800000 x (192 + 8) bytes > 128 MiB
    bm = torch.zeros((big, 6, 4), dtype=torch.float64, device='cuda')
    bo = torch.zeros(big, dtype=torch.float64, device='cuda')
    with pytest.raises(MeError) as ei:
        m.me_compute_noalloc(bm, big, AS, bo)
    assert ei.value.code == ME_EINVAL and 'ME_NOALLOC_SCRATCH_BYTES' in str(ei.value)
    torch.cuda.synchronize()
    assert np.all(bo.cpu().numpy() == 0.0)
