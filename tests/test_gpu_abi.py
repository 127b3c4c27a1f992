"""Entry points of the C ABI beyond me_compute, on the GPU: the host-pointer
variant, the input check, and graph replay across colour-mode and
helicity-filter changes.  Every test prints its case before touching the GPU.
"""
import numpy as np
import pytest

from oracle import me as ome
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to('cuda')


def test_compute_host_matches_device_and_oracle(binding):
    _say('case compute_host gg_ttxg nevt=200 seed=31')
    mom = rambo.generate(5, 200, 31)
    m = binding.MatrixElement('gg_ttxg')
    host = m.me_compute_host(mom, AS)
    dev = m.compute(_dev(mom), AS)
    torch.cuda.synchronize()
    assert np.array_equal(host, dev.cpu().numpy())
    ref = ome.matrix_element(ome.process(5), mom, AS)
    assert np.max(np.abs(host / ref - 1)) < 1e-12


def test_input_check(binding):
    _say('case input_check gg_ttxgg nevt=130 seed=32')
    mom = rambo.generate(6, 130, 32)
    m = binding.MatrixElement('gg_ttxgg', check=True)
    out = torch.full((130,), -7.0, dtype=torch.float64, device='cuda')
    m.me_compute(_dev(mom), 130, AS, out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    good = out.cpu().numpy()
    ref = ome.matrix_element(ome.process(6), mom, AS)
    assert np.max(np.abs(good / ref - 1)) < 1e-12
    # event 37 off shell (a gluon's energy scaled), event 90 not conserving momentum
    bad = mom.copy()
    bad[37, 4, 0] *= 1.001
    bad[90, 5, 1] += 1e-3
    out.fill_(-7.0)
    with pytest.raises(binding.MeError) as ei:
        m.me_compute(_dev(bad), 130, AS, out, torch.cuda.current_stream())
    assert ei.value.code == binding.ME_EINVAL
    assert '2 event(s)' in str(ei.value) and 'event 37' in str(ei.value)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == -7.0)   # nothing written
    # the same events pass with the check off
    m2 = binding.MatrixElement('gg_ttxgg', check=False)
    m2.me_compute(_dev(bad), 130, AS, out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out.cpu().numpy()))


@pytest.mark.parametrize('name,npar', [('gg_ttxg', 5)])
def test_graph_replay_across_mode_changes(binding, name, npar):
    _say(f'case graph_mode_changes {name} nevt=333 seed=33')
    nevt = 333
    mom = _dev(rambo.generate(npar, nevt, 33))
    eager = {}
    for mode in (binding.ME_CS_FP64, binding.ME_CS_FP16X2, binding.ME_CS_BF16X2):
        e = binding.MatrixElement(name, colorsum_mode=mode)
        eager[mode] = e.compute(mom, AS).cpu().numpy()
    g = binding.MatrixElement(name, use_graph=True)
    out = torch.empty(nevt, dtype=torch.float64, device='cuda')
    seq = [binding.ME_CS_FP64, binding.ME_CS_FP16X2, binding.ME_CS_FP16X2, binding.ME_CS_BF16X2,
           binding.ME_CS_FP16X2, binding.ME_CS_FP64, binding.ME_CS_BF16X2]
    for i, mode in enumerate(seq):
        g.me_set_colorsum_mode(mode)
        if i == 3:
            g.me_set_colorsum_mode(binding.ME_CS_FP16X2)   # changed twice between two computes
            g.me_set_colorsum_mode(mode)
        for rep in range(2):   # capture, then replay
            out.fill_(0.0)
            g.compute(mom, AS, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), eager[mode]), (i, mode, rep)


def test_graph_replay_after_helicity_filter(binding):
    _say('case graph_after_filter gg_ttx nevt=200 seed=34')
    nevt = 200
    mom = _dev(rambo.generate(4, nevt, 34))
    ref = binding.MatrixElement('gg_ttx')
    want = ref.compute(mom, AS).cpu().numpy()
    assert len(ref.me_good_helicities()) == 12
    g = binding.MatrixElement('gg_ttx', use_graph=True, all_helicities=True)
    out = torch.empty(nevt, dtype=torch.float64, device='cuda')
    g.compute(mom, AS, out=out)             # captured with all 16 helicities
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy() / want - 1)) < 1e-13
    g.me_filter_helicities(mom, nevt, AS, torch.cuda.current_stream())
    assert len(g.me_good_helicities()) == 12
    out.fill_(0.0)
    g.compute(mom, AS, out=out)             # must not replay the 16-helicity graph
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
