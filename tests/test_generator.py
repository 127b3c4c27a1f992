"""The process generator of the HIP path, checked on the CPU.

The generator (its own diagram enumeration, colour reduction, colour matrix
and evaluation plan) is compared with the oracle, and its emitted device code
is compiled for the host (test-only stand-in header) and evaluated against
the oracle per helicity.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import colour as ocolour, me as ome
from paper_2510_05392_amd import flops, rambo
from paper_2510_05392_amd.gen import colour as gcolour, topology

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from cpu_harness import build as harness  # noqa: E402

AS = 0.118


@pytest.mark.parametrize('n,ndiag', [(2, 3), (3, 16), (4, 123), (5, 1240)])
def test_generator_diagram_counts(n, ndiag):
    plan = topology.Plan(n, sweeps=0) if n < 5 else topology.Plan(n)
    assert plan.ndiagrams == ndiag
    assert len(plan.amps) == len(plan.pieces)


@pytest.mark.parametrize('n', [2, 3, 4, 5])
def test_generator_colour_matrix_matches_oracle(n):
    cf, den = gcolour.colour_matrix(n)
    ref = ocolour.colour_matrix(n)
    for i, row in enumerate(cf):
        for j, v in enumerate(row):
            assert v == ref[i][j] * den


@pytest.mark.parametrize('n', [2, 3, 4])
def test_generator_colour_coefficients_match_oracle(n):
    # the same multiset of (colour flow, coefficient) over all diagram pieces
    plan = topology.Plan(n, sweeps=0)
    proc = ome.process(n + 2)
    mine = [str(sorted(((w, complex(c)) for w, c in col.items()), key=str)) for col in plan.colours]
    theirs = [str(sorted(((proc.basis[s], c) for s, c in cf), key=str)) for cf in proc.coefs]
    assert len(mine) == len(theirs)
    assert sorted(map(str, mine)) == sorted(map(str, theirs))


def test_every_piece_is_evaluated_once():
    for n in (3, 4, 5):
        plan = topology.Plan(n)
        assert sorted(a[0] for a in plan.amps) == list(range(len(plan.pieces)))
        # every group member appears exactly once in the emitted schedule
        seen = [a[0] for _, mem in plan.scheduled_groups() for _, a in mem]
        assert sorted(seen) == list(range(len(plan.pieces)))


def test_flop_model_is_positive_and_monotone():
    f = [flops.per_event_helicity(p) for p in ('gg_ttx', 'gg_ttxg', 'gg_ttxgg')]
    assert all(b > 4 * a for a, b in zip(f, f[1:]))


# count_routine's order in tests/cpu_harness/count_harness.cpp
ROUTINES = ['G', 'Gbeam', 'U', 'V', 'v3', 'v4', 'v4', 'v4', 'Lh', 'Rh', 'L', 'R', 'K', 'KD3', 'KD4', 'KD4', 'KD4',
            'sdot', 'vdot', 'msq']


@pytest.mark.parametrize('name,npar,opt', [('gg_ttx', 4, '-O1'), ('gg_ttxg', 5, '-O1'), ('gg_ttxgg', 6, '-O1'),
                                           ('gg_ttxggg', 7, '-O0')])
def test_flop_figures_equal_the_counted_operations(name, npar, opt):
    """The flop figures of the roofline (per-routine table summed by the emitter)
    equal the operations the generated code performs, counted by compiling it for
    the host with an operation-counting scalar: every routine, and the whole
    one-lane code, group-sum code and colour form of each process, on workload
    events whose top / antitop take either branch of the spinor code."""
    from paper_2510_05392_amd.gen import colour as gc
    h = harness.build_count(name, opt)
    for i, r in enumerate(ROUTINES):
        assert h.routine(i) == flops.ROUTINE[r], r
    plan = topology.Plan(npar - 2)
    amp, sums = flops.amplitudes_flops(name, plan), flops.group_sums_flops(name, plan)
    cf, _ = gc.colour_matrix(npar - 2)
    assert h.colour_sum() == flops.colour_sum_flops(cf)
    mom = rambo.generate(npar, 6, 1003)
    for e in range(mom.shape[0]):
        neg = int((mom[e, 2:4, 3] < 0).sum())
        for hel in (0, 2 ** npar - 1, 5):
            assert h.amplitudes(mom[e], hel) == amp + neg
            assert h.group_sums(mom[e], hel) == sums + neg
    assert flops.diagram_kernel(name, 2) == sums + flops.QUARK_BRANCH_MEAN


@pytest.mark.parametrize('name,npar,nevt,opt,hels', [
    ('gg_ttx', 4, 16, '-O1', None), ('gg_ttxg', 5, 8, '-O1', None),
    ('gg_ttxgg', 6, 6, '-O1', None), ('gg_ttxggg', 7, 2, '-O0', (0, 17, 64, 100, 127))])
def test_generated_code_on_host_vs_oracle(name, npar, nevt, opt, hels):
    h = harness.build(name, opt)
    mom = rambo.generate(npar, nevt, 5)
    proc = ome.process(npar)
    hels = list(range(2 ** npar)) if hels is None else list(hels)
    meh, jam = h.eval(mom, math.sqrt(4 * math.pi * AS), 173.0, hels, want_jamps=True)
    ref = ome.me_helicities(proc, mom, AS, hels)
    assert np.max(np.abs(meh - ref) / ref.max(axis=0)) < 1e-12
    # dual amplitudes agree up to one phase per (event, helicity)
    jo = np.stack([ome.jamps(proc, mom, hh, AS) for hh in hels])
    jscale = np.abs(jo).max(axis=(0, 2))
    num = (jam * np.conj(jo)).sum(axis=2)
    den = (np.abs(jo) ** 2).sum(axis=2)
    ok = den > 1e-20 * jscale[None, :] ** 2
    ph = np.where(ok, num / np.where(ok, den, 1), 1)
    dev = np.abs(jam - ph[..., None] * jo).max(axis=(0, 2))
    assert np.all(dev <= 1e-12 * jscale)


@pytest.mark.parametrize('name,npar,nevt,opt,hels', [
    ('gg_ttx', 4, 16, '-O1', None), ('gg_ttxg', 5, 8, '-O1', None),
    ('gg_ttxgg', 6, 4, '-O1', None), ('gg_ttxggg', 7, 2, '-O0', (0, 17, 64, 100, 127))])
def test_team_program_on_host_vs_oracle(name, npar, nevt, opt, hels):
    # serial emulation of the team executor (every step for all lanes, then the
    # next step) with the same device routines as the GPU
    h = harness.build(name, opt)
    mom = rambo.generate(npar, nevt, 6)
    hels = list(range(2 ** npar)) if hels is None else list(hels)
    meh = h.team_eval(mom, math.sqrt(4 * math.pi * AS), 173.0, hels)
    ref = ome.me_helicities(ome.process(npar), mom, AS, hels)
    assert np.max(np.abs(meh - ref) / ref.max(axis=0)) < 1e-12


def test_team_program_slots_and_schedule():
    # every op runs once, after its operands, and no slot is overwritten while live
    from paper_2510_05392_amd.gen import team
    for n in (3, 4):
        p = team.TeamProgram('x', topology.Plan(n))
        step_of = {}
        for si, (cls, batch) in enumerate(p.passes):
            assert 0 < len(batch) <= p.T and len({p.ops[k][0] for k in batch}) == 1
            for k in batch:
                assert k not in step_of
                step_of[k] = si
        assert set(step_of) == set(p.ops)
        for k, si in step_of.items():
            for d in p.deps(k):
                assert d not in step_of or step_of[d] < si
        # live ranges of objects sharing a slot do not overlap
        last = {}
        for k, si in step_of.items():
            for d in p.deps(k):
                last[d] = max(last.get(d, -1), si)
        ranges = {}
        for key, *_ in p.ext:
            ranges[key] = (-1, last.get(key, -1))
        for k, si in step_of.items():
            if p.ops[k][0] != 'AMP':
                ranges[k] = (si, last.get(k, si))
        by_slot = {}
        for k, (a, b) in ranges.items():
            by_slot.setdefault(p.slot[k], []).append((a, b))
        for s, rs in by_slot.items():
            rs.sort()
            for (a0, b0), (a1, b1) in zip(rs, rs[1:]):
                assert a1 > b0, (s, rs)


@pytest.mark.parametrize('name,npar,nevt,opt,hels,parts,remat,chunk', [
    ('gg_ttx', 4, 16, '-O1', None, None, None, 16), ('gg_ttxg', 5, 8, '-O1', None, None, None, 8),
    ('gg_ttxgg', 6, 4, '-O1', None, None, None, 16), ('gg_ttxgg', 6, 4, '-O1', None, 3, None, 32),
    ('gg_ttxgg', 6, 4, '-O1', None, None, True, 8),
    ('gg_ttxggg', 7, 2, '-O0', (0, 17, 64, 100, 127), None, None, 16),
    ('gg_ttxggg', 7, 1, '-O0', (3, 99), None, None, 8), ('gg_ttxggg', 7, 1, '-O0', (5, 77), None, None, 32)])
def test_split_evaluation_on_host_vs_oracle(name, npar, nevt, opt, hels, parts, remat, chunk):
    # colour-group sums stored per row (by the group-sum parts in turn, with momentum
    # sums kept or recomputed at each use), then the flows formed from them chunk by
    # chunk, compiled for the host
    h = harness.build(name, opt, sums_parts=parts, remat=remat)
    mom = rambo.generate(npar, nevt, 7)
    hels = list(range(2 ** npar)) if hels is None else list(hels)
    meh = h.split_eval(mom, math.sqrt(4 * math.pi * AS), 173.0, hels, chunk)
    ref = ome.me_helicities(ome.process(npar), mom, AS, hels)
    assert np.max(np.abs(meh - ref) / ref.max(axis=0)) < 1e-12


@pytest.mark.parametrize('n', [3, 4, 5])
def test_split_group_order_is_a_permutation(n):
    # the split executor's group order only reorders the scheduled groups
    plan = topology.Plan(n)
    a, b = plan.scheduled_groups(), plan.split_groups()
    assert len(a) == len(b)
    assert sorted(map(repr, a)) == sorted(map(repr, b))


@pytest.mark.parametrize('name,npar,nevt,hels', [('gg_ttx', 4, 9, None), ('gg_ttxg', 5, 31, None),
                                                 ('gg_ttxgg', 6, 7, [0, 5, 22, 41, 63])])
def test_sde_channel_sums_on_host_vs_oracle(name, npar, nevt, hels):
    """Generated single-diagram-enhancement sums (host build) against the oracle's
    channel amplitudes: same channel numbering (keys from independent
    enumerations), per helicity |A_chan|^2 and the sum over all channels."""
    from oracle import sde as osde
    from paper_2510_05392_amd.gen import codegen
    proc = ome.process(npar)
    _, okeys = osde.channels(proc)
    plan = topology.Plan(npar - 2)
    chan = codegen.channels(plan)
    gkeys = sorted(tuple(codegen.tree_key(plan.trees, t) for t in plan.pieces[i]) for i in chan)
    assert gkeys == [tuple(k) for k in okeys]
    h = harness.build_sde(name)
    assert h.nchan == len(okeys)
    mom = rambo.generate(npar, nevt, 4242)
    ids = (np.arange(nevt) % h.nchan) + 1
    ids[-1] = 0                                     # no channel: numerator zero
    hels = list(range(2 ** npar)) if hels is None else hels
    g = math.sqrt(4 * math.pi * AS)
    num, den = h.eval(mom, g, 173.0, hels, ids)
    for k, hel in enumerate(hels):
        ref = osde.channel_amp2(proc, mom, AS, hels=[hel])      # [nchan, nevt]
        rden = ref.sum(axis=0)
        scale = np.maximum(rden, 1e-300)
        assert np.max(np.abs(den[k] - rden) / scale) < 1e-12
        rnum = np.where(ids > 0, ref[np.maximum(ids, 1) - 1, np.arange(nevt)], 0.0)
        assert np.max(np.abs(num[k] - rnum) / scale) < 1e-12


@pytest.mark.parametrize('name,npar,nevt,hels', [('gg_ttx', 4, 16, None), ('gg_ttxg', 5, 8, None),
                                                 ('gg_ttxgg', 6, 4, None), ('gg_ttxggg', 7, 2, (0, 17, 64, 100, 127)),
                                                 ('gg_ttxgggg', 8, 1, (0, 77, 255))])
def test_berends_giele_on_host_vs_oracle_and_lane_code(name, npar, nevt, hels):
    """The Berends-Giele executor's device functions (host build, one row at a time,
    every level in turn): per-helicity colour sums against the oracle, and its dual
    amplitudes identical (to rounding) to the one-lane diagram code's, flow by flow:
    the recursion reaches the same colour-ordered amplitudes, not only the same |M|^2."""
    h = harness.build_bg()
    mom = rambo.generate(npar, nevt, 8)
    proc = ome.process(npar)
    hels = list(range(2 ** npar)) if hels is None else list(hels)
    g = math.sqrt(4 * math.pi * AS)
    jb = h.jamps(npar - 2, mom, g, 173.0, hels)
    cf = np.asarray(proc.cf)
    meh = np.einsum('hei,ij,hej->he', jb.conj(), cf, jb).real
    ref = ome.me_helicities(proc, mom, AS, hels)
    assert np.max(np.abs(meh - ref) / ref.max(axis=0)) < 1e-12
    if npar <= 7:
        lane = harness.build(name, '-O1' if npar < 7 else '-O0')
        _, jl = lane.eval(mom, g, 173.0, hels, want_jamps=True)
        scale = np.abs(jl).max(axis=(0, 2))
        assert np.max(np.abs(jb - jl).max(axis=(0, 2)) / scale) < 1e-12


@pytest.mark.parametrize('npar,nevt,hels', [(6, 3, None), (7, 1, None), (7, 2, (0, 5, 64, 100, 127))])
def test_helicity_recycling_on_host_vs_row_kernel_and_oracle(npar, nevt, hels):
    """The helicity-recycling kernel's work (host build: set-up, stored currents and
    row spinors per helicity variant, then every rotation-cycle item) gives the same
    dual amplitudes as the row kernel, flow by flow and helicity by helicity, also
    when only some helicities are good; per-helicity colour sums against the oracle
    on a few helicities."""
    h = harness.build_bg()
    mom = rambo.generate(npar, nevt, 8)
    hl = list(range(2 ** npar)) if hels is None else list(hels)
    g = math.sqrt(4 * math.pi * AS)
    rec = h.jamps_recycled(npar - 2, mom, g, 173.0, hl)
    row = h.jamps(npar - 2, mom, g, 173.0, hl)
    scale = np.abs(row).max(axis=(0, 2))
    assert np.max(np.abs(rec - row).max(axis=(0, 2)) / scale) < 1e-13
    pick = [0, len(hl) // 3, len(hl) - 1]
    proc = ome.process(npar)
    cf = np.asarray(proc.cf)
    meh = np.einsum('hei,ij,hej->he', rec[pick].conj(), cf, rec[pick]).real
    ref = ome.me_helicities(proc, mom, AS, [hl[k] for k in pick])
    assert np.max(np.abs(meh - ref) / ref.max(axis=0)) < 1e-12


@pytest.mark.parametrize('n', [4, 5])
def test_helicity_recycling_flops_equal_the_counted_operations(n):
    """flops.bgh_event (building-block counts over the recycling kernel's levels and
    cycle items) equals the operations its device functions perform for one event,
    counted on the host with the operation-counting scalar, part by part; the six
    spinor evaluations of the set-up take one more operation each for a quark with
    pz < 0."""
    count = harness.build_count_bg()
    f = flops.bgh_event(n)
    mom = rambo.generate(n + 2, 3, 1003)
    for e in range(mom.shape[0]):
        neg = int((mom[e, 2:4, 3] < 0).sum())
        setup, currents, rows, items = count(n, mom[e])
        assert setup == f['setup'] + 6 * neg
        assert (currents, rows, items) == (f['currents'], f['rows'], f['items'])


@pytest.mark.parametrize('n', [2, 3, 4, 5, 6])
def test_berends_giele_flops_equal_the_counted_operations(n):
    """The Berends-Giele figures of the roofline (flops.bg_row: building-block counts
    summed over the recursion's levels) equal the operations its device functions
    perform, counted on the host with the operation-counting scalar, part by part."""
    count = harness.build_count_bg()
    f = flops.bg_row(n)
    mom = rambo.generate(n + 2, 4, 1003)
    for e in range(mom.shape[0]):
        neg = int((mom[e, 2:4, 3] < 0).sum())
        for hel in (0, 5, 2 ** (n + 2) - 1):
            setup, currents, rows, amps = count(n, mom[e], hel)
            assert setup == f['setup'] + neg
            assert (currents, rows, amps) == (f['currents'], f['rows'], f['amplitudes'])
