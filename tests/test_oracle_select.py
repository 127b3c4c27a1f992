"""Pins of the oracle's helicity / colour selection (CPU only).

The draw must realise the stated probabilities: with stratified random numbers
r_i = (i + 1/2) / N every entry k is drawn N w_k / W times up to one, entries
of zero weight never, and the boundaries follow "first running sum above
r * total".
"""
import numpy as np
import pytest

from oracle import me as ome, select as sel
from paper_2510_05392_amd import rambo

AS = 0.118


def test_draw_boundaries_closed_form():
    w = np.array([[1.0, 1.0, 1.0, 1.0], [0.0, 0.0, 0.0, 0.0], [3.0, 3.0, 3.0, 3.0]])
    r = np.array([0.0, 0.2499999, 0.25, 0.9999999999])
    # total 4: r*4 < 1 -> entry 0; r*4 = 1 is not below the first running sum -> entry 2
    assert list(sel.draw(w, r)) == [0, 0, 2, 2]


def test_draw_last_positive_when_rounding_overshoots():
    w = np.array([[0.1], [0.2], [0.0]])
    # r = 1 is outside [0, 1) but exercises the fallback: no running sum exceeds the total
    assert list(sel.draw(w, np.array([1.0]))) == [1]


def test_stratified_frequencies_match_helicity_weights():
    proc = ome.process(5)
    mom = rambo.generate(5, 1, 77)
    meh = ome.me_helicities(proc, mom, AS)[:, 0]
    n = 20000
    r = (np.arange(n) + 0.5) / n
    picks = sel.draw(np.repeat(meh[:, None], n, axis=1), r)
    counts = np.bincount(picks, minlength=len(meh))
    expect = n * meh / meh.sum()
    assert np.all(np.abs(counts - expect) <= 1.0 + 1e-9)


def test_vanishing_helicities_never_drawn_ggtt():
    # g g -> t tbar: helicities 1, 2, 13, 14 vanish identically (selection rule)
    proc = ome.process(4)
    mom = rambo.generate(4, 400, 78)
    rng = np.random.default_rng(3)
    me2, hel, col = sel.select(proc, mom, AS, rng.random(400), rng.random(400))
    assert not np.isin(hel, [1, 2, 13, 14]).any()
    assert np.allclose(me2, ome.matrix_element(proc, mom, AS), rtol=1e-14)
    assert set(np.unique(col)) <= {0, 1}


def test_colour_draw_follows_flow_weights():
    # one event, one helicity: stratified colour draws reproduce |J_c|^2 / sum |J|^2
    proc = ome.process(5)
    mom = rambo.generate(5, 1, 79)
    jam = ome.jamps(proc, mom, 5, AS)[0]
    w = np.abs(jam) ** 2
    n = 6000
    r = (np.arange(n) + 0.5) / n
    picks = sel.draw(np.repeat(w[:, None], n, axis=1), r)
    counts = np.bincount(picks, minlength=len(w))
    assert np.all(np.abs(counts - n * w / w.sum()) <= 1.0 + 1e-9)


@pytest.mark.parametrize('npar', [4, 5])
def test_select_is_consistent_with_its_parts(npar):
    proc = ome.process(npar)
    mom = rambo.generate(npar, 50, 80 + npar)
    rng = np.random.default_rng(npar)
    rh, rc = rng.random(50), rng.random(50)
    me2, hel, col = sel.select(proc, mom, AS, rh, rc)
    meh = ome.me_helicities(proc, mom, AS)
    assert np.array_equal(hel, sel.draw(meh, rh))
    for e in range(50):
        jam = ome.jamps(proc, mom[e:e + 1], int(hel[e]), AS)[0]
        assert col[e] == sel.draw((np.abs(jam) ** 2)[:, None], rc[e:e + 1])[0]
