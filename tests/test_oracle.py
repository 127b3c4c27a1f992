"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test targets a different part of the oracle so that a plausible mistake
(a dropped term, a wrong sign or index, a transposed operand) fails one of
them:
  counts          diagram enumeration (the paper's complexity table)
  colour matrix   exact Fierz reduction vs Gell-Mann sums, closed identities
  closed form     whole chain at k = 0 (states, vertices, colour, averaging)
  brute colour    colour reduction + colour matrix vs explicit colour sums
  Berends-Giele   diagram enumeration + colour coefficients vs recursion
  Ward identity   relative normalisation of tt~g, ggg and gggg vertices
  completeness    polarisation sums of the external gluons
  invariances     Lorentz, Bose, charge conjugation, parity, scaling
  spinors         Dirac equation, normalisation and completeness
"""
import itertools
import math

import numpy as np
import pytest

from oracle import bg, brute_colour, closed_form, colour, diagrams, me
from oracle.kinematics import (GAMMA, bar, helicities, mdot, polarisation, slash,
                               u_spinor, v_spinor)
from paper_2510_05392_amd import rambo

AS = 0.118
MT = 173.0


# --- enumeration -------------------------------------------------------------

@pytest.mark.parametrize("n,ndiag,ncubic", [(2, 3, 3), (3, 16, 15), (4, 123, 105),
                                            (5, 1240, 945), (6, 15495, 10395)])
def test_diagram_counts(n, ndiag, ncubic):
    # complexity table of the paper: 3/16/123/1240/15495 diagrams; the
    # diagrams with only 3-point vertices number (2 npar - 5)!!
    assert diagrams.count_diagrams(n) == ndiag
    assert diagrams.count_cubic_diagrams(n) == ncubic
    npar = n + 2
    assert ncubic == math.prod(range(2 * npar - 5, 0, -2))


def test_colour_coefficients_are_units():
    for n in (2, 3, 4):
        for piece in diagrams.diagram_pieces(n):
            for w, c in diagrams.piece_colour(piece).items():
                assert sorted(w) == list(range(n))
                assert c in (1, -1, 1j, -1j)


# --- normalisation -------------------------------------------------------------

@pytest.mark.parametrize("npar,expect", [(4, 256), (5, 256), (6, 512), (7, 1536), (8, 6144)])
def test_iden_average_and_symmetry_factor(npar, expect):
    """IDEN = (initial helicity states) x (initial colour states) x (symmetry
    factor of identical final-state particles), reading of the normalisation
    (the paper leaves it implicit in its ME engine).  The values are the
    convention's (4 * 64 * k!), and the symmetry factor is recounted here by
    brute force: the permutations of the final-state species list
    (t, tbar, g, ..., g) that leave it unchanged.

    Mutation caught: dropping the k! factor in ``colour.iden`` (every k >= 2
    fails), or averaging over the final instead of the initial states."""
    k = npar - 4
    final = ('t', 'tbar') + ('g',) * k
    sym = sum(1 for perm in itertools.permutations(range(len(final)))
              if tuple(final[i] for i in perm) == final)
    initial_hel = 2 * 2                      # two gluons, two helicities each
    initial_col = 8 * 8                      # two gluons, eight colours each
    assert initial_hel * initial_col * sym == expect
    assert colour.iden(npar) == expect
    assert me.process(npar).iden == expect


# --- colour matrix -----------------------------------------------------------

def test_colour_matrix_two_gluons_exact():
    from fractions import Fraction as F
    assert colour.colour_matrix(2) == [[F(16, 3), F(-2, 3)], [F(-2, 3), F(16, 3)]]


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_colour_matrix_identities(n):
    cf = colour.colour_matrix(n)
    m = len(cf)
    assert m == math.factorial(n)
    from fractions import Fraction as F
    for i in range(m):
        assert cf[i][i] == 3 * F(4, 3) ** n            # N C_F^n
        for j in range(m):
            assert cf[i][j] == cf[j][i]
    a = np.array([[float(x) for x in r] for r in cf])
    assert np.linalg.eigvalsh(a).min() > -1e-9             # Gram matrix
    # relabelling the gluons permutes rows and columns together
    basis = colour.colour_basis(n)
    index = {p: i for i, p in enumerate(basis)}
    rng = np.random.default_rng(n)
    for _ in range(3):
        pi = rng.permutation(n)
        perm = [index[tuple(pi[x] for x in p)] for p in basis]
        assert np.array_equal(a[np.ix_(perm, perm)], a)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_colour_matrix_vs_gell_mann(n):
    a = colour.colour_matrix_float(n)
    b = colour.gell_mann_colour_matrix(n)
    assert np.allclose(a, b, rtol=0, atol=1e-12)


def test_structure_constants():
    f = colour.structure_constants()
    assert abs(f[0, 1, 2] - 1.0) < 1e-14                  # f^{123} = 1
    assert abs(f[3, 4, 7] - math.sqrt(3) / 2) < 1e-14     # f^{458} = sqrt(3)/2
    assert np.allclose(f, -np.transpose(f, (1, 0, 2)))


# --- external states ---------------------------------------------------------

def _rand_momenta(n, m, seed):
    rng = np.random.default_rng(seed)
    p3 = rng.normal(size=(n, 3)) * 300
    e = np.sqrt(m * m + (p3 ** 2).sum(axis=1))
    return np.concatenate([e[:, None], p3], axis=1)


def test_spinors_dirac_equation_and_normalisation():
    p = _rand_momenta(16, MT, 1)
    ps = slash(p)
    one = np.eye(4)
    for lam in (1, -1):
        u = u_spinor(p, lam, MT)
        v = v_spinor(p, lam, MT)
        assert np.allclose(np.einsum('eab,eb->ea', ps - MT * one, u), 0, atol=1e-9)
        assert np.allclose(np.einsum('eab,eb->ea', ps + MT * one, v), 0, atol=1e-9)
        assert np.allclose(np.einsum('ea,ea->e', bar(u), u), 2 * MT)
        assert np.allclose(np.einsum('ea,ea->e', bar(v), v), -2 * MT)
    uu = sum(np.einsum('ea,eb->eab', u_spinor(p, l, MT), bar(u_spinor(p, l, MT))) for l in (1, -1))
    vv = sum(np.einsum('ea,eb->eab', v_spinor(p, l, MT), bar(v_spinor(p, l, MT))) for l in (1, -1))
    assert np.allclose(uu, ps + MT * one, atol=1e-9)
    assert np.allclose(vv, ps - MT * one, atol=1e-9)


def test_spinors_are_helicity_eigenstates():
    p = _rand_momenta(8, MT, 2)
    pabs = np.sqrt((p[:, 1:] ** 2).sum(axis=1))
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    z = np.zeros((2, 2))
    spin = [np.block([[s, z], [z, s]]) for s in pauli]            # Sigma^i = diag(sigma^i, sigma^i)
    hop = sum(np.einsum('e,ab->eab', p[:, 1 + i] / pabs, s) for i, s in enumerate(spin))
    for lam in (1, -1):
        u = u_spinor(p, lam, MT)
        v = v_spinor(p, lam, MT)
        assert np.allclose(np.einsum('eab,eb->ea', hop, u), lam * u, atol=1e-9)
        # an antiparticle of helicity lam has spinor spin -lam
        assert np.allclose(np.einsum('eab,eb->ea', hop, v), -lam * v, atol=1e-9)


def test_polarisation_vectors():
    k = _rand_momenta(16, 0.0, 3)
    k = np.concatenate([k, [[5.0, 0, 0, 5.0], [5.0, 0, 0, -5.0]]])
    for lam in (1, -1):
        e = polarisation(k, lam)
        assert np.allclose(mdot(e, k), 0, atol=1e-9)
        assert np.allclose(mdot(e, np.conj(e)), -1)
        assert np.allclose(mdot(e, e), 0, atol=1e-12)
    assert np.allclose(mdot(polarisation(k, 1), np.conj(polarisation(k, -1))), 0, atol=1e-12)
    # k along +z: eps(+) = (0, -1, -i, 0)/sqrt(2)
    assert np.allclose(polarisation(np.array([[1.0, 0, 0, 1.0]]), 1)[0],
                       np.array([0, -1, -1j, 0]) / math.sqrt(2))


# --- the whole chain -----------------------------------------------------------

def test_closed_form_gg_ttx():
    mom = rambo.generate(4, 512, 1001)
    a = me.matrix_element(me.process(4), mom, AS)
    b = closed_form.gg_ttx(mom, AS, MT)
    assert np.max(np.abs(a / b - 1)) < 1e-13


def test_closed_form_limits():
    # threshold (beta -> 0, t1 = t2 = 1/2, rho = 1): 7/48 g^4
    s = (2 * MT) ** 2 * (1 + 1e-12)
    e = math.sqrt(s) / 2
    mom = np.array([[[e, 0, 0, e], [e, 0, 0, -e], [e, 0, 0, 0], [e, 0, 0, 0]]])
    g4 = (4 * math.pi * AS) ** 2
    assert abs(closed_form.gg_ttx(mom, AS, MT)[0] / (7 * g4 / 48) - 1) < 1e-9


@pytest.mark.parametrize("npar,nevt", [(4, 16), (5, 6), (6, 2)])
def test_brute_force_colour(npar, nevt):
    mom = rambo.generate(npar, nevt, 11)
    proc = me.process(npar)
    a = me.matrix_element(proc, mom, AS)
    b = brute_colour.matrix_element(proc, mom, AS)
    assert np.max(np.abs(a / b - 1)) < 1e-13


@pytest.mark.parametrize("npar,nevt,hels", [(4, 16, None), (5, 8, None), (6, 4, None),
                                             (7, 2, (0, 37, 77, 127))])
def test_berends_giele(npar, nevt, hels):
    mom = rambo.generate(npar, nevt, 21)
    proc = me.process(npar)
    hels = range(proc.nhel) if hels is None else hels
    a = np.stack([me.jamps(proc, mom, h, AS) for h in hels])
    b = np.stack([bg.jamps(npar, mom, h, AS) for h in hels])
    scale = np.abs(a).max(axis=(0, 2))                    # per event
    assert np.max(np.abs(a - b).max(axis=(0, 2)) / scale) < 1e-12


@pytest.mark.parametrize("npar,nevt", [(4, 8), (5, 8), (6, 4), (7, 2)])
def test_ward_identity(npar, nevt):
    mom = rambo.generate(npar, nevt, 31)
    proc = me.process(npar)
    hels = (0, 3, proc.nhel // 2 + 1, proc.nhel - 1)
    for h in hels:
        ref = np.abs(me.jamps(proc, mom, h, AS)).max(axis=1)
        ref = np.maximum(ref, np.abs(me.jamps(proc, mom, proc.nhel - 1 - h, AS)).max(axis=1))
        for slot in range(npar - 2):
            w = np.abs(me.jamps(proc, mom, h, AS, ward_slot=slot)).max(axis=1)
            assert np.all(w <= 1e-12 * ref)


@pytest.mark.parametrize("npar", [5, 6])
def test_polarisation_completeness(npar):
    # sum_l |M(eps_l)|^2 = -g^{mu nu} M_mu M_nu^*  for one gluon at a time
    mom = rambo.generate(npar, 3, 41)
    proc = me.process(npar)
    h = 5
    hel = helicities(npar, h)
    for slot in (0, npar - 3):
        q = me.slot_particle(slot)
        comps = []
        for mu in range(4):
            e = np.zeros((3, 4), dtype=complex)
            e[:, mu] = 1.0
            comps.append(me.jamps(proc, mom, h, AS, override=(slot, e)))
        x = np.stack(comps, axis=-1)                        # X_mu per colour
        lhs = 0.0
        for lam in (1, -1):
            eps = polarisation(mom[:, q], lam)
            fac = eps if slot < 2 else np.conj(eps)
            lhs = lhs + np.abs(np.einsum('em,esm->es', fac, x)) ** 2
        rhs = -(np.abs(x[..., 0]) ** 2 - (np.abs(x[..., 1:]) ** 2).sum(axis=-1))
        assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-12 * np.abs(lhs).max())


def _boost(mom, beta):
    b2 = (beta ** 2).sum()
    g = 1 / math.sqrt(1 - b2)
    out = mom.copy()
    bp = (mom[..., 1:] * beta).sum(axis=-1)
    out[..., 0] = g * (mom[..., 0] + bp)
    out[..., 1:] = mom[..., 1:] + ((g - 1) * bp / b2 + g * mom[..., 0])[..., None] * beta
    return out


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


@pytest.mark.parametrize("npar,nevt", [(4, 16), (5, 8), (6, 4), (7, 1)])
def test_lorentz_invariance(npar, nevt):
    mom = rambo.generate(npar, nevt, 51)
    proc = me.process(npar)
    base = me.matrix_element(proc, mom, AS)
    boosted = _boost(mom, np.array([0.3, -0.5, 0.6]))
    assert np.max(np.abs(me.matrix_element(proc, boosted, AS) / base - 1)) < 1e-12
    # per-helicity sums are rotation invariant
    rot = mom.copy()
    rot[..., 1:] = mom[..., 1:] @ _rotation(npar).T
    hels = range(proc.nhel) if npar < 7 else (0, 5, 100)
    a = me.me_helicities(proc, mom, AS, hels)
    b = me.me_helicities(proc, rot, AS, hels)
    assert np.all(np.abs(a - b) <= 1e-12 * np.abs(a).max(axis=0))


@pytest.mark.parametrize("npar,nevt", [(5, 8), (6, 4)])
def test_bose_and_charge_conjugation(npar, nevt):
    mom = rambo.generate(npar, nevt, 61)
    proc = me.process(npar)
    base = me.matrix_element(proc, mom, AS)
    sw = mom[:, [1, 0] + list(range(2, npar))]                      # p1 <-> p2
    assert np.max(np.abs(me.matrix_element(proc, sw, AS) / base - 1)) < 1e-12
    perm = list(range(4)) + list(reversed(range(4, npar)))          # final gluons
    assert np.max(np.abs(me.matrix_element(proc, mom[:, perm], AS) / base - 1)) < 1e-12
    cc = mom[:, [0, 1, 3, 2] + list(range(4, npar))]                # t <-> tbar
    assert np.max(np.abs(me.matrix_element(proc, cc, AS) / base - 1)) < 1e-12


@pytest.mark.parametrize("npar,nevt", [(4, 8), (5, 4), (6, 2)])
def test_parity(npar, nevt):
    mom = rambo.generate(npar, nevt, 71)
    proc = me.process(npar)
    pm = mom.copy()
    pm[..., 1:] *= -1
    a = me.me_helicities(proc, mom, AS)
    b = me.me_helicities(proc, pm, AS)[::-1]                       # all helicities flipped
    assert np.all(np.abs(a - b) <= 1e-12 * np.abs(a).max(axis=0))


@pytest.mark.parametrize("npar", [4, 5, 6])
def test_scaling(npar):
    mom = rambo.generate(npar, 4, 81)
    proc = me.process(npar)
    base = me.matrix_element(proc, mom, AS)
    assert np.allclose(me.matrix_element(proc, mom, 0.2) / base, (0.2 / AS) ** (npar - 2), rtol=1e-12)
    proc2 = me.Process(npar, mt=2 * MT)
    scaled = me.matrix_element(proc2, 2 * mom, AS)
    assert np.allclose(scaled / base, 2.0 ** (2 * (4 - npar)), rtol=1e-12)


@pytest.mark.parametrize("npar", [4, 5, 6])
def test_good_helicities(npar):
    # g g -> t tbar: equal gluon helicities (J_z = 0 along the beam) only
    # produce equal t, tbar helicities, so exactly four combinations vanish
    # identically; from one extra gluon on every combination contributes.
    mom = rambo.generate(npar, 16, 91)
    proc = me.process(npar)
    mh = me.me_helicities(proc, mom, AS)
    frac = (mh / mh.sum(axis=0)).max(axis=1)
    dead = set(np.where(frac < 1e-14)[0].tolist())
    if npar == 4:
        assert dead == {0b0001, 0b0010, 0b1101, 0b1110}
        assert max(frac[list(dead)]) < 1e-28
    else:
        assert not dead


# --- phase space inputs --------------------------------------------------------

@pytest.mark.parametrize("npar", [4, 5, 7])
def test_rambo_kinematics(npar):
    mom = rambo.generate(npar, 256, 5)
    tot = mom[:, 2:].sum(axis=1)
    assert np.allclose(tot, [1500.0, 0, 0, 0], atol=1e-9)
    m2 = mom[..., 0] ** 2 - (mom[..., 1:] ** 2).sum(axis=-1)
    masses = np.array([0, 0, MT, MT] + [0] * (npar - 4))
    assert np.allclose(m2, masses ** 2, atol=1e-6)


def test_rambo_massless_weight_is_volume():
    # massless n-body volume (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)!(n-2)!)
    mom, w = rambo.generate(5, 8, 3, mt=0.0, return_weights=True)
    n, s = 3, 1500.0 ** 2
    vol = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (2 * 1)
    assert np.allclose(w, vol)
    # two-body massive: weight = beta / (8 pi) for RAMBO's normalisation
    mom, w = rambo.generate(4, 4, 3, return_weights=True)
    beta = math.sqrt(1 - 4 * MT * MT / s)
    assert np.allclose(w, beta / (8 * math.pi))


def test_extended_precision_mode():
    # the oracle run on np.longdouble inputs works in extended precision
    # throughout: on two-body points built exactly in long double it meets the
    # closed form far below FP64 rounding
    rng = np.random.default_rng(7)
    n = 16
    ld = np.longdouble
    e = ld(750)
    pabs = np.sqrt(e * e - ld(MT) * ld(MT))
    ct = rng.uniform(-1, 1, n).astype(ld)
    st = np.sqrt(1 - ct * ct)
    ph = rng.uniform(0, 2 * np.pi, n).astype(ld)
    p3 = np.stack([np.full(n, e), pabs * st * np.cos(ph), pabs * st * np.sin(ph), pabs * ct], axis=1)
    p4 = p3.copy()
    p4[:, 1:] *= -1
    beam = np.zeros((n, 4), dtype=ld)
    b1, b2 = beam.copy(), beam.copy()
    b1[:, 0] = b1[:, 3] = e
    b2[:, 0] = e
    b2[:, 3] = -e
    mom = np.stack([b1, b2, p3, p4], axis=1)
    a = me.matrix_element(me.process(4), mom, AS)
    b = closed_form.gg_ttx(mom, AS, MT)
    assert a.dtype == np.longdouble
    assert np.max(np.abs(a / b - 1)) < 1e-17
    c = me.matrix_element(me.process(4), mom.astype(np.float64), AS)
    assert np.max(np.abs(c / a.astype(np.float64) - 1)) < 1e-13


def test_rotation_invariance_on_the_stored_ggttgggg_set():
    """The stored oracle values of the first 1024 g g -> t t~ g g g g events of the
    32768-event workload against the oracle's values on a random rotation of each
    (tests/golden/make_golden.py wide_c4a, wide_c4a_rot): the helicity-summed |M|^2 is
    rotation invariant, so the two agree to FP64 rounding (a wrong rotation, or an
    oracle term that is not a Lorentz scalar, would put them far apart)."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden')
    spec = importlib.util.spec_from_file_location('make_golden', os.path.join(here, 'make_golden.py'))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    # the rotation keeps energies and every invariant p_i . p_j
    mom = rambo.generate(8, 16, 1005)
    rot = mg._rotate(mom, 4242)
    assert np.array_equal(rot[..., 0], mom[..., 0])
    for i in range(8):
        for j in range(8):
            assert np.allclose(mdot(rot[:, i], rot[:, j]), mdot(mom[:, i], mom[:, j]), rtol=1e-12, atol=1e-9)
    assert np.max(np.abs(rot[..., 1:] - mom[..., 1:])) > 1.0
    g = np.load(os.path.join(here, 'gg_ttxgggg_seed1005_first1024.npz'))['me']
    r = np.load(os.path.join(here, 'gg_ttxgggg_seed1005_first1024_rot.npz'))['me_rot']
    d = np.abs(r / g - 1)
    assert len(g) == len(r) == 1024
    assert np.median(d) < 1e-13 and np.mean(d < 1e-13) > 0.9 and d.max() < 5e-11
