"""Pins of the oracle's single-diagram-enhancement channel weights (oracle/sde.py).

  * gg -> t tbar: the spin- and polarisation-summed square of each of the three
    diagrams recomputed by Dirac traces (Dirac representation, spinor
    completeness, transverse polarisation sums), sharing no code with the
    oracle's spinors, polarisations or diagram evaluation;
  * the channel count is the number of three-vertex diagrams, (2 npar - 5)!!;
  * rotations leave every channel's summed |A|^2 unchanged (the polarisation
    sums are spatial and transverse, which rotations preserve);
  * relabelling identical gluons permutes the channels: |A_c|^2 at the
    relabelled momenta equals |A_pi(c)|^2 at the original ones, with pi(c)
    found from the channel keys;
  * the weights of all channels sum to one.
"""
import math

import numpy as np
import pytest

from oracle import me, sde
from paper_2510_05392_amd import rambo

AS = 0.118
MT = 173.0


# --- Dirac algebra written out independently (Dirac representation) ------------

_I2 = np.eye(2)
_SIG = [np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
        np.array([[1, 0], [0, -1]], dtype=complex)]
_G = [np.block([[_I2, 0 * _I2], [0 * _I2, -_I2]]).astype(complex)]
_G += [np.block([[0 * _I2, s], [-s, 0 * _I2]]) for s in _SIG]


def _sl(a):
    """gamma^mu a_mu for a four-vector with upper indices."""
    return _G[0] * a[0] - _G[1] * a[1] - _G[2] * a[2] - _G[3] * a[3]


def _dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def _transverse(k):
    """Two real orthonormal spatial vectors perpendicular to k (zero time part)."""
    kh = k[1:] / np.linalg.norm(k[1:])
    trial = np.array([1.0, 0.0, 0.0]) if abs(kh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    a = trial - kh * (trial @ kh)
    a /= np.linalg.norm(a)
    b = np.cross(kh, a)
    return [np.concatenate([[0.0], a]), np.concatenate([[0.0], b])]


def _ggtt_diagram_squares(p, g):
    """[s, t, u] channel: sum over spins and polarisations of |ubar(p3) Gam v(p4)|^2."""
    k1, k2, p3, p4 = p
    one = np.eye(4)
    s = _dot(k1 + k2, k1 + k2)
    qt, qu = p3 - k1, p3 - k2
    out = np.zeros(3)
    for e1 in _transverse(k1):
        for e2 in _transverse(k2):
            v = _dot(e1, e2) * (k1 - k2) + 2 * _dot(k2, e1) * e2 - 2 * _dot(k1, e2) * e1
            gams = [g * g / s * _sl(v),
                    g * g / (_dot(qt, qt) - MT ** 2) * _sl(e1) @ (_sl(qt) + MT * one) @ _sl(e2),
                    g * g / (_dot(qu, qu) - MT ** 2) * _sl(e2) @ (_sl(qu) + MT * one) @ _sl(e1)]
            for d, gam in enumerate(gams):
                gbar = _G[0] @ gam.conj().T @ _G[0]
                out[d] += np.trace((_sl(p3) + MT * one) @ gam @ (_sl(p4) - MT * one) @ gbar).real
    return out


def test_ggtt_channels_against_dirac_traces():
    """Mutations caught: a channel summed over the wrong helicities, an
    amplitude squared without its propagator, the s and t/u channels numbered
    in another order, or a non-transverse polarisation gauge."""
    proc = me.process(4)
    _, keys = sde.channels(proc)
    assert keys == [('(0,1)',), ('0', '1'), ('1', '0')]
    mom = rambo.generate(4, 6, 77)
    g = math.sqrt(4 * math.pi * AS)
    got = sde.channel_amp2(proc, mom, AS)
    for e in range(mom.shape[0]):
        ref = _ggtt_diagram_squares(mom[e], g)
        assert np.allclose(got[:, e], ref, rtol=1e-12, atol=0), (e, got[:, e], ref)


@pytest.mark.parametrize('npar,nchan', [(4, 3), (5, 15), (6, 105), (7, 945)])
def test_channel_count_is_the_three_vertex_diagrams(npar, nchan):
    idx, keys = sde.channels(me.process(npar))
    assert len(idx) == nchan == math.prod(range(2 * npar - 5, 0, -2))
    assert len(set(keys)) == nchan


def _rotation(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


@pytest.mark.parametrize('npar', [5, 6])
def test_channels_rotation_invariant(npar):
    rng = np.random.default_rng(npar)
    mom = rambo.generate(npar, 3, 500 + npar)
    rot = mom.copy()
    rot[..., 1:] = mom[..., 1:] @ _rotation(rng).T
    proc = me.process(npar)
    a = sde.channel_amp2(proc, mom, AS)
    b = sde.channel_amp2(proc, rot, AS)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * a.max())


def _relabel(tree, perm):
    if isinstance(tree, int):
        return perm[tree]
    return ('3', _relabel(tree[1], perm), _relabel(tree[2], perm))


@pytest.mark.parametrize('swap', [(2, 3), (0, 1)])
def test_channels_permute_under_gluon_relabelling(swap):
    """Mutation caught: a channel key that does not follow the diagram's
    structure (e.g. trees not sorted inside a vertex), which breaks the map."""
    npar = 6
    proc = me.process(npar)
    idx, keys = sde.channels(proc)
    slot_perm = list(range(npar - 2))
    slot_perm[swap[0]], slot_perm[swap[1]] = swap[1], swap[0]
    where = {k: c for c, k in enumerate(keys)}
    image = [where[tuple(sde.tree_key(_relabel(t, slot_perm)) for t in proc.pieces[i])] for i in idx]
    assert sorted(image) == list(range(len(keys)))
    mom = rambo.generate(npar, 3, 4242)
    q = [s if s < 2 else s + 2 for s in swap]          # particles of the swapped slots
    pm = mom.copy()
    pm[:, [q[0], q[1]]] = mom[:, [q[1], q[0]]]
    a = sde.channel_amp2(proc, mom, AS)
    b = sde.channel_amp2(proc, pm, AS)
    assert np.allclose(b[image], a, rtol=1e-10, atol=1e-12 * a.max())


def test_weights_sum_to_one():
    proc = me.process(5)
    mom = rambo.generate(5, 4, 9)
    nchan = len(sde.channels(proc)[0])
    tot = np.zeros(4)
    for c in range(1, nchan + 1):
        num, den = sde.channel_weights(proc, mom, AS, np.full(4, c))
        tot += num / den
    assert np.allclose(tot, 1.0, rtol=1e-13)
