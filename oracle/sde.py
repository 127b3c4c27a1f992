"""Single-diagram-enhancement (SDE) channel weights (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's matrix-element engine also takes an event-by-event channel
identifier for MadEvent's single-diagram-enhanced multichannel integration,
which yields extra outputs (section "a closer look at the internals of the ME
engine"); its complexity table counts the SDE channels of each process
(3, 15, 105, 945 for k = 0..3): the diagrams built from three-point vertices
only.  The multichannel method (Maltoni and Stelzer, JHEP 02 (2003) 027)
weights channel c at phase-space point p by

    alpha_c(p) = |A_c(p)|^2 / sum_{d in channels} |A_d(p)|^2,

where A_d is the colour-stripped amplitude of diagram d and both sums run over
the good helicities.  This module returns the numerator and the denominator.

Readings (the paper gives neither):
  * A_d is the Lorentz amplitude whose colour coefficients on the quark-line
    strings are units (+-1, +-i), i.e. the piece amplitude of the diagram
    module; only |A_d|^2 enters, so phase conventions do not matter, but the
    gauge of the external gluons does: polarisations are spatial and
    transverse (the helicity states of the kinematics module).
  * Channel numbering: the channels are the diagrams with three-point vertices
    only, numbered 1..N in ascending order of a canonical key (0 = no channel).
    The key of a diagram is the tuple, from the top end of the quark line to
    the antitop end, of its gluon trees written as strings: a leaf is its
    gluon slot number, a three-gluon vertex is "(" + its two children's
    strings, sorted, joined by "," + ")".  Any numbering works for the method;
    this one is fixed so that two independent enumerations agree.
"""
from __future__ import annotations

import numpy as np

from . import me as _me


def _is_cubic(tree):
    if isinstance(tree, int):
        return True
    return tree[0] == '3' and _is_cubic(tree[1]) and _is_cubic(tree[2])


def tree_key(tree):
    """Canonical string of a three-vertex gluon tree (see the module docstring)."""
    if isinstance(tree, int):
        return str(tree)
    return '(' + ','.join(sorted((tree_key(tree[1]), tree_key(tree[2])))) + ')'


def channels(proc):
    """(piece indices of the channels in channel order, their keys)."""
    cubic = [(tuple(tree_key(t) for t in piece), i)
             for i, piece in enumerate(proc.pieces) if all(_is_cubic(t) for t in piece)]
    cubic.sort()
    return [i for _, i in cubic], [k for k, _ in cubic]


def channel_amp2(proc, mom, alpha_s, hels=None):
    """sum_h |A_c(h)|^2 for every channel c (in channel order): [nchan, nevt]."""
    idx, _ = channels(proc)
    hels = range(proc.nhel) if hels is None else hels
    mom = np.asarray(mom)
    out = np.zeros((len(idx), mom.shape[0]), dtype=np.float64 if mom.dtype != np.longdouble
                   else np.longdouble)
    for h in hels:
        amps = _me.piece_amplitudes(proc, mom, h, alpha_s)
        out += np.abs(amps[idx]) ** 2
    return out


def channel_weights(proc, mom, alpha_s, chan, hels=None):
    """(numerator, denominator) per event for channel ids chan[nevt] in 1..N:
    numerator = sum_h |A_chan|^2, denominator = sum_h sum_c |A_c|^2."""
    a2 = channel_amp2(proc, mom, alpha_s, hels)
    chan = np.asarray(chan)
    num = a2[chan - 1, np.arange(a2.shape[1])]
    return num, a2.sum(axis=0)
