"""Helicity and colour selection for event output (test infrastructure only).

The matrix-element engine of the paper returns, besides |M|^2, one helicity
and one leading colour per event, drawn with two per-event random numbers
from the contributions of the individual helicities and colours (section on
the internals of the ME engine).  The paper does not spell out the rule; the
reading followed here:

  helicity  h drawn with probability ME_h / sum_h' ME_h' over the good
            helicities, by inverting the cumulative sum in ascending helicity
            order: the first h whose running sum exceeds r_hel * total;
  colour    flow c drawn with probability |J_c(h)|^2 / sum_c' |J_c'(h)|^2 for
            the drawn helicity h (the diagonal, always non-negative part of
            the colour sum), by the same rule in the order of the colour basis.

When rounding leaves no running sum above r * total (r close to 1) the last
entry with a positive weight is taken.
"""
from __future__ import annotations

import numpy as np

from . import me as ome


def draw(weights, r):
    """Inverse-CDF draw per event; weights [n][nevt] >= 0, r [nevt] in [0, 1)."""
    weights = np.asarray(weights, dtype=np.float64)
    n, nevt = weights.shape
    out = np.empty(nevt, dtype=np.int64)
    for e in range(nevt):
        w = weights[:, e]
        total = 0.0
        for k in range(n):
            total += w[k]
        t = r[e] * total
        cum, pick, last = 0.0, -1, 0
        for k in range(n):
            cum += w[k]
            if w[k] > 0.0:
                last = k
            if pick < 0 and t < cum:
                pick = k
        out[e] = last if pick < 0 else pick
    return out


def select(proc, mom, alpha_s, r_hel, r_col, good=None):
    """(|M|^2, drawn helicity index, drawn colour-flow index) per event."""
    mom = np.asarray(mom, dtype=np.float64)
    good = list(range(proc.nhel)) if good is None else list(good)
    meh = ome.me_helicities(proc, mom, alpha_s, good)          # [ngood][nevt]
    me2 = meh.sum(axis=0) / proc.iden
    hel = np.asarray(good)[draw(meh, r_hel)]
    col = np.empty(len(mom), dtype=np.int64)
    for h in np.unique(hel):
        idx = np.nonzero(hel == h)[0]
        jam = ome.jamps(proc, mom[idx], int(h), alpha_s)        # [nevt_h][ncol]
        col[idx] = draw((np.abs(jam) ** 2).T, np.asarray(r_col)[idx])
    return me2, hel, col
