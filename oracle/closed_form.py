"""Analytic spin- and colour-averaged |M|^2 for g g -> Q Qbar (oracle pin).

Textbook heavy-quark pair production result (Ellis, Stirling & Webber,
"QCD and Collider Physics", heavy-quark chapter; Combridge 1979):

    <|M|^2> = g^4 (1/(6 t1 t2) - 3/8) (t1^2 + t2^2 + rho - rho^2 / (4 t1 t2)),

with t1 = 2 p1.p3 / s, t2 = 2 p2.p3 / s, rho = 4 m^2 / s.  It already
includes the 1/4 spin and 1/64 colour averages of the incoming gluons.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(axis=-1)


def gg_ttx(mom, alpha_s, mt):
    mom = np.asarray(mom)
    if mom.dtype != np.longdouble:
        mom = mom.astype(np.float64)
    p1, p2, p3 = mom[:, 0], mom[:, 1], mom[:, 2]
    s = _dot(p1 + p2, p1 + p2)
    t1 = 2.0 * _dot(p1, p3) / s
    t2 = 2.0 * _dot(p2, p3) / s
    rho = 4.0 * mt * mt / s
    pi = np.arccos(np.asarray(-1.0, dtype=mom.dtype))
    g4 = (4 * pi * np.asarray(alpha_s, dtype=mom.dtype)) ** 2
    return g4 * (1 / (6 * t1 * t2) - np.asarray(0.375, dtype=mom.dtype)) * (
        t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))
