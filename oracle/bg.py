"""Colour-ordered Berends-Giele recursion (oracle cross-check).

An algorithm independent of diagram enumeration for the dual amplitudes: the
paper names Berends-Giele recursion as the better-scaling alternative for
many gluons (discussion section).  The colour-ordered vertices follow from
the same Feynman rules as the diagram oracle, by taking the coefficient of
one ordering of T's (f^{abc} T^a = -i[T^b, T^c]):

  quark-gluon            i g gamma^mu
  ggg (children A, B)    -i g [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
                         with k = -(P_A+P_B), p = P_A, q = P_B
  gggg (children A,B,C)  -i g^2 [J_A^mu (J_B.J_C) - 2 J_B^mu (J_A.J_C) + J_C^mu (J_A.J_B)]

Off-shell gluon currents of ordered gluon sets are built recursively,
    J(1..k) = (-i/P^2) [ sum_j V3(J(1..j), J(j+1..k))
                         + sum_{j<l} V4(J(1..j), J(j+1..l), J(l+1..k)) ],
and the quark line absorbs ordered blocks from the top end.  The amplitude
for ordering sigma is the coefficient of (T^{a_s1} ... T^{a_sn})_{i j} in
the full amplitude, i.e. the dual amplitude J_sigma of the diagram oracle.
"""
from __future__ import annotations

import numpy as np

from .kinematics import helicities, mdot, slash
from .me import coupling, gluon_states, quark_propagator, quark_states


def _v3(ja, pa, jb, pb, g):
    k = -(pa + pb)
    v = (ja * mdot(k - pa, jb)[:, None] + mdot(ja, jb)[:, None] * (pa - pb)
         + jb * mdot(pb - k, ja)[:, None])
    return -1j * g * v


def _v4(ja, jb, jc, g):
    v = (ja * mdot(jb, jc)[:, None] - 2.0 * jb * mdot(ja, jc)[:, None]
         + jc * mdot(ja, jb)[:, None])
    return -1j * g * g * v


class _BG:
    def __init__(self, mom, hel, mt, g, ward_slot=None):
        self.ext = gluon_states(mom, hel, ward_slot)
        self.ubar3, self.v4 = quark_states(mom, hel, mt)
        self.p3 = mom[:, 2]
        self.mt = mt
        self.g = g
        self.cur = {}
        self.quark = {}

    def current(self, seq):
        if len(seq) == 1:
            return self.ext[seq[0]]
        hit = self.cur.get(seq)
        if hit is not None:
            return hit
        k = len(seq)
        acc = 0.0
        for j in range(1, k):
            ja, pa = self.current(seq[:j])
            jb, pb = self.current(seq[j:])
            acc = acc + _v3(ja, pa, jb, pb, self.g)
        for j in range(1, k - 1):
            for l in range(j + 1, k):
                ja, _ = self.current(seq[:j])
                jb, _ = self.current(seq[j:l])
                jc, _ = self.current(seq[l:])
                acc = acc + _v4(ja, jb, jc, self.g)
        p = sum(self.ext[s][1] for s in seq)
        res = ((-1j / mdot(p, p))[:, None] * acc, p)
        self.cur[seq] = res
        return res

    def row(self, seq):
        """Top-line row spinor having absorbed the ordered gluons `seq` (with propagator)."""
        if not seq:
            return self.ubar3
        hit = self.quark.get(seq)
        if hit is not None:
            return hit
        q = self.p3 - sum(self.ext[s][1] for s in seq)
        acc = 0.0
        for i in range(len(seq)):
            j, _ = self.current(seq[i:])
            acc = acc + np.einsum('ea,eab->eb', self.row(seq[:i]), 1j * self.g * slash(j))
        r = np.einsum('ea,eab->eb', acc, quark_propagator(q, self.mt))
        self.quark[seq] = r
        return r

    def amplitude(self, seq):
        acc = 0.0
        for i in range(len(seq)):
            j, _ = self.current(seq[i:])
            acc = acc + np.einsum('ea,eab->eb', self.row(seq[:i]), 1j * self.g * slash(j))
        return np.einsum('ea,ea->e', acc, self.v4)


def jamps(npar, mom, h, alpha_s, mt=173.0, basis=None, ward_slot=None):
    """Colour-ordered amplitudes for every ordering in `basis` (default: all, lexicographic)."""
    import itertools
    mom = np.asarray(mom)
    if mom.dtype != np.longdouble:
        mom = mom.astype(np.float64)
    n = npar - 2
    basis = list(itertools.permutations(range(n))) if basis is None else basis
    bg = _BG(mom, helicities(npar, h), mt, coupling(alpha_s, mom.dtype), ward_slot)
    return np.stack([bg.amplitude(tuple(s)) for s in basis], axis=1)
