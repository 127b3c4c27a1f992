"""Colour algebra for one quark line and n gluons (oracle).

Colour basis: for n gluons the n! strings (T^{a_s1} ... T^{a_sn})_{i j},
i the colour of the outgoing top and j that of the outgoing antitop, with
the permutations s listed in lexicographic order of the gluon labels.  The
paper's colour matrix ("colormatrix" in the pseudo-code of the monolithic
kernel; C in the colour-sum equation J^H C J) is the Gram matrix of these
strings:

    CF[s, t] = sum_{a, i, j} conj((T^s)_{ij}) (T^t)_{ij}
             = sum_a Tr(T^{a_sn} ... T^{a_s1} T^{a_t1} ... T^{a_tn}).

It is computed exactly (Fractions) by repeated use of the SU(N) Fierz
identity  sum_a T^a_{ij} T^a_{kl} = 1/2 (d_il d_kj - d_ij d_kl / N), N = 3,
in its two trace forms
    Tr(A T^a B T^a)   = 1/2 (Tr A Tr B - Tr(AB)/N)
    Tr(A T^a) Tr(B T^a) = 1/2 (Tr(AB) - Tr A Tr B / N).
The summed gluon labels are dummy indices, so a trace product is memoised
on its pattern of letters (letters renamed in order of first appearance).
An independent numeric check with explicit Gell-Mann matrices lives in
``gell_mann_colour_matrix``.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache

import numpy as np

NC = 3


def colour_basis(n):
    """Lexicographically ordered permutations of gluon slots 0..n-1."""
    return list(itertools.permutations(range(n)))


def _canon(traces):
    """Rename letters by first appearance and sort traces (cyclic-invariant)."""
    # rotate each trace to its lexicographically smallest rotation of the raw
    # letters first so that the product representation is order-independent
    rots = []
    for t in traces:
        if not t:
            rots.append(t)
            continue
        rots.append(min(t[i:] + t[:i] for i in range(len(t))))
    rots.sort(key=lambda t: (len(t), t))
    rename = {}
    out = []
    for t in rots:
        out.append(tuple(rename.setdefault(x, len(rename)) for x in t))
    return tuple(out)


@lru_cache(maxsize=None)
def _eval(traces):
    """Value of a product of traces in which every letter appears exactly twice."""
    # drop empty traces (each is Tr(1) = N)
    factor = Fraction(1)
    live = []
    for t in traces:
        if len(t) == 0:
            factor *= NC
        else:
            live.append(t)
    if not live:
        return factor
    # a single letter alone in a trace: Tr(T^a) = 0
    for t in live:
        if len(t) == 1:
            return Fraction(0)
    letter = live[0][0]
    where = [(ti, pos) for ti, t in enumerate(live) for pos, x in enumerate(t) if x == letter]
    (t1, p1), (t2, p2) = where
    half = Fraction(1, 2)
    if t1 == t2:
        t = live[t1]
        # rotate so the first occurrence is at the end: Tr(A T^a B T^a) with
        # A = letters strictly between, B = the remainder
        a_part = t[p1 + 1:p2]
        b_part = t[p2 + 1:] + t[:p1]
        rest = live[:t1] + live[t1 + 1:]
        r1 = _eval(_canon(rest + [a_part, b_part]))
        r2 = _eval(_canon(rest + [a_part + b_part]))
        return factor * half * (r1 - r2 / NC)
    ta, tb = live[t1], live[t2]
    # Tr(A T^a) Tr(B T^a): rotate each so the letter is last
    a_part = ta[p1 + 1:] + ta[:p1]
    b_part = tb[p2 + 1:] + tb[:p2]
    rest = [t for k, t in enumerate(live) if k not in (t1, t2)]
    r1 = _eval(_canon(rest + [a_part + b_part]))
    r2 = _eval(_canon(rest + [a_part, b_part]))
    return factor * half * (r1 - r2 / NC)


def colour_matrix_entry(s, t):
    """Exact CF[s, t] = Tr(T^{s_n}..T^{s_1} T^{t_1}..T^{t_n})."""
    word = tuple(reversed(s)) + tuple(t)
    return _eval(_canon([word]))


def colour_matrix(n):
    """Exact colour matrix (list of lists of Fractions) for n gluons."""
    basis = colour_basis(n)
    return [[colour_matrix_entry(s, t) for t in basis] for s in basis]


def colour_matrix_float(n):
    cf = colour_matrix(n)
    return np.array([[float(x) for x in row] for row in cf])


# --- explicit SU(3) generators (independent numeric cross-check) -----------

def gell_mann():
    """The eight Gell-Mann matrices lambda^a; T^a = lambda^a / 2."""
    l = np.zeros((8, 3, 3), dtype=complex)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def generators():
    return gell_mann() / 2.0


def structure_constants():
    """f^{abc} = -2 i Tr(T^a [T^b, T^c])."""
    t = generators()
    comm = np.einsum('bij,cjk->bcik', t, t) - np.einsum('cij,bjk->bcik', t, t)
    f = -2j * np.einsum('aij,bcji->abc', t, comm)
    return f.real


def string_tensor(perm):
    """Explicit (T^{a_p1} ... T^{a_pn})_{ij} as an array [8]*n + [3, 3].

    Axis q of the result is the colour of gluon slot q (not of position q).
    """
    n = len(perm)
    t = generators()
    out = np.zeros((8,) * n + (3, 3), dtype=complex)
    for a in itertools.product(range(8), repeat=n):
        m = np.eye(3, dtype=complex)
        for slot in perm:
            m = m @ t[a[slot]]
        out[a] = m
    return out


def gell_mann_colour_matrix(n):
    """CF from explicit colour sums (float); practical for n <= 4."""
    basis = colour_basis(n)
    tens = [string_tensor(p).reshape(-1) for p in basis]
    return np.array([[np.vdot(ts, tt) for tt in tens] for ts in tens]).real


def iden(npar):
    """Initial-state average and final-state symmetry factor: 4 * 64 * k!."""
    k = npar - 4
    f = 1
    for i in range(2, k + 1):
        f *= i
    return 4 * 64 * f
