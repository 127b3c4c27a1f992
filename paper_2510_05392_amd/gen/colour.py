"""Exact colour matrix of the quark-line colour basis (generator side).

Basis: the n! strings (T^{a_s1} ... T^{a_sn})_{i j} of one quark line with
n gluons, permutations s in lexicographic order (the paper's "leading
colours": 2, 6, 24, 120, 720 for two to six gluons, complexity table).

    CF[s, t] = sum_a Tr(T^{s_n} ... T^{s_1} T^{t_1} ... T^{t_n})

is evaluated by expanding every summed gluon index with
    T^a_{ij} T^a_{kl} = 1/2 (d_il d_kj - d_ij d_kl / N),   N = 3,
over all 2^n choices of term and counting the closed index loops (each worth
a factor N) with a union-find on the 2n trace indices.  Relabelling the
summed gluons is free, so CF[s, t] = R[s^-1 t] with R the first row; only
that row is expanded.  The result is returned as an integer matrix times
1/denominator (the paper keeps its colour matrix as integers plus a common
denominator, "colormatrix" in its monolithic-kernel pseudo-code).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

NC = 3


def basis(n):
    return list(itertools.permutations(range(n)))


def _find(parent, x):
    while parent[x] != x:
        parent[x] = parent[parent[x]]
        x = parent[x]
    return x


def _trace_value(word):
    """sum over the gluon indices of Tr(T^{w_0} ... T^{w_{L-1}}); each letter twice."""
    length = len(word)
    pos = {}
    for k, a in enumerate(word):
        pos.setdefault(a, []).append(k)
    pairs = list(pos.values())
    total = Fraction(0)
    # matrix k carries indices (k, k+1 mod L); a delta joins two index nodes
    for choice in itertools.product((0, 1), repeat=len(pairs)):
        parent = list(range(length))
        for (k, l), c in zip(pairs, choice):
            ik, ik1 = k, (k + 1) % length
            il, il1 = l, (l + 1) % length
            if c == 0:       # d_{i_k i_{l+1}} d_{i_l i_{k+1}}
                joins = ((ik, il1), (il, ik1))
            else:            # -1/N d_{i_k i_{k+1}} d_{i_l i_{l+1}}
                joins = ((ik, ik1), (il, il1))
            for x, y in joins:
                rx, ry = _find(parent, x), _find(parent, y)
                if rx != ry:
                    parent[rx] = ry
        loops = len({_find(parent, x) for x in range(length)})
        nsecond = sum(choice)
        total += Fraction(NC) ** loops * Fraction(-1, NC) ** nsecond
    return total / 2 ** len(pairs)


def colour_matrix(n):
    """(cf_int, denominator): exact CF = cf_int / denominator, cf_int symmetric."""
    bas = basis(n)
    index = {p: i for i, p in enumerate(bas)}
    ident = tuple(range(n))
    row = {}
    for t in bas:
        row[t] = _trace_value(tuple(reversed(ident)) + t)
    den = 1
    for v in row.values():
        den = den * v.denominator // math.gcd(den, v.denominator)
    m = len(bas)
    cf = [[0] * m for _ in range(m)]
    for s in bas:
        inv = [0] * n
        for k, a in enumerate(s):
            inv[a] = k
        for t in bas:
            pi = tuple(inv[a] for a in t)
            v = row[pi] * den
            assert v.denominator == 1
            cf[index[s]][index[t]] = int(v)
    return cf, den
