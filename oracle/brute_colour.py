"""Explicit-colour brute-force |M|^2 (oracle cross-check).

Sums |M|^2 over every explicit colour assignment of the external gluons
(a_i in 1..8) and of the top pair (i, j in 1..3), with Gell-Mann generators
T^a and f^{abc} = -2i Tr(T^a [T^b, T^c]) contracted along each diagram as the
Feynman rules state (no reduction onto colour strings, no colour matrix).
This pins the colour reduction and the colour matrix of the diagram oracle,
which the paper computes as the quadratic form J^H C J (colour-sum equation).
Practical for up to four gluons.
"""
from __future__ import annotations

import numpy as np

from .colour import generators, structure_constants
from .me import piece_amplitudes

_LEAF = 'ABCDEFGHIJKLMNOP'


def _tree_tensor(tree, f):
    """(K, slots): K[e, a_s1, a_s2, ...] = colour factor with root-line colour e."""
    if isinstance(tree, int):
        return np.eye(8), [tree]
    if tree[0] == '3':
        ka, sa = _tree_tensor(tree[1], f)
        kb, sb = _tree_tensor(tree[2], f)
        la = _LEAF[:len(sa)]
        lb = _LEAF[len(sa):len(sa) + len(sb)]
        k = np.einsum(f'exy,x{la},y{lb}->e{la}{lb}', f, ka, kb)
        return k, sa + sb
    s = tree[1]
    (ka, sa), (kb, sb), (kc, sc) = (_tree_tensor(t, f) for t in tree[2:])
    la = _LEAF[:len(sa)]
    lb = _LEAF[len(sa):len(sa) + len(sb)]
    lc = _LEAF[len(sa) + len(sb):len(sa) + len(sb) + len(sc)]
    # legs: a = parent (index 'a'), b = child A ('b'), c = child B ('c'), d = child C ('d'); e summed
    ff = {0: 'abe,cde', 1: 'ace,bde', 2: 'ade,bce'}[s]
    k = np.einsum(f'{ff},b{la},c{lb},d{lc}->a{la}{lb}{lc}', f, f, ka, kb, kc)
    return k, sa + sb + sc


def piece_colour_tensor(piece, n):
    """C[a_0, ..., a_{n-1}, i, j] for one diagram piece."""
    t = generators()
    f = structure_constants()
    mat = None
    slots = []
    for tree in piece:
        k, s = _tree_tensor(tree, f)
        ls = _LEAF[:len(s)]
        m = np.einsum(f'eij,e{ls}->{ls}ij', t, k)   # leaves..., i, j
        if mat is None:
            mat, slots = m, list(s)
        else:
            l1 = _LEAF[:len(slots)]
            l2 = _LEAF[len(slots):len(slots) + len(s)]
            mat = np.einsum(f'{l1}ij,{l2}jk->{l1}{l2}ik', mat, m)
            slots = slots + list(s)
    order = np.argsort(slots)
    return np.transpose(mat, list(order) + [n, n + 1])


def matrix_element(proc, mom, alpha_s):
    n = proc.ngluon
    tens = np.stack([piece_colour_tensor(p, n).reshape(-1) for p in proc.pieces])  # [npiece, ncol]
    total = 0.0
    for h in range(proc.nhel):
        amps = piece_amplitudes(proc, mom, h, alpha_s)           # [npiece, nevt]
        m = tens.T @ amps                                        # [ncol, nevt]
        total = total + (np.abs(m) ** 2).sum(axis=0)
    return total / proc.iden
