"""Tree-level Feynman diagrams of g g -> t tbar + k g and their colour (oracle).

Every tree diagram of this process has one top line running from the outgoing
top to the outgoing antitop.  Along it sit m >= 1 quark-gluon vertices, and
at each one hangs a gluon subtree: either an external gluon, or an internal
gluon ending in a three-gluon (ggg) or four-gluon (gggg) vertex whose other
legs are again subtrees.  A diagram is therefore an ordered sequence of
gluon trees whose leaf sets partition the n = k + 2 external gluons; the
order along the line matters, the order of the children of a gluon vertex
does not.  The paper lists the resulting counts (3, 16, 123, 1240, 15495
diagrams for k = 0..4) in its complexity table.

A four-gluon vertex carries three colour structures, each with its own
Lorentz structure (the textbook Feynman rule)

    -i g^2 [ f^{abe} f^{cde} (g^{mu rho} g^{nu sig} - g^{mu sig} g^{nu rho})
           + f^{ace} f^{bde} (g^{mu nu} g^{rho sig} - g^{mu sig} g^{nu rho})
           + f^{ade} f^{bce} (g^{mu nu} g^{rho sig} - g^{mu rho} g^{nu sig}) ],

so a diagram splits into 3^(#gggg) "pieces", each with a single colour
factor.  Trees here are piece-labelled:

    leaf       int  (gluon slot)
    ('3', A, B)            ggg vertex, children A, B
    ('4', s, A, B, C)      gggg vertex, structure s in {0,1,2}, legs (b,c,d)

Colour factors reduce onto the quark-line strings with
    f^{abc} T^a = -i [T^b, T^c]
applied at each gluon vertex (parent leg a):
    ggg:   T^a f^{abc}            -> -i [B, C]
    gggg:  T^a f^{abe} f^{cde}    -> -[B, [C, D]]     (s = 0)
           T^a f^{ace} f^{bde}    -> -[C, [B, D]]     (s = 1)
           T^a f^{ade} f^{bce}    -> -[D, [B, C]]     (s = 2)
which yields the coefficients c_{d,sigma} in {+-1, +-i} of the paper's
"jamp += c * amp" step (pseudo-code of the monolithic kernel).
"""
from __future__ import annotations

import itertools
from functools import lru_cache


def _set_partitions(items, k):
    """Unordered partitions of the tuple `items` into k non-empty blocks.

    Blocks are returned in order of their smallest element.
    """
    items = tuple(items)
    if k == 1:
        yield (items,)
        return
    if len(items) < k:
        return
    first, rest = items[0], items[1:]
    # the block containing `first`: choose which other items join it
    for r in range(0, len(rest) - k + 2):
        for comb in itertools.combinations(rest, r):
            block = (first,) + comb
            remaining = tuple(x for x in rest if x not in comb)
            for sub in _set_partitions(remaining, k - 1):
                yield (block,) + sub


@lru_cache(maxsize=None)
def gluon_trees(leaves):
    """All piece-labelled gluon trees whose leaf set is the sorted tuple `leaves`."""
    if len(leaves) == 1:
        return (leaves[0],)
    out = []
    for a, b in _set_partitions(leaves, 2):
        for ta in gluon_trees(a):
            for tb in gluon_trees(b):
                out.append(('3', ta, tb))
    for a, b, c in _set_partitions(leaves, 3):
        for ta in gluon_trees(a):
            for tb in gluon_trees(b):
                for tc in gluon_trees(c):
                    for s in range(3):
                        out.append(('4', s, ta, tb, tc))
    return tuple(out)


def _ordered_partitions(items):
    """All ordered sequences of non-empty blocks partitioning `items`."""
    items = tuple(items)
    for k in range(1, len(items) + 1):
        for part in _set_partitions(items, k):
            for perm in itertools.permutations(part):
                yield perm


def diagram_pieces(n):
    """All diagram pieces for n gluons: tuples of trees along the top line.

    The first tree is attached next to the outgoing top.
    """
    out = []
    for blocks in _ordered_partitions(range(n)):
        for trees in itertools.product(*(gluon_trees(b) for b in blocks)):
            out.append(tuple(trees))
    return out


def _has_piece_label(tree, nonzero):
    if isinstance(tree, int):
        return False
    if tree[0] == '3':
        return _has_piece_label(tree[1], nonzero) or _has_piece_label(tree[2], nonzero)
    if tree[1] != 0:
        nonzero[0] = True
    return any(_has_piece_label(t, nonzero) for t in tree[2:])


def count_diagrams(n):
    """Number of Feynman diagrams (each gggg vertex counted once)."""
    count = 0
    for piece in diagram_pieces(n):
        flag = [False]
        for t in piece:
            _has_piece_label(t, flag)
        if not flag[0]:
            count += 1
    return count


def count_cubic_diagrams(n):
    """Number of diagrams with only three-point vertices."""
    def cubic(t):
        if isinstance(t, int):
            return True
        return t[0] == '3' and cubic(t[1]) and cubic(t[2])
    return sum(1 for p in diagram_pieces(n) if all(cubic(t) for t in p))


# --- colour reduction -------------------------------------------------------

def _mul(x, y):
    out = {}
    for wx, cx in x.items():
        for wy, cy in y.items():
            w = wx + wy
            out[w] = out.get(w, 0) + cx * cy
    return out


def _add(x, y, sy=1):
    out = dict(x)
    for w, c in y.items():
        out[w] = out.get(w, 0) + sy * c
    return out


def _comm(x, y):
    return _add(_mul(x, y), _mul(y, x), -1)


def _scale(x, c):
    return {w: c * v for w, v in x.items()}


def tree_colour(tree):
    """Expansion of T^{root} x (colour factor of the tree) onto T-words."""
    if isinstance(tree, int):
        return {(tree,): 1}
    if tree[0] == '3':
        return _scale(_comm(tree_colour(tree[1]), tree_colour(tree[2])), -1j)
    s, b, c, d = tree[1], tree_colour(tree[2]), tree_colour(tree[3]), tree_colour(tree[4])
    if s == 0:
        return _scale(_comm(b, _comm(c, d)), -1)
    if s == 1:
        return _scale(_comm(c, _comm(b, d)), -1)
    return _scale(_comm(d, _comm(b, c)), -1)


def piece_colour(piece):
    """Colour coefficients {permutation: c} of a diagram piece."""
    acc = {(): 1}
    for t in piece:
        acc = _mul(acc, tree_colour(t))
    return {w: c for w, c in acc.items() if c != 0}
