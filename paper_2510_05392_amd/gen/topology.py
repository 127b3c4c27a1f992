"""Diagram topology, colour coefficients and the evaluation plan (generator side).

A tree diagram of g g -> t tbar + k g has one top line (outgoing top ... outgoing
antitop) carrying m >= 1 quark-gluon vertices; a gluon tree hangs at each of
them (a single external gluon, or an internal gluon ending in a ggg or gggg
vertex).  Enumerating ordered sequences of gluon trees over a partition of
the n = k + 2 gluons gives the paper's counts (complexity table: 3, 16, 123,
1240, 15495).  A gggg vertex is split into its three colour structures
("pieces"), each with its own Lorentz factor.

Evaluation plan.  As in the paper's generated code (wavefunctions computed
once and reused by many amplitudes, section "a closer look at the internals
of the ME engine"), every amplitude here is a contraction of two memoised
off-shell currents:

  G(s)       external gluon polarisation              (4 complex)
  U, V       ubar(top) row spinor, v(antitop) column spinor
  J(tree)    gluon current of a gluon tree, propagator included
  Lh(T1..Tj) ubar Gam(T1) S ... Gam(Tj)        (row spinor, no final propagator)
  L(T1..Tj)  Lh(T1..Tj) S(q_j)
  Rh(Tj..Tm) Gam(Tj) S ... Gam(Tm) v           (column spinor)
  R(Tj..Tm)  S(q_{j-1}) Rh(Tj..Tm)
  K(P | Q)   L(P) (i g gamma^mu) R(Q)           (gluon current of the top line with one hole)

  amplitude = L . Rh  |  Lh . R  (cut on a top propagator)   or   K . J (cut on the gluon
  line that attaches a tree to the top line).

Gam(T) = i g gamma.J(T), S(q) = i (qslash + m) / (q^2 - m^2).  For every diagram
piece a greedy optimiser picks the cut whose not-yet-computed currents cost the
fewest FP64 flops.
"""
from __future__ import annotations

import itertools

# --- gluon trees (interned) --------------------------------------------------


class Trees:
    """Interned piece-labelled gluon trees indexed by leaf bit masks."""

    def __init__(self, n):
        self.n = n
        self.nodes = []          # id -> ('leaf', slot) | ('v3', a, b) | ('v4', s, a, b, c)
        self.mask = []           # id -> leaf bit mask
        self.by_mask = {}
        for m in range(1, 1 << n):
            self._build(m)

    def _add(self, node, mask):
        self.nodes.append(node)
        self.mask.append(mask)
        return len(self.nodes) - 1

    def _build(self, mask):
        if mask in self.by_mask:
            return self.by_mask[mask]
        ids = []
        if mask & (mask - 1) == 0:
            ids.append(self._add(('leaf', mask.bit_length() - 1), mask))
        else:
            low = mask & -mask
            rest = mask ^ low
            # two blocks: the one holding the lowest leaf first
            sub = rest
            while True:
                a = low | sub
                b = mask ^ a
                if b:
                    for ta in self._build(a):
                        for tb in self._build(b):
                            ids.append(self._add(('v3', ta, tb), mask))
                if sub == 0:
                    break
                sub = (sub - 1) & rest
            # three blocks, ordered by their lowest leaves
            sub = rest
            while True:
                a = low | sub
                rem = mask ^ a
                if rem:
                    low2 = rem & -rem
                    rest2 = rem ^ low2
                    sub2 = rest2
                    while True:
                        b = low2 | sub2
                        c = rem ^ b
                        if c:
                            for ta in self._build(a):
                                for tb in self._build(b):
                                    for tc in self._build(c):
                                        for s in range(3):
                                            ids.append(self._add(('v4', s, ta, tb, tc), mask))
                        if sub2 == 0:
                            break
                        sub2 = (sub2 - 1) & rest2
                if sub == 0:
                    break
                sub = (sub - 1) & rest
        self.by_mask[mask] = ids
        return ids

    def is_full(self, t):
        """True for a piece label 0 at every gggg node (counts a diagram once)."""
        node = self.nodes[t]
        if node[0] == 'leaf':
            return True
        if node[0] == 'v3':
            return self.is_full(node[1]) and self.is_full(node[2])
        return node[1] == 0 and all(self.is_full(c) for c in node[2:])


def diagram_pieces(trees):
    """Ordered tuples of tree ids whose masks partition all gluons."""
    full = (1 << trees.n) - 1
    out = []

    def rec(remaining, prefix):
        if remaining == 0:
            out.append(tuple(prefix))
            return
        sub = remaining
        while sub:
            for t in trees.by_mask[sub]:
                prefix.append(t)
                rec(remaining ^ sub, prefix)
                prefix.pop()
            sub = (sub - 1) & remaining

    rec(full, [])
    return out


# --- colour: leaf orderings of each tree -------------------------------------

# coefficient of each ordering of the children (b, c, d) of a gggg piece,
# from T^a f^{abe} f^{cde} = -[b,[c,d]], T^a f^{ace} f^{bde} = -[c,[b,d]],
# T^a f^{ade} f^{bce} = -[d,[b,c]]
_V4_ORDERS = {
    0: {(0, 1, 2): -1, (0, 2, 1): 1, (1, 2, 0): 1, (2, 1, 0): -1},
    1: {(1, 0, 2): -1, (1, 2, 0): 1, (0, 2, 1): 1, (2, 0, 1): -1},
    2: {(2, 0, 1): -1, (2, 1, 0): 1, (0, 1, 2): 1, (1, 0, 2): -1},
}


def tree_orderings(trees, t, memo):
    """{leaf ordering: coefficient} of T^{root} (colour of tree t)."""
    if t in memo:
        return memo[t]
    node = trees.nodes[t]
    out = {}
    if node[0] == 'leaf':
        out[(node[1],)] = 1
    elif node[0] == 'v3':
        # f^{abc} T^a = -i [T^b, T^c]
        oa = tree_orderings(trees, node[1], memo)
        ob = tree_orderings(trees, node[2], memo)
        for wa, ca in oa.items():
            for wb, cb in ob.items():
                out[wa + wb] = out.get(wa + wb, 0) - 1j * ca * cb
                out[wb + wa] = out.get(wb + wa, 0) + 1j * ca * cb
    else:
        kids = [tree_orderings(trees, c, memo) for c in node[2:]]
        for order, sign in _V4_ORDERS[node[1]].items():
            for combo in itertools.product(*(kids[i].items() for i in order)):
                w = tuple(x for wc in combo for x in wc[0])
                c = sign
                for wc in combo:
                    c = c * wc[1]
                out[w] = out.get(w, 0) + c
    out = {w: c for w, c in out.items() if c != 0}
    memo[t] = out
    return out


def piece_colour(trees, piece, memo):
    acc = {(): 1}
    for t in piece:
        nxt = {}
        o = tree_orderings(trees, t, memo)
        for w1, c1 in acc.items():
            for w2, c2 in o.items():
                nxt[w1 + w2] = nxt.get(w1 + w2, 0) + c1 * c2
        acc = nxt
    return {w: c for w, c in acc.items() if c != 0}


# --- evaluation plan ---------------------------------------------------------

# FP64 flop estimates of each building block (add, mul = 1; used only to rank choices)
COST = {'G': 30, 'U': 40, 'V': 40, 'v3': 140, 'v4': 120, 'Lh': 64, 'L': 80,
        'Rh': 64, 'R': 80, 'K': 100, 'dot': 30}


class Plan:
    """Objects (currents) in evaluation order and amplitudes as contractions."""

    def __init__(self, n):
        self.n = n
        self.trees = Trees(n)
        self.pieces = diagram_pieces(self.trees)
        memo = {}
        self.colours = [piece_colour(self.trees, p, memo) for p in self.pieces]
        self.basis = list(itertools.permutations(range(n)))
        self.ndiagrams = sum(1 for p in self.pieces if all(self.trees.is_full(t) for t in p))
        self.objects = {}        # key -> dependency keys
        self.order = []          # computed keys in dependency order
        self.amps = []           # (piece index, key_a, key_b)
        self._choose()

    # object keys: ('G', slot) ('U',) ('V',) ('J', t) ('Lh', seq) ('L', seq)
    #              ('Rh', seq) ('R', seq) ('K', prefix, suffix)
    def deps(self, key):
        kind = key[0]
        if kind in ('G', 'U', 'V'):
            return ()
        if kind == 'J':
            node = self.trees.nodes[key[1]]
            if node[0] == 'leaf':
                return (('G', node[1]),)
            kids = node[1:] if node[0] == 'v3' else node[2:]
            return tuple(self.jkey(c) for c in kids)
        if kind == 'Lh':
            seq = key[1]
            prev = ('L', seq[:-1]) if len(seq) > 1 else ('U',)
            return (prev, self.jkey(seq[-1]))
        if kind == 'L':
            return (('Lh', key[1]),)
        if kind == 'Rh':
            seq = key[1]
            nxt = ('R', seq[1:]) if len(seq) > 1 else ('V',)
            return (nxt, self.jkey(seq[0]))
        if kind == 'R':
            return (('Rh', key[1]),)
        if kind == 'K':
            left = ('L', key[1]) if key[1] else ('U',)
            right = ('R', key[2]) if key[2] else ('V',)
            return (left, right)
        raise KeyError(key)

    def jkey(self, t):
        node = self.trees.nodes[t]
        if node[0] == 'leaf':
            return ('G', node[1])
        return ('J', t)

    def cost(self, key):
        kind = key[0]
        if kind == 'J':
            return COST[self.trees.nodes[key[1]][0]]
        return COST[kind]

    def _missing_cost(self, key, seen):
        if key in self.objects or key in seen:
            return 0
        seen.add(key)
        return self.cost(key) + sum(self._missing_cost(d, seen) for d in self.deps(key))

    def _add(self, key):
        if key in self.objects:
            return
        ds = self.deps(key)
        for d in ds:
            self._add(d)
        self.objects[key] = ds
        self.order.append(key)

    def candidates(self, piece):
        m = len(piece)
        out = []
        for j in range(1, m):
            pre, suf = piece[:j], piece[j:]
            out.append((('L', pre), ('Rh', suf)))
            out.append((('Lh', pre), ('R', suf) if suf else ('V',)))
        if m == 1:
            out.append((('Lh', piece), ('V',)))
        for j in range(m):
            out.append((('K', piece[:j], piece[j + 1:]), self.jkey(piece[j])))
        return out

    def _choose(self):
        # visit pieces so that those sharing long prefixes are adjacent
        order = sorted(range(len(self.pieces)), key=lambda i: (len(self.pieces[i]), self.pieces[i]))
        for i in order:
            best = None
            for a, b in self.candidates(self.pieces[i]):
                seen = set()
                c = self._missing_cost(a, seen) + self._missing_cost(b, seen)
                if best is None or c < best[0]:
                    best = (c, a, b)
            _, a, b = best
            self._add(a)
            self._add(b)
            self.amps.append((i, a, b))

    # --- summaries -----------------------------------------------------------
    def flops(self):
        return sum(self.cost(k) for k in self.order) + COST['dot'] * len(self.amps)

    def counts(self):
        out = {}
        for k in self.order:
            kind = k[0] if k[0] != 'J' else self.trees.nodes[k[1]][0]
            out[kind] = out.get(kind, 0) + 1
        out['amp'] = len(self.amps)
        return out
