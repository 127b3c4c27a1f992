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
COST = {'G': 24, 'U': 35, 'V': 37, 'v3': 162, 'v4': 133, 'Lh': 72, 'L': 79,
        'Rh': 72, 'R': 79, 'K': 80, 'KD3': 170, 'KD4': 140, 'dot': 30, 'ffv': 102}


class Plan:
    """Objects (currents) in evaluation order and amplitudes as contractions.

    Every diagram piece is evaluated by cutting one internal line (or at one
    quark-gluon vertex) and contracting the memoised currents on both sides:
      top-line cut         L . Rh  or  Lh . R
      quark-gluon vertex   L (i g gamma.J) R                         ('ffv')
      gluon-line cut       K . J   (line attaching a tree to the top line) or
                           KD . J  (line inside a tree; KD is the top-line current
                           carried through the gluon vertices above the cut)
    A greedy pass followed by refinement sweeps picks, per piece, the cut whose
    missing currents cost the fewest flops given all other pieces' choices.
    """

    def __init__(self, n, sweeps=6):
        self.n = n
        self.trees = Trees(n)
        self.pieces = diagram_pieces(self.trees)
        memo = {}
        self.colours = [piece_colour(self.trees, p, memo) for p in self.pieces]
        self.basis = list(itertools.permutations(range(n)))
        self.ndiagrams = sum(1 for p in self.pieces if all(self.trees.is_full(t) for t in p))
        self._deps = {}
        self._cands = [self.candidates(p) for p in self.pieces]
        self._choose(sweeps)

    # object keys: ('G', slot) ('U',) ('V',) ('J', t) ('Lh', seq) ('L', seq) ('Rh', seq)
    #              ('R', seq) ('K', prefix, suffix) ('KD', prefix, suffix, steps)
    # a step is (kind, s, hole_leg, siblings): the gluon vertex below the previous
    # line, its colour structure, the leg that stays open and the other children.
    def deps(self, key):
        hit = self._deps.get(key)
        if hit is not None:
            return hit
        kind = key[0]
        if kind in ('G', 'U', 'V'):
            out = ()
        elif kind == 'J':
            node = self.trees.nodes[key[1]]
            if node[0] == 'leaf':
                out = (('G', node[1]),)
            else:
                kids = node[1:] if node[0] == 'v3' else node[2:]
                out = tuple(self.jkey(c) for c in kids)
        elif kind == 'Lh':
            seq = key[1]
            prev = ('L', seq[:-1]) if len(seq) > 1 else ('U',)
            out = (prev, self.jkey(seq[-1]))
        elif kind == 'L':
            out = (('Lh', key[1]),)
        elif kind == 'Rh':
            seq = key[1]
            nxt = ('R', seq[1:]) if len(seq) > 1 else ('V',)
            out = (nxt, self.jkey(seq[0]))
        elif kind == 'R':
            out = (('Rh', key[1]),)
        elif kind == 'K':
            left = ('L', key[1]) if key[1] else ('U',)
            right = ('R', key[2]) if key[2] else ('V',)
            out = (left, right)
        elif kind == 'KD':
            pre, suf, steps = key[1], key[2], key[3]
            parent = ('KD', pre, suf, steps[:-1]) if len(steps) > 1 else ('K', pre, suf)
            out = (parent,) + tuple(self.jkey(t) for t in steps[-1][3])
        else:
            raise KeyError(key)
        self._deps[key] = out
        return out

    def jkey(self, t):
        node = self.trees.nodes[t]
        if node[0] == 'leaf':
            return ('G', node[1])
        return ('J', t)

    def routine(self, key):
        """Name of the device routine that computes object `key`."""
        kind = key[0]
        if kind == 'J':
            return self.trees.nodes[key[1]][0]
        if kind == 'KD':
            return 'KD3' if key[3][-1][0] == 'v3' else 'KD4'
        return kind

    def cost(self, key):
        return COST[self.routine(key)]

    def hole_mask(self, key):
        """Gluons below the open line of a K / KD current (the parent-line subtree for KD)."""
        full = (1 << self.n) - 1
        m = full
        for t in key[1] + key[2]:
            m &= ~self.trees.mask[t]
        if key[0] == 'KD':
            for step in key[3][:-1]:
                for t in step[3]:
                    m &= ~self.trees.mask[t]
        return m

    def _lines(self, t, steps):
        """(steps, subtree) for every gluon line strictly inside tree t."""
        node = self.trees.nodes[t]
        if node[0] == 'leaf':
            return
        kids = node[1:] if node[0] == 'v3' else node[2:]
        s = 0 if node[0] == 'v3' else node[1]
        for pos, child in enumerate(kids):
            sibs = tuple(k for i, k in enumerate(kids) if i != pos)
            st = steps + ((node[0], s, pos + 1, sibs),)
            yield st, child
            yield from self._lines(child, st)

    def candidates(self, piece):
        """(contraction cost, required objects) for every way to evaluate a piece."""
        m = len(piece)
        out = []
        for j in range(1, m):
            pre, suf = piece[:j], piece[j:]
            out.append((COST['dot'], (('L', pre), ('Rh', suf))))
            out.append((COST['dot'], (('Lh', pre), ('R', suf))))
        if m == 1:
            out.append((COST['dot'], (('Lh', piece), ('V',))))
        for j in range(m):
            pre, suf = piece[:j], piece[j + 1:]
            left = ('L', pre) if pre else ('U',)
            right = ('R', suf) if suf else ('V',)
            out.append((COST['ffv'], (left, self.jkey(piece[j]), right)))
            out.append((COST['dot'], (('K', pre, suf), self.jkey(piece[j]))))
            for steps, sub in self._lines(piece[j], ()):
                out.append((COST['dot'], (('KD', pre, suf, steps), self.jkey(sub))))
        return out

    # --- greedy choice with refinement ------------------------------------
    def _missing(self, key, seen):
        if self.refs.get(key, 0) > 0 or key in seen:
            return 0
        seen.add(key)
        c = self.cost(key)
        if self.amortise:
            c = c / self.popularity.get(key, 1)
        return c + sum(self._missing(d, seen) for d in self.deps(key))

    def _closure(self, objs, out):
        for o in objs:
            if o not in out:
                out.add(o)
                self._closure(self.deps(o), out)

    def _inc(self, key):
        r = self.refs.get(key, 0)
        self.refs[key] = r + 1
        if r == 0:
            for d in self.deps(key):
                self._inc(d)

    def _dec(self, key):
        r = self.refs[key] - 1
        self.refs[key] = r
        if r == 0:
            for d in self.deps(key):
                self._dec(d)

    def _best(self, i):
        best = None
        for c, objs in self._cands[i]:
            seen = set()
            tot = c + sum(self._missing(o, seen) for o in objs)
            if best is None or tot < best[0]:
                best = (tot, objs)
        return best[1]

    def _choose(self, sweeps):
        self.refs = {}
        # popularity: in how many pieces' candidate sets (with dependencies) an object appears
        self.popularity = {}
        for cands in self._cands:
            objs = set()
            for _, c in cands:
                self._closure(c, objs)
            for o in objs:
                self.popularity[o] = self.popularity.get(o, 0) + 1
        order = sorted(range(len(self.pieces)), key=lambda i: (len(self.pieces[i]), self.pieces[i]))
        choice = [None] * len(self.pieces)
        # first pass: costs amortised over the pieces that could share an object
        self.amortise = True
        for i in order:
            choice[i] = self._best(i)
            for o in choice[i]:
                self._inc(o)
        self.amortise = False
        for _ in range(sweeps):
            changed = 0
            for i in order:
                for o in choice[i]:
                    self._dec(o)
                new = self._best(i)
                if new != choice[i]:
                    changed += 1
                choice[i] = new
                for o in new:
                    self._inc(o)
            if not changed:
                break
        self.choice = choice
        # evaluation order: dependencies first, in the order pieces are visited
        self.objects = {}
        self.order = []

        def add(key):
            if key in self.objects:
                return
            for d in self.deps(key):
                add(d)
            self.objects[key] = self.deps(key)
            self.order.append(key)

        self.amps = []
        for i in order:
            for o in choice[i]:
                add(o)
            self.amps.append((i,) + tuple(choice[i]))

    def colour_groups(self):
        """Amplitudes grouped by colour vector (equal up to a unit factor).

        Returns [(key, members)], key = ((colour index, coefficient relative to
        the lead), ...), members = [(lead coefficient, amp), ...], in order of
        first appearance in self.amps.
        """
        index = {p: i for i, p in enumerate(self.basis)}
        groups = {}
        order = []
        for amp in self.amps:
            items = sorted((index[w], complex(v)) for w, v in self.colours[amp[0]].items())
            lead = items[0][1]
            key = tuple((i, v / lead) for i, v in items)
            if key not in groups:
                groups[key] = []
                order.append(key)
            groups[key].append((lead, amp))
        return [(k, groups[k]) for k in order]

    def peak_live(self, groups):
        """Largest number of currents alive at once when groups run in this order."""
        events = []
        seen = set()

        def need(k):
            if k in seen:
                return
            for d in self.objects[k]:
                need(d)
            seen.add(k)
            events.append(('obj', k))

        for gi, (key, members) in enumerate(groups):
            for lead, amp in members:
                for o in amp[1:]:
                    need(o)
            events.append(('grp', gi))
        last = {}
        for i, ev in enumerate(events):
            if ev[0] == 'obj':
                for d in self.objects[ev[1]]:
                    last[d] = i
            else:
                for lead, amp in groups[ev[1]][1]:
                    for o in amp[1:]:
                        last[o] = i
        alive, peak = set(), 0
        for i, ev in enumerate(events):
            if ev[0] == 'obj':
                alive.add(ev[1])
            peak = max(peak, len(alive))
            if ev[0] == 'grp':
                alive = {o for o in alive if last.get(o, -1) > i}
        return peak

    def scheduled_groups(self, alphas=(0.5, 0.75, 1.0)):
        """colour_groups() reordered to keep few currents alive at once.

        List scheduling: repeatedly emit the group whose evaluation creates the
        fewest new currents net of alpha x the currents it retires (a current
        retires after its last consumer); the order with the smallest peak over
        a few alphas is kept.  The order only affects register pressure.
        """
        groups = self.colour_groups()
        if len(groups) > 2000:
            # the list scheduler is quadratic in the number of groups; large
            # processes (which only get the team program, where the order sets
            # the LDS frame size, not registers) take the groups in the order
            # of their earliest current in the plan
            pos = {k: i for i, k in enumerate(self.order)}
            return sorted(groups, key=lambda g: min(pos[o] for _, a in g[1] for o in a[1:]))
        best = None
        for a in alphas:
            order = self._schedule(a)
            pk = self.peak_live(order)
            if best is None or pk < best[0]:
                best = (pk, order)
        return best[1]

    def split_groups(self, weight=0.25, window=16):
        """scheduled_groups() reordered for the split executor's group-sum code, in
        which no colour flows are live and the registers hold only currents.

        Greedy: the next group is the one whose currents (with everything they
        depend on) are mostly computed already, counting weight x its currents
        among the last `window` ones touched (a stand-in for what is still in
        registers) in its favour.  On g g -> t t~ g g g this cuts the spill traffic
        of an optimal (furthest-next-use) register allocation of 12 to 24 currents
        by 18-34 % against the scheduled order.
        """
        cached = getattr(self, '_split_groups', None)
        if cached is not None:
            return cached
        base = self.scheduled_groups()
        if len(base) > 2000:
            self._split_groups = base
            return base

        def closure(ops):
            out, stack = set(), list(ops)
            while stack:
                k = stack.pop()
                if k not in out:
                    out.add(k)
                    stack.extend(self.objects[k])
            return out

        cl = [closure({o for _, a in members for o in a[1:]}) for _, members in base]
        done, order, recent = set(), [], []
        remaining = list(range(len(base)))
        while remaining:
            last = set(recent[-window:])
            best = min(remaining, key=lambda gi: (len(cl[gi] - done) - weight * len(cl[gi] & last), gi))
            remaining.remove(best)
            order.append(best)
            done |= cl[best]
            recent.extend(sorted(cl[best] - last, key=str))
        self._split_groups = [base[i] for i in order]
        return self._split_groups

    def _schedule(self, alpha):
        groups = self.colour_groups()
        gops = []
        for key, members in groups:
            ops = []
            for lead, amp in members:
                for o in amp[1:]:
                    if o not in ops:
                        ops.append(o)
            gops.append(ops)
        uses = {}
        for k in self.order:
            for d in self.objects[k]:
                uses[d] = uses.get(d, 0) + 1
        for ops in gops:
            for o in ops:
                uses[o] = uses.get(o, 0) + 1
        computed, alive = set(), set()
        remaining = list(range(len(groups)))
        out = []

        def closure(ops):
            res, seen = [], set()

            def rec(k):
                if k in computed or k in seen:
                    return
                seen.add(k)
                for d in self.objects[k]:
                    rec(d)
                res.append(k)
            for o in ops:
                rec(o)
            return res

        while remaining:
            best = None
            for g in remaining:
                new = closure(gops[g])
                dec = {}
                for k in new:
                    for d in self.objects[k]:
                        dec[d] = dec.get(d, 0) + 1
                for o in gops[g]:
                    dec[o] = dec.get(o, 0) + 1
                newset = set(new)
                freed = sum(1 for o, c in dec.items()
                            if uses[o] == c and (o in alive or o in newset))
                score = len(new) - alpha * freed
                if best is None or score < best[0]:
                    best = (score, g, new)
            _, g, new = best
            for k in new:
                computed.add(k)
                alive.add(k)
                for d in self.objects[k]:
                    uses[d] -= 1
            for o in gops[g]:
                uses[o] -= 1
            alive = {o for o in alive if uses[o] > 0}
            remaining.remove(g)
            out.append(groups[g])
        return out

    # --- summaries -----------------------------------------------------------
    def flops(self):
        tot = sum(self.cost(k) for k in self.order)
        for a in self.amps:
            tot += COST['ffv'] if len(a) == 4 else COST['dot']
        return tot

    def counts(self):
        out = {}
        for k in self.order:
            kind = k[0] if k[0] != 'J' else self.trees.nodes[k[1]][0]
            out[kind] = out.get(kind, 0) + 1
        out['amp'] = len(self.amps)
        out['ffv'] = sum(1 for a in self.amps if len(a) == 4)
        return out
