"""Wave-cooperative ("team") program for one process, from its evaluation plan.

The straight-line kernel gives every lane one (event, helicity) and keeps all
of its currents in registers; from three gluons on that state outgrows the
register file and spills.  The team program instead spreads the work of one
(event, helicity) over a team of T lanes:

  * every current, row/column spinor and amplitude of the plan is an "op" of
    one routine class (ggg vertex, gggg vertex, quark-gluon vertex on a row or
    on a column, top propagator on a row or a column, top-line gluon current,
    amplitude contraction);
  * ops are scheduled into passes: a pass runs up to T ready ops of one class,
    lane i taking op i, so all lanes execute the same routine on their own
    operands; the pass order follows the plan's emission order, which keeps
    the number of live objects small;
  * objects live in a frame in LDS (one slot of four complex numbers each);
    slots are reused once their last reader has run; momenta are read from a
    per-event table of signed momentum sums, also in LDS;
  * each pass of amplitudes is followed by a pass in which every lane adds
    the amplitudes to the colour flows it owns (flow k belongs to lane k mod T
    and lives in that lane's registers) with their coefficients in
    {+1, -1, +i, -i};
  * the colour sum: the flows go to LDS, lane t forms
    sum_j CF_ij Re(conj(J_i) J_j) for its rows i, and the team reduces.

Operand tables are uint16 arrays laid out [operand][T] per pass, so that the
lanes of a pass read them coalesced.  This module only plans and emits code;
the kernel that runs it is csrc/me_team.h.
"""
from __future__ import annotations

import collections
import heapq

from .colour import colour_matrix
from .topology import Plan

T_DEFAULT = 32


def team_width(n):
    """Lanes per team: 64 (one team per wavefront) when the program has enough
    parallel ops per step, else 32."""
    return 64 if n >= 5 else 32


def team_window(n):
    """How far (in emission order) a step may reach ahead of its earliest op:
    bounded for the largest programs, where it cuts the LDS frame by a quarter
    at a few per cent of lane use."""
    return 4096 if n >= 6 else None
NONE = 0xFFFF
MSTRIDE = 5     # doubles between momentum-table entries (must match me_team.h)
LDS_BYTES = 160 * 1024   # LDS of one compute unit


def slot_particle(slot):
    return slot if slot < 2 else slot + 2


# V4 colour structures: two terms (sign, a, b, c, d) = sign g^{ab} g^{cd} over legs 0..3
_V4_TERMS = {0: ((1, 0, 2, 1, 3), (-1, 0, 3, 1, 2)),
             1: ((1, 0, 1, 2, 3), (-1, 0, 3, 1, 2)),
             2: ((1, 0, 1, 2, 3), (-1, 0, 2, 1, 3))}


def v4_terms(s, hole, legs):
    """(partner, dot_x, dot_y) per term of the gggg vertex with leg `hole` open."""
    out = []
    for sg, a, b, c, d in _V4_TERMS[s]:
        if a == hole or b == hole:
            partner = b if a == hole else a
            x, y = c, d
        else:
            partner = d if c == hole else c
            x, y = a, b
        out.append((sg, legs[partner], legs[x], legs[y]))
    assert out[0][0] == 1 and out[1][0] == -1
    return out


class TeamProgram:
    """Passes, slot assignment and tables of one process for a team of T lanes."""

    CLASSES = ('V3', 'V4', 'ROWV', 'VCOL', 'ROWP', 'PCOL', 'LINE', 'AMP')
    NOPER = {'V3': 6, 'V4': 8, 'ROWV': 3, 'VCOL': 3, 'ROWP': 3, 'PCOL': 3, 'LINE': 3, 'AMP': 3}

    def __init__(self, name, plan: Plan, T=T_DEFAULT, window=None):
        self.name = name
        self.plan = plan
        self.T = T
        self.window = window if window is not None else 1 << 30
        self.n = plan.n
        self.npar = self.n + 2
        self.ncol = len(plan.basis)
        self.moms = {}        # particle mask -> momentum table index
        self.ops = {}         # key -> (class, operand spec)
        self.ext = []         # (key, kind, particle, outgoing)
        self.amp_info = {}    # amp op key -> [(flow, coefficient)]
        self._build_ops()
        self._schedule()
        self._allocate()

    # ------------------------------------------------------------ momenta
    def gmask(self, gluon_mask):
        m = 0
        for s in range(self.n):
            if gluon_mask >> s & 1:
                m |= 1 << slot_particle(s)
        return m

    def mom(self, pmask, neg=False):
        """Operand code of +-(sum of signed momenta k_q over the particles of pmask)."""
        if pmask not in self.moms:
            self.moms[pmask] = len(self.moms)
        return self.moms[pmask] | (0x8000 if neg else 0)

    # ------------------------------------------------------------ ops
    def _build_ops(self):
        plan = self.plan
        tm = plan.trees.mask
        for key in plan.order:
            kind = key[0]
            if kind == 'G':
                s = key[1]
                self.ext.append((key, 'G', slot_particle(s), int(s >= 2)))
            elif kind == 'U':
                self.ext.append((key, 'U', 2, 1))
            elif kind == 'V':
                self.ext.append((key, 'V', 3, 1))
            elif kind == 'J':
                node = plan.trees.nodes[key[1]]
                if node[0] == 'v3':
                    a, b = node[1], node[2]
                    ma, mb = self.gmask(tm[a]), self.gmask(tm[b])
                    self.ops[key] = ('V3', [plan.jkey(a), self.mom(ma), plan.jkey(b), self.mom(mb),
                                            self.mom(ma | mb)])
                else:
                    s, a, b, c = node[1], node[2], node[3], node[4]
                    legs = [None, plan.jkey(a), plan.jkey(b), plan.jkey(c)]
                    t = v4_terms(s, 0, legs)
                    self.ops[key] = ('V4', [t[0][1], t[0][2], t[0][3], t[1][1], t[1][2], t[1][3],
                                            self.mom(self.gmask(tm[key[1]]))])
            elif kind == 'Lh':
                seq = key[1]
                prev = ('L', seq[:-1]) if len(seq) > 1 else ('U',)
                self.ops[key] = ('ROWV', [prev, plan.jkey(seq[-1])])
            elif kind == 'L':
                seq = key[1]
                m = 0
                for t in seq:
                    m |= tm[t]
                # q = p3 - P = -(k_t + P) with k_t = -p3 the signed top momentum
                self.ops[key] = ('ROWP', [('Lh', seq), self.mom(self.gmask(m) | (1 << 2), neg=True)])
            elif kind == 'Rh':
                seq = key[1]
                nxt = ('R', seq[1:]) if len(seq) > 1 else ('V',)
                self.ops[key] = ('VCOL', [plan.jkey(seq[0]), nxt])
            elif kind == 'R':
                seq = key[1]
                m = 0
                for t in seq:
                    m |= tm[t]
                # q = P - p4 = P + k_tbar
                self.ops[key] = ('PCOL', [('Rh', seq), self.mom(self.gmask(m) | (1 << 3))])
            elif kind == 'K':
                left = ('L', key[1]) if key[1] else ('U',)
                right = ('R', key[2]) if key[2] else ('V',)
                self.ops[key] = ('LINE', [left, right])
            elif kind == 'KD':
                pre, suf, steps = key[1], key[2], key[3]
                parent = ('KD', pre, suf, steps[:-1]) if len(steps) > 1 else ('K', pre, suf)
                vkind, s, hole, sibs = steps[-1]
                tmask = self.gmask(plan.hole_mask(key))
                if vkind == 'v3':
                    sib = plan.jkey(sibs[0])
                    psib = self.mom(self.gmask(tm[sibs[0]]))
                    pn = self.mom(tmask, neg=True)
                    if hole == 1:
                        spec = [sib, psib, parent, pn]
                    else:
                        spec = [parent, pn, sib, psib]
                    self.ops[key] = ('V3', spec + [self.mom(tmask)])
                else:
                    legs = [parent]
                    it = iter(plan.jkey(t) for t in sibs)
                    for leg in range(1, 4):
                        legs.append(None if leg == hole else next(it))
                    t = v4_terms(s, hole, legs)
                    self.ops[key] = ('V4', [t[0][1], t[0][2], t[0][3], t[1][1], t[1][2], t[1][3],
                                            self.mom(tmask)])
            else:
                raise KeyError(key)
        # amplitudes in the plan's group order; a quark-gluon vertex amplitude
        # first forms the row L (i g gamma.J) as a temporary
        self.amp_order = []
        for gi, (ckey, members) in enumerate(plan.scheduled_groups()):
            for lead, amp in members:
                objs = amp[1:]
                akey = ('A', len(self.amp_order))
                if len(objs) == 3:
                    tkey = ('T', len(self.amp_order))
                    self.ops[tkey] = ('ROWV', [objs[0], objs[1]])
                    self.ops[akey] = ('AMP', [tkey, objs[2], 0])
                else:
                    metric = 1 if objs[0][0] in ('K', 'KD') else 0
                    self.ops[akey] = ('AMP', [objs[0], objs[1], metric])
                self.amp_info[akey] = [(k, complex(lead) * complex(rel)) for k, rel in ckey]
                self.amp_order.append(akey)

    def deps(self, key):
        cls, spec = self.ops[key]
        return [x for x in spec if isinstance(x, tuple)]

    # ------------------------------------------------------------ scheduling
    def _rank(self):
        order = []
        seen = set(k for k, *_ in self.ext)

        def need(k):
            if k in seen:
                return
            for d in self.deps(k):
                need(d)
            seen.add(k)
            order.append(k)

        for akey in self.amp_order:
            need(akey)
        return {k: i for i, k in enumerate(order)}

    def _schedule(self):
        rank = self._rank()
        users = collections.defaultdict(list)
        indeg = {}
        for k in self.ops:
            ds = [d for d in self.deps(k) if d in self.ops]
            indeg[k] = len(ds)
            for d in ds:
                users[d].append(k)
        # per class a heap of ready ops by rank; each step takes the class whose
        # earliest ready op comes first in the emission order
        ready = collections.defaultdict(list)
        for k in self.ops:
            if indeg[k] == 0:
                heapq.heappush(ready[self.ops[k][0]], (rank[k], k))
        passes = []
        done = 0
        while done < len(self.ops):
            cls = min((c for c in ready if ready[c]), key=lambda c: ready[c][0][0])
            heap = ready[cls]
            # ops far ahead of the earliest ready one would stretch live ranges
            limit = heap[0][0] + self.window
            batch = []
            while heap and len(batch) < self.T and heap[0][0] <= limit:
                batch.append(heapq.heappop(heap)[1])
            passes.append((cls, batch))
            for k in batch:
                done += 1
                for u in users[k]:
                    indeg[u] -= 1
                    if indeg[u] == 0:
                        heapq.heappush(ready[self.ops[u][0]], (rank[u], u))
        self.passes = passes

    def _allocate(self):
        """Slots for externals and op outputs; a slot is reused after its last reader's pass."""
        last = {}
        for pi, (cls, batch) in enumerate(self.passes):
            for k in batch:
                for d in self.deps(k):
                    last[d] = pi
        slot = {}
        free = []
        nslot = 0

        def get():
            nonlocal nslot
            if free:
                return free.pop()
            nslot += 1
            return nslot - 1

        for key, *_ in self.ext:
            slot[key] = get()
        for pi, (cls, batch) in enumerate(self.passes):
            if cls != 'AMP':
                for k in batch:
                    slot[k] = get()
            dead = set()
            for k in batch:
                for d in self.deps(k):
                    if last.get(d) == pi:
                        dead.add(d)
            free.extend(slot[d] for d in dead)
            # objects nobody reads (none expected) are released at once
            for k in batch:
                if cls != 'AMP' and k not in last:
                    free.append(slot[k])
            free.sort(reverse=True)
        self.slot = slot
        self.nslot = max(nslot, 1)

    # ------------------------------------------------------------ tables
    def tables(self):
        """Operand rows, flow words and step records.

        ops:   uint16, one row of 8 operands per lane per step (rows padded to T
               per step, unused operands 0), so that a lane reads its operands
               of a step with one 16-byte load;
        flows: uint32 records per AMP step, laid out [record][lane] (see
               _flow_records);
        steps: (class, n, first row, record offset, records per lane).
        """
        T = self.T
        ops, flows, steps = [], [], []
        nloc = (self.ncol + T - 1) // T
        for cls, batch in self.passes:
            row0 = len(ops) // 8
            for i in range(T):
                if i < len(batch):
                    k = batch[i]
                    spec = self.ops[k][1]
                    if cls == 'AMP':
                        a, b, metric = spec
                        row = [self.slot[a], self.slot[b], metric]
                    else:
                        row = [self.slot[x] if isinstance(x, tuple) else x for x in spec] + [self.slot[k]]
                    assert len(row) == self.NOPER[cls], (cls, row)
                else:
                    row = []
                ops += row + [0] * (8 - len(row))
            rec = {'cls': cls, 'n': len(batch), 'row': row0, 'foff': 0, 'mw': 0}
            if cls == 'AMP':
                rec['foff'], rec['mw'] = len(flows), self._flow_records(batch, flows)
            steps.append(rec)
        return ops, flows, steps

    def _flow_records(self, batch, flows):
        """Colour-flow records of one amplitude step; returns records per lane.

        Every flow touched by the step is given to one lane (longest lists
        first, to the least loaded lane), so no two lanes update one flow.  A
        lane's records are sorted by flow: 4 * amp lane + coefficient (bits
        0-7; coefficient 0: +1, 1: -1, 2: +i, 3: -i, the amplitude step stores
        all four products), flow (bits 8-19), bit 20 set on the last record of
        a flow (the lane then adds its running sum to the flow in LDS).
        Padding records are 0xFFFFFFFF.
        """
        T = self.T
        per_flow = collections.defaultdict(list)
        for i, akey in enumerate(batch):
            for k, c in self.amp_info[akey]:
                code = {1: 0, -1: 1, 1j: 2, -1j: 3}[complex(round(c.real), round(c.imag))]
                per_flow[k].append((i << 2) | code)
        load = [0] * T
        lanes = [[] for _ in range(T)]
        free = [(0, t) for t in range(T)]
        for k in sorted(per_flow, key=lambda k: (-len(per_flow[k]), k)):
            _, t = heapq.heappop(free)
            ents = per_flow[k]
            for n, e in enumerate(ents):
                lanes[t].append(e | (k << 8) | ((1 << 20) if n == len(ents) - 1 else 0))
            load[t] += len(ents)
            heapq.heappush(free, (load[t], t))
        assert self.ncol < (1 << 12)
        r = max(load)
        for q in range(r):
            for t in range(T):
                flows.append(lanes[t][q] if q < len(lanes[t]) else 0xFFFFFFFF)
        return r

    def stats(self):
        util = sum(len(b) for _, b in self.passes) / (self.T * len(self.passes))
        return {'ops': len(self.ops), 'passes': len(self.passes), 'lane_util': util,
                'slots': self.nslot, 'momenta': len(self.moms)}


CLASS_ID = {'V3': 0, 'V4': 1, 'ROWV': 2, 'VCOL': 3, 'ROWP': 4, 'PCOL': 5, 'LINE': 6, 'AMP': 7, 'FLOWS': 8}


def emit(name, plan, T=None):
    """HIP source of struct me::<name>_team (the team program of the process)."""
    T = T or team_width(plan.n)
    prog = TeamProgram(name, plan, T, team_window(plan.n))
    ops, flows, steps = prog.tables()
    cf, den = colour_matrix(plan.n)
    ncol = prog.ncol
    npar = prog.npar
    nmom = len(prog.moms)
    nloc = (ncol + T - 1) // T
    # frame layout (doubles): slots SLOT doubles apart | colour flows | momentum
    # table (MSTRIDE doubles apart) | external momenta | amplitude buffer.  SLOT is
    # 9 (an odd number of 8-byte words spreads the lanes over the LDS banks),
    # or 8 when that lets one more workgroup fit in a compute unit's LDS.
    def layout(slot):
        joff = prog.nslot * slot
        moff = joff + 2 * ncol
        poff = moff + nmom * MSTRIDE
        aoff = poff + npar * 4
        return joff, moff, poff, aoff, aoff + T * 8

    teams = 64 // T
    per_cu = {sl: LDS_BYTES // (teams * 8 * layout(sl)[4]) for sl in (9, 8)}
    slot = 8 if per_cu[8] > per_cu[9] else 9
    joff, moff, poff, aoff, frame = layout(slot)
    words = []
    for r in steps:
        words += [CLASS_ID[r['cls']] | (r['n'] << 8), r['row']]
        if r['cls'] == 'AMP':
            words += [r['foff'], r['mw']]
    fmaxw = max((r['mw'] for r in steps), default=1)
    assert max(ops, default=0) <= 0xFFFF
    L = []
    st = prog.stats()
    L.append(f"// Team program of {name}: {st['ops']} ops in {st['passes']} steps of up to {T} lanes "
             f"(lane use {st['lane_util']:.2f}),")
    L.append(f"// {prog.nslot} object slots, {nmom} momentum sums; LDS frame {frame * 8} bytes.")
    L.append("namespace me {")
    L.append(f"alignas(16) static __device__ const uint16_t TEAMOPS_{name}[{max(8, len(ops))}] = {{"
             + ', '.join(str(v) for v in ops) + "};")
    L.append(f"static __device__ const uint32_t TEAMFLOW_{name}[{max(1, len(flows))}] = {{"
             + ', '.join(f'{v}u' for v in flows) + "};")
    L.append(f"static __device__ const uint32_t TEAMPROG_{name}[{len(words)}] = {{"
             + ', '.join(str(v) for v in words) + "};")
    masks = sorted(prog.moms.items(), key=lambda kv: kv[1])
    L.append(f"static __device__ const uint16_t TEAMMOM_{name}[{nmom}] = {{"
             + ', '.join(str(m) for m, _ in masks) + "};")
    flat = ', '.join(str(cf[j][i]) for j in range(ncol) for i in range(ncol))
    L.append(f"static __device__ const int32_t TEAMCF_{name}[{ncol * ncol}] = {{{flat}}};")
    L.append(f"struct {name}_team {{")
    L.append(f'  static constexpr const char* NAME = "{name}";')
    for k, v in (('T', T), ('SLOT', slot), ('NPAR', npar), ('NCOL', ncol), ('NLOC', nloc), ('NMOM', nmom),
                 ('JOFF', joff),
                 ('MOFF', moff), ('POFF', poff), ('AOFF', aoff), ('FRAME', frame), ('NPROGW', len(words)),
                 ('NEXT', len(prog.ext)), ('RMAX', fmaxw)):
        L.append(f"  static constexpr int {k} = {v};")
    L.append(f"  static __device__ __forceinline__ const uint16_t* ops() {{ return TEAMOPS_{name}; }}")
    L.append(f"  static __device__ __forceinline__ const uint32_t* flows() {{ return TEAMFLOW_{name}; }}")
    L.append(f"  static __device__ __forceinline__ const uint32_t* program() {{ return TEAMPROG_{name}; }}")
    L.append(f"  static __device__ __forceinline__ const uint16_t* momentum_masks() {{ return TEAMMOM_{name}; }}")
    L.append(f"  static __device__ __forceinline__ const int32_t* colour_matrix() {{ return TEAMCF_{name}; }}")
    L.append("  // external states: lane t < NEXT computes external state t of the frame")
    L.append("  static __device__ __forceinline__ void externals(double* F, int t, int hel, double mt) {")
    L.append("    switch (t) {")
    for i, (key, kind, q, outgoing) in enumerate(prog.ext):
        kid = {'U': 0, 'V': 1, 'G': 2}[kind]
        L.append(f"      case {i}: team_external<{kid}, {q}, {outgoing}, NPAR, SLOT>(F, POFF, {prog.slot[key]}, hel, mt); "
                 "break;")
    L.append("      default: break;")
    L.append("    }")
    L.append("  }")
    L.append("};")
    L.append("}  // namespace me")
    return '\n'.join(L) + '\n', prog
