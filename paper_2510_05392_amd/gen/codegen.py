"""Emit HIP device code for one process from its evaluation plan.

The emitted header defines, for process <name>:

  constexpr int NPAR, NCOL, NHEL, IDEN, CF_DEN
  __device__ void amplitudes(p, lam, g, mt, jamp)   -- one (event, helicity):
        external states, currents and amplitudes of every diagram piece,
        accumulated into the dual amplitudes jamp[NCOL]
  __device__ double colour_sum(jamp)                 -- sum_ij CF_int[i][j] Re(J_i^* J_j)
                                                        (triangular: off-diagonal terms
                                                        once, doubled), not yet / CF_DEN
  CF_INT[NCOL*NCOL] (host table)
  __device__ void group_sums_part<K>(p, lam, g, mt, sout, sstride)
                                                     -- split executor: the colour-group
        sums of one (event, helicity) in part K of the groups, stored instead of
        accumulated into flows
  __device__ void flow_chunk(w, c, b, acc)           -- split executor: wave w's share of
        the flow updates from chunk c of group sums staged in LDS

Everything is straight-line code: the generator has already resolved the
diagram structure, so the compiler sees fixed register operands.
"""
from __future__ import annotations

import math

from . import team as team_gen
from .colour import colour_matrix
from .topology import Plan

PROCESS_NPAR = {'gg_ttx': 4, 'gg_ttxg': 5, 'gg_ttxgg': 6, 'gg_ttxggg': 7, 'gg_ttxgggg': 8}


def slot_particle(slot):
    return slot if slot < 2 else slot + 2


def _cx(c):
    """(re, im) of a colour coefficient in {+-1, +-i}."""
    c = complex(c)
    return int(round(c.real)), int(round(c.imag))


class Emitter:
    def __init__(self, name, plan: Plan, remat=False):
        """remat: recompute each momentum sum from the external momenta at every use
        (through an opaque copy, so that the compiler keeps them apart) instead of
        keeping it live from its first use."""
        self.name = name
        self.plan = plan
        self.remat = remat
        self.nremat = 0
        self.n = plan.n
        self.npar = self.n + 2
        self.lines = []
        self.names = {}
        self.masks_done = set()
        self.neg_done = set()
        self.basis_index = {p: i for i, p in enumerate(plan.basis)}
        # FP64 operations of the code written so far, one (event, helicity)
        from .. import flops
        self.fl = flops
        self.ops = 0

    def var(self, key):
        if key not in self.names:
            self.names[key] = f"w{len(self.names)}"
        return self.names[key]

    def mom(self, mask):
        """Name of the momentum flowing into the diagram through the gluons of `mask`."""
        name = f"P{mask}"
        if self.remat and bin(mask).count('1') == 1 and (mask & 3):
            return f"p[{slot_particle(mask.bit_length() - 1)}]"   # an incoming momentum itself
        if self.remat:
            self.nremat += 1
            name = f"P{mask}_{self.nremat}"
        elif mask in self.masks_done:
            return name
        self.masks_done.add(mask)
        terms = []
        for s in range(self.n):
            if mask >> s & 1:
                sign = '+' if s < 2 else '-'
                terms.append((sign, slot_particle(s)))
        comps = []
        for u in range(4):
            expr = ''.join(f" {sg} p[{q}][{u}]" for sg, q in terms).strip()
            if expr.startswith('+ '):
                expr = expr[2:]
            elif expr.startswith('- '):
                expr = '-' + expr[2:]
            if self.remat:
                # the first term through an opaque copy: no two sums are merged
                first = f"p[{terms[0][1]}][{u}]"
                expr = expr.replace(first, f"opaque({first})", 1)
            comps.append(expr)
        self.lines.append(f"  const double {name}[4] = {{{', '.join(comps)}}};")
        self.ops += self.fl.momentum_sum(len(terms))
        return name

    def tree_mask(self, t):
        return self.plan.trees.mask[t]

    def seq_mask(self, seq):
        m = 0
        for t in seq:
            m |= self.tree_mask(t)
        return m

    def emit_object(self, key):
        kind = key[0]
        out = self.var(key)
        L = self.lines
        if kind == 'G':
            s = key[1]
            q = slot_particle(s)
            outgoing = 'true' if s >= 2 else 'false'
            L.append(f"  cx {out}[4]; ext_gluon(p[{q}], lam[{q}], {outgoing}, {out});")
            self.ops += self.fl.ROUTINE['Gbeam' if s < 2 else 'G']
        elif kind == 'U':
            L.append(f"  cx {out}[4]; ext_ubar(p[2], lam[2], mt, {out});")
            self.ops += self.fl.ROUTINE['U']
        elif kind == 'V':
            L.append(f"  cx {out}[4]; ext_v(p[3], lam[3], mt, {out});")
            self.ops += self.fl.ROUTINE['V']
        elif kind == 'J':
            node = self.plan.trees.nodes[key[1]]
            if node[0] == 'v3':
                a, b = node[1], node[2]
                pa, pb = self.mom(self.tree_mask(a)), self.mom(self.tree_mask(b))
                va, vb = self.var(self.plan.jkey(a)), self.var(self.plan.jkey(b))
                L.append(f"  cx {out}[4]; v3_current({va}, {pa}, {vb}, {pb}, g, {out});")
                self.ops += self.fl.ROUTINE['v3']
            else:
                s, a, b, c = node[1], node[2], node[3], node[4]
                pm = self.mom(self.tree_mask(key[1]))
                va, vb, vc = (self.var(self.plan.jkey(x)) for x in (a, b, c))
                L.append(f"  cx {out}[4]; v4_current<{s}>({va}, {vb}, {vc}, {pm}, g, {out});")
                self.ops += self.fl.ROUTINE['v4']
        elif kind == 'Lh':
            seq = key[1]
            prev = self.var(('L', seq[:-1]) if len(seq) > 1 else ('U',))
            j = self.var(self.plan.jkey(seq[-1]))
            L.append(f"  cx {out}[4]; row_vertex({prev}, {j}, g, {out});")
            self.ops += self.fl.ROUTINE['Lh']
        elif kind == 'L':
            seq = key[1]
            pm = self.mom(self.seq_mask(seq))
            src = self.var(('Lh', seq))
            # momentum along the fermion arrow: p3 - P(seq)
            L.append(f"  cx {out}[4]; {{ const double q[4] = {{p[2][0] - {pm}[0], p[2][1] - {pm}[1], "
                     f"p[2][2] - {pm}[2], p[2][3] - {pm}[3]}}; row_prop({src}, q, mt, {out}); }}")
            self.ops += self.fl.OPS['qsub'] + self.fl.ROUTINE['L']
        elif kind == 'Rh':
            seq = key[1]
            nxt = self.var(('R', seq[1:]) if len(seq) > 1 else ('V',))
            j = self.var(self.plan.jkey(seq[0]))
            L.append(f"  cx {out}[4]; vertex_col({j}, {nxt}, g, {out});")
            self.ops += self.fl.ROUTINE['Rh']
        elif kind == 'R':
            seq = key[1]
            pm = self.mom(self.seq_mask(seq))
            src = self.var(('Rh', seq))
            # momentum along the fermion arrow: P(seq) - p4
            L.append(f"  cx {out}[4]; {{ const double q[4] = {{{pm}[0] - p[3][0], {pm}[1] - p[3][1], "
                     f"{pm}[2] - p[3][2], {pm}[3] - p[3][3]}}; prop_col(q, mt, {src}, {out}); }}")
            self.ops += self.fl.OPS['qsub'] + self.fl.ROUTINE['R']
        elif kind == 'K':
            left = self.var(('L', key[1]) if key[1] else ('U',))
            right = self.var(('R', key[2]) if key[2] else ('V',))
            L.append(f"  cx {out}[4]; line_current({left}, {right}, g, {out});")
            self.ops += self.fl.ROUTINE['K']
        elif kind == 'KD':
            self.emit_kd(key, out)
        else:
            raise KeyError(key)

    def negmom(self, mask):
        name = f"N{mask}"
        if self.remat:
            self.nremat += 1
            name = f"N{mask}_{self.nremat}"
        elif mask in self.neg_done:
            return name
        self.neg_done.add(mask)
        pm = self.mom(mask)
        self.lines.append(f"  const double {name}[4] = {{-{pm}[0], -{pm}[1], -{pm}[2], -{pm}[3]}};")
        return name

    def emit_kd(self, key, out):
        """Top-line current carried through one more gluon vertex (the last step)."""
        pre, suf, steps = key[1], key[2], key[3]
        parent = self.var(('KD', pre, suf, steps[:-1]) if len(steps) > 1 else ('K', pre, suf))
        kind, s, hole, sibs = steps[-1]
        tmask = self.plan.hole_mask(key)             # subtree below the parent line
        npt = self.negmom(tmask)                      # incoming momentum of the parent leg
        sib_vars = [self.var(self.plan.jkey(t)) for t in sibs]
        sib_moms = [self.mom(self.tree_mask(t)) for t in sibs]
        f = f"(-g / msq({self.mom(tmask)}))" if kind == 'v3' else f"(-g * g / msq({self.mom(tmask)}))"
        self.ops += self.fl.ROUTINE['msq'] + self.fl.OPS['kd3_factor' if kind == 'v3' else 'kd4_factor']
        self.ops += self.fl.ROUTINE['KD3' if kind == 'v3' else 'KD4']
        if kind == 'v3':
            # legs (parent, A, B); the two given legs in cyclic order after the open one
            if hole == 1:
                args = f"{sib_vars[0]}, {sib_moms[0]}, {parent}, {npt}"
            else:
                args = f"{parent}, {npt}, {sib_vars[0]}, {sib_moms[0]}"
            self.lines.append(f"  cx {out}[4]; v3_open({args}, {f}, {out});")
        else:
            legs = [parent]
            it = iter(sib_vars)
            for leg in range(1, 4):
                legs.append('nullptr' if leg == hole else next(it))
            self.lines.append(f"  cx {out}[4]; v4_open<{s}, {hole}>({', '.join(legs)}, {f}, {out});")

    def amp_expr(self, objs):
        """(setup lines, expression) of one amplitude contraction."""
        if len(objs) == 3:
            # quark-gluon vertex amplitude  L (i g gamma.J) R
            left, j, right = (self.var(o) for o in objs)
            self.ops += self.fl.ROUTINE['Lh'] + self.fl.ROUTINE['sdot']
            return [f"cx t[4]; row_vertex({left}, {j}, g, t);"], f"sdot(t, {right})"
        va, vb = self.var(objs[0]), self.var(objs[1])
        op = 'vdot' if objs[0][0] in ('K', 'KD') else 'sdot'
        self.ops += self.fl.ROUTINE[op]
        return [], f"{op}({va}, {vb})"

    @staticmethod
    def _scaled(expr, c):
        """expr times a unit c in {+-1, +-i}, as (sign, expression)."""
        re, im = _cx(c)
        if re == 1:
            return '+', expr
        if re == -1:
            return '-', expr
        if im == 1:
            return '+', f"times_i({expr})"
        if im == -1:
            return '-', f"times_i({expr})"
        raise ValueError(c)

    def amplitudes(self, split=False, groups=None):
        """Pieces sharing one colour vector (up to a unit factor) are summed first,
        then the sum is added once to each of its colour flows.  With split set the
        sum of group gi is stored to sout[2 gi sstride] (real) and
        sout[(2 gi + 1) sstride] (imaginary) instead, and the flows are formed by
        flow_chunks() in a second kernel; groups (a range of group indices) then
        restricts the code to those groups and the currents they need."""
        done = set()

        def need(key):
            if key in done:
                return
            for d in self.plan.objects[key]:
                need(d)
            self.emit_object(key)
            done.add(key)

        order = self.plan.split_groups() if split else self.plan.scheduled_groups()
        for gi, (key, members) in enumerate(order):
            if groups is not None and gi not in groups:
                continue
            first_lead = members[0][0]
            acc = f"s{gi}"
            for n_m, (lead, amp) in enumerate(members):
                for o in amp[1:]:
                    need(o)
                setup, expr = self.amp_expr(amp[1:])
                sign, term = self._scaled('a', lead / first_lead)
                head = "  { " + ' '.join(setup) + f" const cx a = {expr}; "
                if n_m == 0:
                    assert sign == '+' and term == 'a'
                    self.lines.append(f"  cx {acc};")
                    self.lines.append(head + f"{acc} = a; }}")
                else:
                    self.lines.append(head + f"{acc} = {acc} {sign} {term}; }}")
                    self.ops += self.fl.OPS['cadd']
            if split:
                self.lines.append(f"  sout[{2 * gi} * sstride] = {acc}.r; sout[{2 * gi + 1} * sstride] = {acc}.i;")
                continue
            # distribute the group sum over its colour flows
            for k, rel in key:
                sign, term = self._scaled(acc, rel * first_lead)
                self.lines.append(f"  jamp[{k}] = jamp[{k}] {sign} {term};")
                self.ops += self.fl.OPS['cadd']
        return self.lines

    def channel_sums(self, channel_of_piece):
        """Single-diagram-enhancement sums of one (event, helicity): for every diagram
        built from three-point vertices only (a channel, numbered by
        channel_of_piece), |A|^2 of its Lorentz amplitude (colour coefficients
        +-1, +-i, so |A|^2 is the diagram's own) is added to *den, and to *num when
        the channel is `chan`.  Only the currents these diagrams need are made."""
        done = set()

        def need(key):
            if key in done:
                return
            for d in self.plan.objects[key]:
                need(d)
            self.emit_object(key)
            done.add(key)

        for key, members in self.plan.scheduled_groups():
            for lead, amp in members:
                cid = channel_of_piece.get(amp[0])
                if cid is None:
                    continue
                for o in amp[1:]:
                    need(o)
                setup, expr = self.amp_expr(amp[1:])
                self.lines.append("  { " + ' '.join(setup) + f" const cx a = {expr}; "
                                  f"const double q = a.r * a.r + a.i * a.i; *den += q; "
                                  f"*num += chan == {cid} ? q : 0.0; }}")
                self.ops += self.fl.OPS['channel']
        return self.lines

    def flow_chunks(self, nwave, chunk):
        """Flows formed from group sums staged through LDS, chunk by chunk: wave w of
        the workgroup owns flows [w fpw, (w + 1) fpw) and keeps them in acc
        (acc[2 lk] real, acc[2 lk + 1] imaginary part of local flow lk); chunk c holds
        groups [c chunk, (c + 1) chunk) of the order amplitudes() stores them in, group
        c chunk + gl at b[2 gl 64] (real) and b[(2 gl + 1) 64] (imaginary)."""
        groups = self.plan.split_groups()
        fpw = -(-len(self.plan.basis) // nwave)
        nch = -(-len(groups) // chunk)
        lines = [f"  switch (w * {nch} + c) {{"]
        for w in range(nwave):
            for c in range(nch):
                body = []
                for gl, (key, members) in enumerate(groups[c * chunk:(c + 1) * chunk]):
                    mine = [(k, rel) for k, rel in key if k // fpw == w]
                    if not mine:
                        continue
                    first_lead = members[0][0]
                    body.append(f"    {{ const double sr = b[{2 * gl * 64}], si = b[{(2 * gl + 1) * 64}];")
                    for k, rel in mine:
                        lk = k - w * fpw
                        re_, im_ = _cx(rel * first_lead)
                        if re_:
                            op = '+' if re_ > 0 else '-'
                            body.append(f"      acc[{2 * lk}] {op}= sr; acc[{2 * lk + 1}] {op}= si;")
                        else:
                            # (sr + i si) times +-i = -+si +- i sr
                            op, nop = ('+', '-') if im_ > 0 else ('-', '+')
                            body.append(f"      acc[{2 * lk}] {nop}= si; acc[{2 * lk + 1}] {op}= sr;")
                    body.append("    }")
                if body:
                    lines.append(f"  case {w * nch + c}: {{")
                    lines.extend(body)
                    lines.append("    break; }")
        lines.append("  default: break;")
        lines.append("  }")
        return lines


def colour_sum_code(cf, ncol):
    lines = ["  double acc = 0.0;"]
    for i in range(ncol):
        tr = [f"{cf[i][i]}.0 * jamp[{i}].r"]
        ti = [f"{cf[i][i]}.0 * jamp[{i}].i"]
        for j in range(i + 1, ncol):
            c = 2 * cf[i][j]
            if c == 0:
                continue
            tr.append(f"{c}.0 * jamp[{j}].r")
            ti.append(f"{c}.0 * jamp[{j}].i")
        lines.append(f"  {{ const double tr = {' + '.join(tr)};")
        lines.append(f"    const double ti = {' + '.join(ti)};")
        lines.append(f"    acc += jamp[{i}].r * tr + jamp[{i}].i * ti; }}")
    lines.append("  return acc;")
    return lines


# Staged flow formation of the split executor: waves per workgroup (each owns a
# contiguous quarter of the colour flows) and colour groups per LDS chunk.
FLOW_WAVES = 4
FLOW_CHUNK = 16
# chunk sizes compiled for the autotuner (each a flow_chunk_<CH> function)
FLOW_CHUNKS = (8, 16, 32)
# waves per SIMD of the group-sum kernel variants compiled for the autotuner
SUMS_WPE_VARIANTS = (1, 2)

# Split executor's group-sum kernels: the groups (in scheduled order) are cut into
# SUMS_PARTS contiguous ranges, one kernel each, each computing only the currents
# its groups need (currents shared between ranges are recomputed: fewer live
# currents per kernel, less spill traffic); SUMS_WPE waves per SIMD for them.
SUMS_PARTS = {}
SUMS_WPE = {'gg_ttxggg': 2}
# momentum sums recomputed at each use in the group-sum code (Emitter remat)
SUMS_REMAT = {}

# Largest process that also gets the one-lane-per-(event, helicity) code; beyond
# it the straight-line function would be too large to compile in reasonable
# time, and only the team program is generated.
LANE_MAX_NPAR = 7


def part_ranges(ngroup, nparts):
    return [range(k * ngroup // nparts, (k + 1) * ngroup // nparts) for k in range(nparts)]


def tree_key(trees, t):
    """Canonical string of a gluon tree built from three-point vertices: a leaf is
    its gluon slot number, a vertex "(" + its two children's strings, sorted,
    joined by "," + ")"."""
    node = trees.nodes[t]
    if node[0] == 'leaf':
        return str(node[1])
    assert node[0] == 'v3'
    return '(' + ','.join(sorted((tree_key(trees, node[1]), tree_key(trees, node[2])))) + ')'


def _cubic(trees, t):
    node = trees.nodes[t]
    if node[0] == 'leaf':
        return True
    return node[0] == 'v3' and _cubic(trees, node[1]) and _cubic(trees, node[2])


def channels(plan):
    """{piece index: channel number} for the single-diagram-enhancement channels:
    the diagrams with three-point vertices only, numbered 1..N in ascending order
    of the tuple of their gluon trees' keys taken from the top end of the quark
    line (any numbering serves the method; this one is fixed so that two
    independent enumerations agree)."""
    keyed = sorted((tuple(tree_key(plan.trees, t) for t in piece), i)
                   for i, piece in enumerate(plan.pieces) if all(_cubic(plan.trees, t) for t in piece))
    return {i: c + 1 for c, (_, i) in enumerate(keyed)}


def generate_sde(name, plan=None):
    """Source of the single-diagram-enhancement function of a one-lane process."""
    npar = PROCESS_NPAR[name]
    plan = plan or Plan(npar - 2)
    chan = channels(plan)
    body = Emitter(name, plan).channel_sums(chan)
    out = [f"// Generated for process {name}: single-diagram-enhancement sums over its "
           f"{len(chan)} channels.  Do not edit.",
           "#pragma once", '#include "me_device.h"', "namespace me {", f"struct {name}_sde {{",
           f'  static constexpr const char* NAME = "{name}";',
           f"  static constexpr int NPAR = {npar};",
           f"  static constexpr int NCHAN = {len(chan)};",
           "  static __device__ __forceinline__ void channel_amp2(const double (*p)[4], const int* lam, double g, "
           "double mt, int chan, double* num, double* den) {"]
    out.extend('  ' + l for l in body)
    out += ["  }", "};", "}  // namespace me"]
    return '\n'.join(out) + '\n', len(chan)


def generate(name, sums_parts=None, sums_wpe=None, remat=None):
    npar = PROCESS_NPAR[name]
    remat = SUMS_REMAT.get(name, False) if remat is None else remat
    n = npar - 2
    plan = Plan(n)
    cf, den = colour_matrix(n)
    ncol = len(plan.basis)
    iden = 4 * 64 * math.factorial(npar - 4)
    lane = npar <= LANE_MAX_NPAR
    body = Emitter(name, plan).amplitudes() if lane else []
    ngroup = len(plan.scheduled_groups())
    nparts = sums_parts or SUMS_PARTS.get(name, 1)
    wpe = sums_wpe or SUMS_WPE.get(name, 1)
    parts = [Emitter(name, plan, remat=remat).amplitudes(split=True, groups=r)
             for r in part_ranges(ngroup, nparts)] if lane else []
    assemble = {ch: Emitter(name, plan).flow_chunks(FLOW_WAVES, ch) for ch in FLOW_CHUNKS} if lane else {}
    team_src, _ = team_gen.emit(name, plan)
    out = []
    out.append(f"// Generated for process {name}: {plan.ndiagrams} Feynman diagrams, "
               f"{len(plan.pieces)} colour-structure pieces,")
    out.append(f"// {len(plan.order)} currents, {ncol} colour flows.  Do not edit.")
    out.append("#pragma once")
    out.append('#include "me_device.h"')
    out.append('#include "me_team.h"')
    out.append(team_src.rstrip('\n'))
    out.append("namespace me {")
    flat = ', '.join(str(cf[i][j]) for i in range(ncol) for j in range(ncol))
    out.append(f"static const int CF_INT_{name}[{ncol * ncol}] = {{{flat}}};")
    out.append(f"struct {name} {{")
    out.append(f'  static constexpr const char* NAME = "{name}";')
    out.append(f"  static constexpr int NPAR = {npar};")
    out.append(f"  static constexpr int NCOL = {ncol};")
    out.append(f"  static constexpr int NHEL = {1 << npar};")
    out.append(f"  static constexpr int IDEN = {iden};")
    out.append(f"  static constexpr int CF_DEN = {den};")
    out.append(f"  static constexpr int NDIAG = {plan.ndiagrams};")
    out.append(f"  static const int* cf_int() {{ return CF_INT_{name}; }}")
    out.append(f"  using Team = {name}_team;")
    out.append(f"  static constexpr bool LANE = {'true' if lane else 'false'};")
    if lane:
        out.append("  static __device__ __forceinline__ void amplitudes(const double (*p)[4], const int* lam, "
                   "double g, double mt, cx* jamp) {")
        out.extend('  ' + l for l in body)
        out.append("  }")
        out.append("  static __device__ __forceinline__ double colour_sum(const cx* jamp) {")
        out.extend('  ' + l for l in colour_sum_code(cf, ncol))
        out.append("  }")
        out.append("  // split evaluation: colour-group sums of one (event, helicity), stride sstride")
        out.append(f"  static constexpr int NGROUP = {ngroup};")
        out.append(f"  static constexpr int NPART = {nparts};   // group-sum kernels")
        out.append(f"  static constexpr int SUMS_WPE = {wpe};   // their waves per SIMD")
        for k, lines in enumerate(parts):
            out.append(f"  static __device__ __forceinline__ void group_sums_{k}(const double (*p)[4], const int* lam, "
                       "double g, double mt, double* sout, int64_t sstride) {")
            out.extend('  ' + l for l in lines)
            out.append("  }")
        out.append("  template <int K>")
        out.append("  static __device__ __forceinline__ void group_sums_part(const double (*p)[4], const int* lam, "
                   "double g, double mt, double* sout, int64_t sstride) {")
        for k in range(nparts):
            kw = 'if' if k == 0 else 'else if'
            out.append(f"    {kw} constexpr (K == {k}) group_sums_{k}(p, lam, g, mt, sout, sstride);")
        out.append("  }")
        out.append(f"  static constexpr int FCHUNK = {FLOW_CHUNK};   // group sums per LDS chunk (default)")
        out.append(f"  static constexpr int FPW = {-(-ncol // FLOW_WAVES)};   // colour flows per wave")
        for ch, lines in assemble.items():
            out.append(f"  static __device__ __forceinline__ void flow_chunk_{ch}(int w, int c, const double* b, "
                       "double* acc) {")
            out.extend('  ' + l for l in lines)
            out.append("  }")
        out.append("  // wave w's flow updates from chunk c of CH group sums (CH one of the compiled sizes)")
        out.append("  template <int CH>")
        out.append("  static __device__ __forceinline__ void flow_chunk_t(int w, int c, const double* b, double* acc) {")
        for k, ch in enumerate(FLOW_CHUNKS):
            kw = 'if' if k == 0 else 'else if'
            out.append(f"    {kw} constexpr (CH == {ch}) flow_chunk_{ch}(w, c, b, acc);")
        out.append("  }")
        out.append("  static __device__ __forceinline__ void flow_chunk(int w, int c, const double* b, double* acc) {")
        out.append("    flow_chunk_t<FCHUNK>(w, c, b, acc);")
        out.append("  }")
    out.append("};")
    out.append("}  // namespace me")
    return '\n'.join(out) + '\n', plan, (cf, den)
