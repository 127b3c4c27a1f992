"""Algorithmic FP64 work of one (event, helicity) of the generated path.

Counting rules: every real addition, subtraction, multiplication, division and
square root the device code writes is one flop; negation and the factor i are
free.  ROUTINE holds the count of one call of each device routine
(csrc/me_device.h) and OPS the counts of the arithmetic the generator writes
inline; the generator's Emitter adds them up as it writes a process's code, so
a process's figure is exactly the operations its code performs (beam gluons
along +-z take the branch without the azimuth divisions, as in every event of
the workloads).  tests/test_generator.py compiles the generated code for the
host with an operation-counting scalar and checks these figures against the
count, routine by routine and process by process.  This is the number the
benchmark's roofline fraction divides by the measured kernel time.
"""
from __future__ import annotations

ROUTINE = {
    'G': 24,          # ext_gluon, momentum with a transverse component
    'Gbeam': 22,      # ext_gluon along +-z (no azimuth divisions)
    'U': 35,          # ext_ubar
    'V': 37,          # ext_v
    'v3': 166,        # v3_current
    'v4': 141,        # v4_current<S>
    'Lh': 80,         # row_vertex
    'Rh': 80,         # vertex_col
    'L': 94,          # row_prop
    'R': 94,          # prop_col
    'K': 80,          # line_current
    'KD3': 154,       # v3_open
    'KD4': 132,       # v4_open<S, H>
    'sdot': 30,       # spinor contraction
    'vdot': 30,       # Minkowski product of complex vectors
    'msq': 7,         # Minkowski square of a real vector
}

OPS = {
    'qsub': 4,        # q = p3 - P or P - p4 before a top propagator
    'kd3_factor': 1,  # -g / P^2 (after msq)
    'kd4_factor': 2,  # -g g / P^2 (after msq)
    'cadd': 2,        # complex addition: a group-sum member, or a colour-flow update
    'channel': 5,     # |A|^2 (3), added to the channel sum (1) and the selected channel (1)
}

# ext_ubar and ext_v take one more division when the top (antitop) has pz < 0
# (|p| + pz formed without cancellation); ROUTINE counts pz >= 0.  Over the
# workloads each of the two is in the backward hemisphere in half of the events,
# so the per-(event, helicity) figures below add the mean, one operation.
QUARK_BRANCH_MEAN = 1


def momentum_sum(nterms):
    """Flops of one four-momentum sum of nterms external momenta."""
    return 4 * (nterms - 1)


def _plan(name):
    from .gen import codegen
    from .gen.topology import Plan
    return Plan(codegen.PROCESS_NPAR[name] - 2)


def colour_sum_flops(cf):
    """Triangular quadratic form sum_ij CF_ij Re(J_i^* J_j) with integer CF as the
    one-lane code writes it: per row i, the products with its diagonal and its
    non-zero entries j > i for the real and imaginary parts, their sums, and the
    row's two products and two additions into the accumulator."""
    n = len(cf)
    total = 0
    for i in range(n):
        nnz = sum(1 for j in range(i + 1, n) if cf[i][j] != 0)
        total += 2 * (2 * nnz + 1) + 4
    return total


def amplitudes_flops(name, plan=None):
    """Dual amplitudes of one (event, helicity): currents, contractions, group sums
    and colour-flow updates of the one-lane code."""
    from .gen import codegen
    plan = plan or _plan(name)
    em = codegen.Emitter(name, plan)
    em.amplitudes()
    return em.ops


def group_sums_flops(name, plan=None):
    """Colour-group sums of one (event, helicity) of the split executor (all parts)."""
    from .gen import codegen
    plan = plan or _plan(name)
    nparts = codegen.SUMS_PARTS.get(name, 1)
    remat = codegen.SUMS_REMAT.get(name, False)
    total = 0
    for r in codegen.part_ranges(len(plan.scheduled_groups()), nparts):
        em = codegen.Emitter(name, plan, remat=remat)
        em.amplitudes(split=True, groups=r)
        total += em.ops
    return total


def per_event_helicity(name):
    plan = _plan(name)
    from .gen.colour import colour_matrix
    cf, _ = colour_matrix(plan.n)
    return amplitudes_flops(name, plan) + colour_sum_flops(cf)


def flow_updates(plan):
    """Colour-flow accumulations (one per (group, flow) pair) of a plan."""
    return sum(len(key) for key, _ in plan.colour_groups())


# Berends-Giele executor (csrc/me_bg.h): counts of its building blocks, read off
# the code at the same rules and pinned, with the totals below, by compiling it
# for the host with the operation-counting scalar (tests/test_generator.py)
BG = {
    'sum_bit': 8,      # one gluon momentum into one subset sum: sign times p, added (4 components)
    'line': 80,        # Q = line_current(ubar, v)
    'v3': 154,         # bg_v3: one split of a three-gluon vertex, accumulated
    'v4': 188,         # bg_v4: one split of a four-gluon vertex, accumulated
    'close': 35,       # 1 / P^2, the two couplings and their combination into the current
    'row_term': 88,    # row_vertex of one block, accumulated
    'row_close': 98,   # q = p3 - P and the top propagator
    'amp_term': 112,   # row_vertex, sdot with v, accumulated
    'q_dot': 30,       # Q . J of a stored current (kept beside it)
    'v3q': 112,        # one split of a three-gluon vertex contracted with Q, accumulated
    'v4q': 116,        # one split of a four-gluon vertex contracted with Q, accumulated
    'qclose': 17,      # 1 / P^2, the couplings and their combination into Q . J(sigma)
    # helicity-recycling kernel (csrc/me_bgh.h): propagator factors of every gluon
    # subset formed once in the set-up, row-vertex sums without their factor i g
    'close_h': 27,     # the couplings and their combination into the current (1 / P^2 read)
    'rg': 64,          # bgh_rg: r . gamma.J, first term of a row-vertex sum
    'rg_acc': 72,      # bgh_rg_acc: r . gamma.J accumulated
    'prop_h': 67,      # bgh_prop: i g and the top propagator (q, 1 / (q^2 - m^2) read)
    'amp_h': 64,       # Q . J(sigma) + i g W' v of one quark helicity pair
    'subset_h': 14,    # per gluon subset: q = p3 - P and 1 / (q^2 - m^2)
    'ginv_h': 8,       # per subset of >= 2 gluons: 1 / P^2
}


def bg_row(n):
    """FP64 flops of one (event, helicity) row of the Berends-Giele executor with n
    gluons (beams along +-z; the spinor branch for pz < 0 not included, as ROUTINE)."""
    import math
    cnt = [0] + [math.perm(n, L) for L in range(1, n + 1)]

    def current(L):
        return (L - 1) * BG['v3'] + math.comb(L - 1, 2) * BG['v4'] + BG['close']

    def row(i):
        return i * BG['row_term'] + BG['row_close']

    def qcurrent(L):
        return (L - 1) * BG['v3q'] + math.comb(L - 1, 2) * BG['v4q'] + BG['qclose']

    setup = 8 * n * 2 ** (n - 1) + 2 * ROUTINE['Gbeam'] + (n - 2) * ROUTINE['G'] + ROUTINE['U'] + ROUTINE['V'] \
        + BG['line']
    # stored currents with their Q.J, and Q.J of the external gluons
    currents = n * BG['q_dot'] + sum(cnt[L] * (current(L) + BG['q_dot']) for L in range(2, n))
    rows = sum(cnt[L] * row(L) for L in range(1, n - 1))
    amps = cnt[n] * (qcurrent(n) + (n - 2) * BG['amp_term'] + row(n - 1) + BG['amp_term'])
    return {'setup': setup, 'currents': currents, 'rows': rows, 'amplitudes': amps,
            'total': setup + currents + rows + amps}


def bgh_event(n):
    """FP64 flops of one event of the helicity-recycling Berends-Giele kernel with n
    gluons (n = 4, 5) and every helicity good: the set-up (momentum sums, propagator
    factors of every gluon subset, external states), currents of length L <= n-2 once
    per helicity variant of their gluons (2^L), row spinors of length L <= n-3 once per
    variant (2^(L+1)), and (n-1)! 2^n cycle items, each forming the n currents of
    length n-1 along its rotation cycle and, per ordering, the full current, the two
    row spinors and W of each top helicity, and four amplitudes (beams along +-z; the
    spinor branch for pz < 0 not included)."""
    import math
    cnt = [0] + [math.perm(n, L) for L in range(1, n + 1)]

    def current(L):
        return (L - 1) * BG['v3'] + math.comb(L - 1, 2) * BG['v4'] + BG['close_h']

    def row(L):
        return BG['rg'] + (L - 1) * BG['rg_acc'] + BG['prop_h']

    setup = 8 * n * 2 ** (n - 1) + BG['subset_h'] * 2 ** n + BG['ginv_h'] * (2 ** n - n - 1) \
        + 2 * (2 * ROUTINE['Gbeam'] + (n - 2) * ROUTINE['G']) + 6 * (ROUTINE['U'] + ROUTINE['V']) + 4 * BG['line']
    currents = sum(cnt[L] * 2 ** L * current(L) for L in range(2, n - 1))
    rows = sum(cnt[L] * 2 ** (L + 1) * row(L) for L in range(1, n - 2))
    # per top helicity: R(sigma[:n-2]), R(sigma[:n-1]) and W' (the n-2 further terms
    # of W after its first, from R(sigma[:n-2]))
    per_u = row(n - 2) + row(n - 1) + BG['rg'] + (n - 2) * BG['rg_acc']
    per_order = current(n) + 2 * per_u + 4 * BG['amp_h']
    items = cnt[n] // n * 2 ** n * (n * current(n - 1) + n * per_order)
    return {'setup': setup, 'currents': currents, 'rows': rows, 'items': items,
            'total': setup + currents + rows + items}


def diagram_kernel(name, executor, bg_variant=0):
    """FP64 flops per (event, helicity) of the kernel that evaluates the diagrams:
    everything for the one-lane and team executors (flows and colour form are fused
    into it; the team program runs the same routines), the group sums alone for the
    split executor (executor 2), whose flows and colour form run in kernels of their
    own, the recursion alone for the Berends-Giele executor (executor 3), whose
    colour form is a kernel of its own; with helicity recycling (launch variant 3)
    the kernel's flops per event divided by the 2^npar helicity rows (every helicity
    of these processes is good), and with the FP64 colour form fused into it
    (variants 4 and 5) the triangular colour form of each row on top (algorithmic
    count; the matrix cores execute the block-triangular product)."""
    if executor == 2:
        return group_sums_flops(name) + QUARK_BRANCH_MEAN
    if executor == 3:
        from .gen import codegen
        npar = codegen.PROCESS_NPAR[name]
        if bg_variant in (3, 4, 5):
            # per event over every helicity, shared out over the 2^npar rows
            f = (bgh_event(npar - 2)['total'] + 6 * QUARK_BRANCH_MEAN) / 2 ** npar
            if bg_variant in (4, 5):
                from .gen.colour import colour_matrix
                cf, _ = colour_matrix(npar - 2)
                f += colour_sum_flops(cf)
            return f
        return bg_row(npar - 2)['total'] + QUARK_BRANCH_MEAN
    return per_event_helicity(name) + QUARK_BRANCH_MEAN


def split_bytes(name):
    """Algorithmic HBM bytes per (event, helicity) row of the split executor's
    kernels: the sums kernel writes 2 NGROUP doubles; the flows kernel reads them
    and writes 2 NCOL doubles; the colour kernel reads the 2 NCOL doubles and writes
    one partial sum."""
    plan = _plan(name)
    ngroup, ncol = len(plan.colour_groups()), len(plan.basis)
    return {'sums': 8 * 2 * ngroup, 'flows': 8 * (2 * ngroup + 2 * ncol), 'colour': 8 * (2 * ncol + 1)}
