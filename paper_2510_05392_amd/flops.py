"""Algorithmic FP64 work of one (event, helicity) of the generated path.

Counting rules: every real add, subtract, multiply, divide and square root is
one flop (a fused multiply-add is two); complex add = 2, complex multiply = 6,
complex a + b*c = 8, real x complex = 2, multiplication by +-i and negation
are free.  The per-routine figures below are read off the device routines
(csrc/me_device.h) at those rules, counting each distinct intermediate once;
a process's figure is the sum over its evaluation plan (currents, amplitude
contractions, colour-flow accumulation) plus the triangular colour quadratic
form.  This is the number the benchmark's roofline fraction divides by the
measured kernel time.
"""
from __future__ import annotations

ROUTINE = {
    'G': 24,          # ext_gluon: polar angles (10), components (14)
    'U': 35,          # ext_ubar: helicity spinor (16), omegas (11), scaling (8)
    'V': 37,          # ext_v: as ext_ubar plus two sign products
    'v3': 162,        # v3_current: momenta (16), three dots (58), 1/P^2 (8), combine (80)
    'v4': 133,        # v4_current: 1/P^2 (9), two complex dots (60), combine (64)
    'KD3': 162,       # v3_open on a top-line current: as v3_current
    'KD4': 133,       # v4_open on a top-line current: as v4_current
    'Lh': 72,         # row_vertex: slash blocks (8), 2x2 blocks (56), coupling (8)
    'Rh': 72,         # vertex_col
    'L': 79,          # row_prop: q (4), propagator blocks + 1/(q^2-m^2) (11), product (56), scale (8)
    'R': 79,          # prop_col
    'K': 80,          # line_current: 8 complex products (48), combinations (24), coupling (8)
    'dot': 30,        # sdot / vdot: 4 complex products, 3 complex adds
    'ffv': 102,       # row_vertex + sdot
    'jamp': 2,        # one complex accumulation (group sum or colour flow)
}


def plan_flops(plan):
    """FP64 flops per (event, helicity) for the diagram part of an evaluation plan."""
    total = 0
    masks = set()
    for key in plan.order:
        r = plan.routine(key)
        total += ROUTINE[r]
        if key[0] == 'J':
            node = plan.trees.nodes[key[1]]
            kids = node[1:] if node[0] == 'v3' else node[2:]
            masks.add(plan.trees.mask[key[1]])
            masks.update(plan.trees.mask[c] for c in kids)
        elif key[0] in ('L', 'R'):
            m = 0
            for t in key[1]:
                m |= plan.trees.mask[t]
            masks.add(m)
        elif key[0] == 'KD':
            masks.add(plan.hole_mask(key))
            masks.update(plan.trees.mask[t] for t in key[3][-1][3])
    # momentum sums P(mask) = sum of |mask| external momenta, once per mask
    total += sum(4 * (bin(m).count('1') - 1) for m in masks)
    for amp in plan.amps:
        total += ROUTINE['ffv'] if len(amp) == 4 else ROUTINE['dot']
    # pieces with the same colour vector are summed, then added to each of its flows
    for key, members in plan.colour_groups():
        total += ROUTINE['jamp'] * (len(members) - 1 + len(key))
    return total


def colour_sum_flops(ncol):
    """Triangular quadratic form sum_ij CF_ij Re(J_i^* J_j) with integer CF."""
    return 2 * ncol * ncol + 4 * ncol


def _plan(name):
    from .gen import codegen
    from .gen.topology import Plan
    return Plan(codegen.PROCESS_NPAR[name] - 2)


def per_event_helicity(name):
    plan = _plan(name)
    return plan_flops(plan) + colour_sum_flops(len(plan.basis))


def flow_updates(plan):
    """Colour-flow accumulations (one per (group, flow) pair) of a plan."""
    return sum(len(key) for key, _ in plan.colour_groups())


def diagram_kernel(name, executor):
    """FP64 flops per (event, helicity) of the kernel that evaluates the diagrams:
    everything for the one-lane and team executors (flows and colour form are fused
    into it), the group sums alone for the split executor (executor 2), whose flows
    and colour form run in kernels of their own."""
    plan = _plan(name)
    if executor == 2:
        return plan_flops(plan) - ROUTINE['jamp'] * flow_updates(plan)
    return plan_flops(plan) + colour_sum_flops(len(plan.basis))


def split_bytes(name):
    """Algorithmic HBM bytes per (event, helicity) row of the split executor's
    kernels: the sums kernel writes 2 NGROUP doubles; the flows kernel reads them
    and writes 2 NCOL doubles; the colour kernel reads the 2 NCOL doubles and writes
    one partial sum."""
    plan = _plan(name)
    ngroup, ncol = len(plan.colour_groups()), len(plan.basis)
    return {'sums': 8 * 2 * ngroup, 'flows': 8 * (2 * ngroup + 2 * ncol), 'colour': 8 * (2 * ncol + 1)}
