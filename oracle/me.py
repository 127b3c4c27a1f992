"""Leading-order |M|^2 for g g -> t tbar + k g from Feynman diagrams (oracle).

Steps, in the order of the paper's monolithic kernel (pseudo-code of the
"ihel0" engine and the colour-sum equation J^H C J = A^T C A + B^T C B):

  1. external states for helicity combination h (kinematics module);
  2. every diagram piece's Lorentz amplitude, by contracting its gluon trees
     into the top line  ubar(p3) [i g gamma.J1] S(q1) [i g gamma.J2] ... v(p4);
  3. dual amplitudes  J_sigma = sum_d c_{d,sigma} A_d;
  4. colour sum  ME_h = Re(J^H CF J)  (full double loop over colours);
  5. helicity sum and average  ME = sum_h ME_h / IDEN,  IDEN = 4*64*k!.

Feynman rules (Peskin & Schroeder ch. 16, all gluon momenta incoming):
  quark-gluon vertex       i g gamma^mu T^a
  ggg vertex               g f^{abc} [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
  gggg vertex              see the diagrams module
  top propagator           i (qslash + m) / (q^2 - m^2)   (zero width)
  gluon propagator         -i g_{mu nu} / P^2             (Feynman gauge)
The colour factors are carried by the piece coefficients, so everything here
is colour-stripped.  All arrays carry a leading event axis.
"""
from __future__ import annotations

import math

import numpy as np

from . import colour as _colour
from . import diagrams as _diagrams
from .kinematics import bar, cdtype, helicities, mdot, polarisation, slash, u_spinor, v_spinor

PROCESSES = {'gg_ttx': 4, 'gg_ttxg': 5, 'gg_ttxgg': 6, 'gg_ttxggg': 7, 'gg_ttxgggg': 8}


def slot_particle(slot):
    """Process-order index of gluon slot (slots 0,1 incoming; 2.. outgoing)."""
    return slot if slot < 2 else slot + 2


class Process:
    """Diagram pieces, colour coefficients and colour matrix for one process."""

    def __init__(self, npar, mt=173.0):
        if npar < 4:
            raise ValueError('npar >= 4')
        self.npar = npar
        self.ngluon = npar - 2
        self.mt = float(mt)
        self.basis = _colour.colour_basis(self.ngluon)
        index = {p: i for i, p in enumerate(self.basis)}
        self.pieces = _diagrams.diagram_pieces(self.ngluon)
        self.coefs = []
        for piece in self.pieces:
            c = _diagrams.piece_colour(piece)
            self.coefs.append([(index[w], complex(v)) for w, v in sorted(c.items())])
        self.ncolour = len(self.basis)
        self.nhel = 2 ** npar
        self.iden = _colour.iden(npar)
        self._cf = None

    @property
    def cf(self):
        if self._cf is None:
            self._cf = _colour.colour_matrix_float(self.ngluon)
        return self._cf

    @property
    def cf_ext(self):
        """The colour matrix in extended precision (exact rationals rounded once)."""
        exact = _colour.colour_matrix(self.ngluon)
        return np.array([[np.longdouble(x.numerator) / np.longdouble(x.denominator) for x in row]
                         for row in exact])


def gluon_states(mom, hel, ward_slot=None, override=None):
    """Per gluon slot: (external factor J^mu, momentum flowing into the diagram).

    The external factor is eps for an incoming and eps* for an outgoing gluon.
    ward_slot replaces that gluon's factor by k/E (gauge-invariance check);
    override = (slot, vector[nevt, 4]) replaces it by an arbitrary vector.
    """
    out = []
    n = mom.shape[1] - 2
    for slot in range(n):
        q = slot_particle(slot)
        p = mom[:, q]
        pin = p if slot < 2 else -p
        if override is not None and slot == override[0]:
            out.append((np.asarray(override[1], dtype=cdtype(p)), pin))
            continue
        if slot == ward_slot:
            out.append(((p / p[:, :1]).astype(cdtype(p)), pin))
            continue
        eps = polarisation(p, hel[q])
        out.append((eps if slot < 2 else np.conj(eps), pin))
    return out


def quark_states(mom, hel, mt):
    ubar3 = bar(u_spinor(mom[:, 2], hel[2], mt))
    v4 = v_spinor(mom[:, 3], hel[3], mt)
    return ubar3, v4


def vvv(ja, pa, jb, pb, g):
    """ggg vertex (colour-stripped) with the gluon propagator: current to the parent."""
    p = pa + pb
    k = -p
    v = (ja * mdot(k - pa, jb)[:, None] + mdot(ja, jb)[:, None] * (pa - pb)
         + jb * mdot(pb - k, ja)[:, None])
    return (-1j / mdot(p, p))[:, None] * g * v, p


def vvvv(s, ja, jb, jc, g):
    """gggg vertex structure s (colour-stripped) with the gluon propagator."""
    if s == 0:
        lor = jb * mdot(ja, jc)[:, None] - jc * mdot(ja, jb)[:, None]
    elif s == 1:
        lor = ja * mdot(jb, jc)[:, None] - jc * mdot(ja, jb)[:, None]
    else:
        lor = ja * mdot(jb, jc)[:, None] - jb * mdot(ja, jc)[:, None]
    return -1j * g * g * lor


def quark_propagator(q, m):
    den = mdot(q, q) - m * m
    s = slash(q)
    s = s + m * np.eye(4)
    return (1j / den)[:, None, None] * s


class _Evaluator:
    def __init__(self, proc, mom, hel, g, ward_slot=None, override=None):
        self.proc = proc
        self.g = g
        self.ext = gluon_states(mom, hel, ward_slot, override)
        self.ubar3, self.v4 = quark_states(mom, hel, proc.mt)
        self.p3 = mom[:, 2]
        self.trees = {}
        self.rows = {}

    def tree(self, t):
        """(current, momentum) of a gluon tree, memoised."""
        if isinstance(t, int):
            return self.ext[t]
        hit = self.trees.get(t)
        if hit is not None:
            return hit
        if t[0] == '3':
            ja, pa = self.tree(t[1])
            jb, pb = self.tree(t[2])
            res = vvv(ja, pa, jb, pb, self.g)
        else:
            ja, pa = self.tree(t[2])
            jb, pb = self.tree(t[3])
            jc, pc = self.tree(t[4])
            p = pa + pb + pc
            lor = vvvv(t[1], ja, jb, jc, self.g)
            res = ((-1j / mdot(p, p))[:, None] * lor, p)
        self.trees[t] = res
        return res

    def row(self, prefix):
        """ubar(p3) [i g J1-slash] S(q1) ... [i g Jj-slash] S(qj) for a prefix of trees."""
        if not prefix:
            return self.ubar3, self.p3
        hit = self.rows.get(prefix)
        if hit is not None:
            return hit
        prev, q = self.row(prefix[:-1])
        j, p = self.tree(prefix[-1])
        r = np.einsum('ea,eab->eb', prev, 1j * self.g * slash(j))
        q = q - p
        r = np.einsum('ea,eab->eb', r, quark_propagator(q, self.proc.mt))
        self.rows[prefix] = (r, q)
        return r, q

    def amplitude(self, piece):
        prev, _ = self.row(piece[:-1])
        j, _ = self.tree(piece[-1])
        r = np.einsum('ea,eab->eb', prev, 1j * self.g * slash(j))
        return np.einsum('ea,ea->e', r, self.v4)


def coupling(alpha_s, dtype=np.float64):
    """g = sqrt(4 pi alpha_s) in the working precision."""
    pi = np.arccos(np.asarray(-1.0, dtype=dtype))
    return np.sqrt(4 * pi * np.asarray(alpha_s, dtype=dtype))


def _momenta(mom):
    mom = np.asarray(mom)
    return mom if mom.dtype == np.longdouble else mom.astype(np.float64)


def jamps(proc, mom, h, alpha_s, ward_slot=None, override=None):
    """Dual amplitudes J[nevt, ncolour] for helicity combination h."""
    mom = _momenta(mom)
    hel = helicities(proc.npar, h)
    ev = _Evaluator(proc, mom, hel, coupling(alpha_s, mom.dtype), ward_slot, override)
    out = np.zeros((mom.shape[0], proc.ncolour), dtype=cdtype(mom))
    for piece, coefs in zip(proc.pieces, proc.coefs):
        a = ev.amplitude(piece)
        for s, c in coefs:
            out[:, s] += c * a
    return out


def piece_amplitudes(proc, mom, h, alpha_s):
    """Colour-stripped Lorentz amplitude of every diagram piece, [npiece, nevt]."""
    mom = _momenta(mom)
    ev = _Evaluator(proc, mom, helicities(proc.npar, h), coupling(alpha_s, mom.dtype))
    return np.stack([ev.amplitude(piece) for piece in proc.pieces])


def colour_sum(proc, jamp):
    """ME_h = sum_{s,t} conj(J_s) CF_st J_t, real part (full double loop)."""
    cf = proc.cf if jamp.dtype == np.complex128 else proc.cf_ext
    return np.einsum('es,st,et->e', np.conj(jamp), cf, jamp).real


def me_helicities(proc, mom, alpha_s, hels=None):
    """Per-helicity colour sums ME_h, shape [nhel, nevt] (not divided by IDEN)."""
    hels = range(proc.nhel) if hels is None else hels
    return np.stack([colour_sum(proc, jamps(proc, mom, h, alpha_s)) for h in hels])


def matrix_element(proc, mom, alpha_s):
    """Helicity- and colour-summed, initial-state averaged |M|^2 per event."""
    return me_helicities(proc, mom, alpha_s).sum(axis=0) / proc.iden


_CACHE = {}


def process(name_or_npar, mt=173.0):
    npar = PROCESSES[name_or_npar] if isinstance(name_or_npar, str) else int(name_or_npar)
    key = (npar, float(mt))
    if key not in _CACHE:
        _CACHE[key] = Process(npar, mt)
    return _CACHE[key]
