"""Minkowski algebra, Dirac matrices and helicity external states (oracle).

Conventions (textbook, Peskin & Schroeder ch. 3 and 16):
  metric diag(+1,-1,-1,-1); four-vectors stored with upper indices (x^0..x^3);
  chiral (Weyl) representation  gamma^0 = [[0,1],[1,0]],
  gamma^i = [[0, sigma^i], [-sigma^i, 0]].
External states are helicity eigenstates:
  u(p,l)  = ( sqrt(E - l|p|) chi_l , sqrt(E + l|p|) chi_l )
  v(p,l)  = ( sqrt(E + l|p|) chi_-l , -sqrt(E - l|p|) chi_-l )
  eps(k,l) = (-l e1 - i e2)/sqrt(2),  e1 = (0, cos t cos f, cos t sin f, -sin t),
                                       e2 = (0, -sin f, cos f, 0).
The paper's external-wavefunction routines compute the same objects for the
outgoing top (u-bar), the outgoing antitop (v) and the gluons (section "a
closer look at the internals of the ME engine"); it leaves their formulas to
HELAS.  Particles moving exactly along -z take the theta = pi limit with
phi = 0.

All functions are vectorised over a leading event axis and keep the precision
of their inputs: float64 momenta give complex128 results, np.longdouble momenta
give np.clongdouble results (used to adjudicate ill-conditioned events).
"""
from __future__ import annotations

import numpy as np

METRIC = np.array([1.0, -1.0, -1.0, -1.0])

_S0 = np.eye(2, dtype=complex)
_S1 = np.array([[0, 1], [1, 0]], dtype=complex)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
_S3 = np.array([[1, 0], [0, -1]], dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)

GAMMA = np.array([
    np.block([[_Z2, _S0], [_S0, _Z2]]),
    np.block([[_Z2, _S1], [-_S1, _Z2]]),
    np.block([[_Z2, _S2], [-_S2, _Z2]]),
    np.block([[_Z2, _S3], [-_S3, _Z2]]),
])  # GAMMA[mu] = gamma^mu (upper index)


def mdot(a, b):
    """Minkowski product a.b = a^0 b^0 - a.b (no complex conjugation)."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def cdtype(x):
    """Complex dtype matching the precision of array x."""
    return np.clongdouble if np.asarray(x).dtype in (np.longdouble, np.clongdouble) else np.complex128


def slash(a):
    """gamma^mu a_mu as a [..., 4, 4] matrix."""
    a = np.asarray(a)
    return np.einsum('...m,mab->...ab', a * METRIC, GAMMA.astype(cdtype(a)))


def _chi(p3, lam):
    """Two-component helicity eigenstate: (sigma . phat) chi = lam chi."""
    px, py, pz = p3[..., 0], p3[..., 1], p3[..., 2]
    pt2 = px * px + py * py
    pabs = np.sqrt(pt2 + pz * pz)
    # |p| + pz, written as pt^2 / (|p| - pz) when pz < 0 (same number, no cancellation)
    with np.errstate(divide='ignore', invalid='ignore'):
        ppz = np.where(pz >= 0, pabs + pz, pt2 / (pabs - pz))
    out = np.zeros(p3.shape[:-1] + (2,), dtype=cdtype(p3))
    reg = ppz > 0.0
    # generic direction: cos(t/2) = sqrt((|p|+pz)/2|p|), e^{if} sin(t/2) = (px+i py)/sqrt(2|p|(|p|+pz))
    with np.errstate(divide='ignore', invalid='ignore'):
        c = np.sqrt(ppz / (2.0 * pabs))
        sp = (px + 1j * py) / np.sqrt(2.0 * pabs * ppz)
    if lam > 0:
        out[..., 0] = np.where(reg, c, 0.0)
        out[..., 1] = np.where(reg, sp, 1.0)
    else:
        out[..., 0] = np.where(reg, -np.conj(sp), -1.0)
        out[..., 1] = np.where(reg, c, 0.0)
    return out


def _e_minus_p(e, pabs, m):
    """E - |p| evaluated as m^2 / (E + |p|): the same number without cancellation."""
    return m * m / (e + pabs)


def _omegas(p, lam, m):
    """(sqrt(E - lam|p|), sqrt(E + lam|p|))."""
    e = p[..., 0]
    pabs = np.sqrt((p[..., 1:] ** 2).sum(axis=-1))
    small = np.sqrt(_e_minus_p(e, pabs, m))
    big = np.sqrt(e + pabs)
    return (small, big) if lam > 0 else (big, small)


def u_spinor(p, lam, m):
    chi = _chi(p[..., 1:], lam)
    a, b = _omegas(p, lam, m)
    return np.concatenate([a[..., None] * chi, b[..., None] * chi], axis=-1)


def v_spinor(p, lam, m):
    eta = _chi(p[..., 1:], -lam)
    b, a = _omegas(p, lam, m)          # a = sqrt(E + lam|p|), b = sqrt(E - lam|p|)
    return np.concatenate([a[..., None] * eta, -b[..., None] * eta], axis=-1)


def bar(spinor):
    """Dirac adjoint psi^dagger gamma^0 as a row spinor."""
    return np.einsum('...a,ab->...b', np.conj(spinor), GAMMA[0].astype(cdtype(spinor)))


def polarisation(k, lam):
    """Massless vector polarisation eps^mu(k, lam) (helicity lam = +-1)."""
    kx, ky, kz = k[..., 1], k[..., 2], k[..., 3]
    kt = np.sqrt(kx * kx + ky * ky)
    kabs = np.sqrt(kt * kt + kz * kz)
    ct = kz / kabs
    st = kt / kabs
    with np.errstate(divide='ignore', invalid='ignore'):
        cf = np.where(kt > 0, kx / kt, 1.0)
        sf = np.where(kt > 0, ky / kt, 0.0)
    zero = np.zeros_like(kx)
    e1 = np.stack([zero, ct * cf, ct * sf, -st], axis=-1)
    e2 = np.stack([zero, -sf, cf, zero], axis=-1)
    return (-lam * e1 - 1j * e2) / np.sqrt(np.asarray(2.0, dtype=kx.dtype))


def helicities(npar, h):
    """Helicity of each particle for combination index h in [0, 2^npar).

    Particle q (0-based, process order) has helicity +1 when bit (npar-1-q)
    of h is set, else -1: the last particle varies fastest.
    """
    return [1 if (h >> (npar - 1 - q)) & 1 else -1 for q in range(npar)]
