"""Seeded flat phase-space points (RAMBO) for g g -> t tbar + k g.

This module only produces inputs.  It holds none of the matrix-element
arithmetic; the oracle tests, the GPU tests and the benchmark all draw their
momenta from it, so both sides of every parity check see identical events.

The paper generates its events inside its standalone application from random
numbers (software architecture review, "three software areas"); it does not
name the generator.  Here we use the RAMBO algorithm of Kleiss, Stirling and
Ellis, Comput. Phys. Commun. 40 (1986) 359: isotropic massless momenta with
energy density q0*exp(-q0), a conformal boost/scale onto the centre-of-mass
frame, then a Newton solve for the common rescaling xi that puts the final
state on its mass shells.

Layout: ``momenta[nevt][npar][4]`` with (E, px, py, pz) in GeV, float64,
particle order g(1) g(2) t(3) tbar(4) g(5) ... g(npar).  Beams run along +-z.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_SQRTS = 1500.0
DEFAULT_MT = 173.0


def _massless(r: np.ndarray, sqrts: float) -> np.ndarray:
    """Massless RAMBO step; r has shape [nevt, n, 4] of uniforms in [0,1)."""
    c = 2.0 * r[..., 0] - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    f = 2.0 * math.pi * r[..., 1]
    # -log of a product of two uniforms: energy density q0*exp(-q0).
    # 1 - r keeps the argument in (0, 1].
    q0 = -np.log((1.0 - r[..., 2]) * (1.0 - r[..., 3]))
    q = np.stack([q0, q0 * s * np.cos(f), q0 * s * np.sin(f), q0 * c], axis=-1)
    Q = q.sum(axis=1)                                      # [nevt, 4]
    M = np.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(axis=1))
    b = -Q[:, 1:] / M[:, None]
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    x = sqrts / M
    bq = (b[:, None, :] * q[..., 1:]).sum(axis=-1)         # [nevt, n]
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gam[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:] + b[:, None, :] * q[..., :1] + a[:, None, None] * bq[..., None] * b[:, None, :])
    return p


def _massive(p: np.ndarray, masses: np.ndarray, sqrts: float):
    """Rescale massless momenta p onto mass shells; returns (k, xi).

    Before the rescaling, the rounding residue of the massless boost (it grows
    with the boost factor, up to ~1e-11 relative) is removed from the three-
    momenta and the massless energies are reset to |p|, so that the final
    points conserve momentum and sit on their mass shells to a few ulps; the
    Newton solve for xi then restores the energy sum exactly.
    """
    m2 = masses ** 2
    p3 = p[..., 1:] - p[..., 1:].sum(axis=1, keepdims=True) / p.shape[1]
    p0 = np.sqrt((p3 ** 2).sum(axis=-1))
    xi = np.full(p.shape[0], math.sqrt(max(0.0, 1.0 - (masses.sum() / sqrts) ** 2)))
    for _ in range(60):
        e = np.sqrt(m2[None, :] + (xi[:, None] * p0) ** 2)
        f = e.sum(axis=1) - sqrts
        df = (xi[:, None] * p0 ** 2 / e).sum(axis=1)
        step = f / df
        xi = xi - step
        if np.all(np.abs(step) <= 1e-16 * np.abs(xi)):
            break
    k = np.empty_like(p)
    k[..., 1:] = xi[:, None, None] * p3
    k[..., 0] = np.sqrt(m2[None, :] + (xi[:, None] * p0) ** 2)
    return k, xi


def rambo_weight(k: np.ndarray, masses: np.ndarray, sqrts: float) -> np.ndarray:
    """Phase-space weight of massive RAMBO points (KSE 1986, massive correction)."""
    n = k.shape[1]
    s = sqrts * sqrts
    w0 = ((2.0 * math.pi) ** (4 - 3 * n) * (math.pi / 2.0) ** (n - 1) * s ** (n - 2)
          / (math.factorial(n - 1) * math.factorial(n - 2)))
    if not np.any(masses > 0):
        return np.full(k.shape[0], w0)
    kabs = np.sqrt((k[..., 1:] ** 2).sum(axis=-1))
    e = k[..., 0]
    t1 = (kabs.sum(axis=1) / sqrts) ** (2 * n - 3)
    t2 = np.prod(kabs / e, axis=1)
    t3 = sqrts / (kabs ** 2 / e).sum(axis=1)
    return w0 * t1 * t2 * t3


def generate(npar: int, nevt: int, seed: int, sqrts: float = DEFAULT_SQRTS,
             mt: float = DEFAULT_MT, return_weights: bool = False):
    """Return momenta[nevt][npar][4] (float64) for g g -> t tbar + (npar-4) g."""
    if npar < 4:
        raise ValueError("npar must be >= 4")
    nf = npar - 2
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.random((nevt, nf, 4))
    masses = np.zeros(nf)
    masses[0] = mt
    masses[1] = mt
    pl = _massless(r, sqrts)
    k, _ = _massive(pl, masses, sqrts)
    mom = np.empty((nevt, npar, 4))
    e = 0.5 * sqrts
    mom[:, 0] = (e, 0.0, 0.0, e)
    mom[:, 1] = (e, 0.0, 0.0, -e)
    mom[:, 2:] = k
    if return_weights:
        return mom, rambo_weight(k, masses, sqrts)
    return mom
