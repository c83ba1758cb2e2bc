"""Closed-form evolution of a single cavity mode under the REFLECT closure.

Under the image closure every operator of the scheme (the Pade derivative,
the compact operator M, the source conditioning G) acts diagonally on the
sine/cosine modes of the staggered grids, so a single sampled mode stays a
single mode and its amplitudes obey a small recurrence.  The symbols follow
from the stencils alone:
  second difference      : -sigma,            sigma = 4 sin^2(theta/2)
  Pade derivative (x h)  : 2 sin(theta/2) / a(theta),  a = (22 + 2 cos theta)/24
  M  (eq:ell scaled)     : alpha + beta (sum sigma - sum_{d<e} sigma_d sigma_e / 6)
  G  (P2 scaled)         : alpha - sum sigma / 12
with theta = pi k h.  This file is test code; it never calls the oracle.
"""
from __future__ import annotations

import numpy as np


def _symbols(k, n, r):
    h = 1.0 / n
    th = np.pi * np.asarray(k, dtype=np.float64) * h
    sig = 4.0 * np.sin(th / 2) ** 2
    dh = 2.0 * np.sin(th / 2) / ((22.0 + 2.0 * np.cos(th)) / 24.0)
    alpha = 1.0 + 2.0 / r ** 2
    beta = r ** 2 / 24.0
    mixed = sum(sig[a] * sig[b] for a in range(len(k)) for b in range(a + 1, len(k)))
    lam = alpha + beta * (sig.sum() - mixed / 6.0)
    g = alpha - sig.sum() / 12.0
    return dh, lam, g, alpha


def evolve_2d(k, n, r, z, amps, nsteps, tracked=True):
    """amps = (A, Bx, By, C): Ez = A s s, Hx = Bx s c, Hy = By c s, l = C s s."""
    (dx, dy), lam, g, alpha = _symbols(k, n, r)
    A, Bx, By, C = amps
    for _ in range(nsteps):
        craw = -dx * By + dy * Bx
        phi = z * g * craw / lam
        A_new = A + r * phi
        C = C + 24.0 / r ** 2 * (A_new - A) - 24.0 / r * z * craw
        A = A_new
        ge = alpha * A + C / 12.0 if tracked else g * A
        Bx = Bx + r * (-(1.0 / z) * dy * ge) / lam
        By = By + r * ((1.0 / z) * dx * ge) / lam
    return A, Bx, By, C


def evolve_3d(k, n, r, z, a, b, c, nsteps, tracked=True):
    """a, b, c: E, H and l amplitude 3-vectors of the cube mode
    E_s ~ cos along s, sin elsewhere;  H_s ~ sin along s, cos elsewhere.
    Pade curl in amplitude space: (curl H) = -(d x b), (curl E) = d x a."""
    d, lam, g, alpha = _symbols(k, n, r)
    a = np.array(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    c = np.array(c, dtype=np.float64)
    for _ in range(nsteps):
        craw = -np.cross(d, b)
        a_new = a + r * z * g * craw / lam
        c = c + 24.0 / r ** 2 * (a_new - a) - 24.0 / r * z * craw
        a = a_new
        ge = alpha * a + c / 12.0 if tracked else g * a
        b = b + r * (-(1.0 / z) * np.cross(d, ge)) / lam
    return a, b, c
