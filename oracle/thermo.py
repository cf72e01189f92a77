"""Plain reference for the thermodynamics built on converged solutions (TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

Entropy (the paragraph on entropy after the magnetization results): importance
sampling gives no entropy directly, so it follows from the Maxwell relation
dS/dmu = dN/dT, integrated over mu from the empty system (mu -> -inf, S = 0).
Per site, s_i(mu) = int_{mu_0}^{mu} dn_i/dT dmu' with the lowest grid point
mu_0 taken as empty.  Readings: dn/dT as the central difference of densities
at T_lo and T_hi (the estimate belongs to T = (T_lo + T_hi) / 2), the mu
integral by the trapezoid rule on the given grid.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import cumulative_trapezoid


def entropy_from_densities(mu, n_lo, n_hi, T_lo, T_hi):
    """mu (K,) ascending; n_lo, n_hi (K, S) densities at T_lo < T_hi.
    Returns s (K, S): the entropy of each site at every grid point."""
    dndT = (np.asarray(n_hi, dtype=np.float64) - np.asarray(n_lo, dtype=np.float64)) / (T_hi - T_lo)
    return cumulative_trapezoid(dndT, np.asarray(mu, dtype=np.float64), axis=0, initial=0.0)


def staggered(values, coords):
    """(-1)^(x + y) values_i: the staggered pattern of a square lattice (for
    m_i = n_up,i - n_dn,i this is the staggered magnetization)."""
    c = np.asarray(coords)
    return np.where(c.sum(axis=1) % 2 == 0, 1.0, -1.0) * np.asarray(values)
