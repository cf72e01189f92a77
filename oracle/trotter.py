"""Plain reference for the removal of the Trotter error (TEST INFRASTRUCTURE
ONLY, like the rest of ``oracle/``).

The paper removes the systematic error of the time discretisation by
extrapolating dtau -> 0 (the sentence on the discretisation error after
Eq. (2), citing the extrapolation literature).  Reading: observables of the
discretised problem are even in dtau, O(dtau) = c0 + c1 dtau^2 (+ c2 dtau^4),
fitted by weighted least squares over runs at several L with weights
1 / err^2; c0 is the dtau -> 0 estimate, its error the square root of the
corresponding diagonal element of the fit's covariance (A^T W A)^-1.
"""
from __future__ import annotations

import numpy as np


def fit(dtau, value, err=None, order: int = 1):
    """Coefficients c_0 .. c_order of sum_k c_k dtau^(2k) and their errors
    (None without input errors)."""
    x = np.asarray(dtau, dtype=np.float64) ** 2
    y = np.asarray(value, dtype=np.float64)
    A = np.stack([x ** k for k in range(order + 1)], axis=1)
    if err is None:
        c = np.linalg.lstsq(A, y, rcond=None)[0]
        return c, None
    w = 1.0 / np.asarray(err, dtype=np.float64)
    c = np.linalg.lstsq(A * w[:, None], y * w, rcond=None)[0]
    cov = np.linalg.inv((A * (w ** 2)[:, None]).T @ A)
    return c, np.sqrt(np.diag(cov))
