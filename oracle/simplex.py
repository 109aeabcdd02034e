"""Simplex projection, pruning map and coefficient step (FP64 oracle).

* Euclidean projection onto ``Delta_q`` (used by eq. coefficient-update and by
  the spectral candidates of eq. spectral-candidates).  The paper does not say
  how it is computed; the projection is unique, so any exact method gives the
  same point.  Here: the sort-based method -- sort descending, find the
  largest ``k`` with ``v_(k) - (sum_{i<=k} v_(i) - 1)/k > 0``, shift by that
  threshold and clip at zero.
* Pruning ``I_tau(beta) = {r : beta_r > tau}`` with renormalisation
  ``beta_check = beta_I / sum(beta_I)`` and the tuple ``P_tau`` (eq. truncation-map).
  Reading for the case the paper does not discuss: if no entry exceeds
  ``tau`` the largest entry is kept alone.
"""
from __future__ import annotations

import numpy as np


def project_simplex(v) -> np.ndarray:
    """Euclidean projection of ``v`` onto the probability simplex."""
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    u = np.sort(v)[::-1]
    css = np.cumsum(u)
    k = np.arange(1, v.size + 1)
    cond = u - (css - 1.0) / k > 0
    rho = int(np.nonzero(cond)[0][-1])
    theta = (css[rho] - 1.0) / (rho + 1)
    return np.maximum(v - theta, 0.0)


def prune(beta, tau: float):
    """``(keep_idx, beta_check)`` of the pruning map: strict ``beta_r > tau``, renormalised."""
    beta = np.asarray(beta, dtype=np.float64)
    keep = np.nonzero(beta > tau)[0]
    if keep.size == 0:
        keep = np.array([int(np.argmax(beta))])
    b = beta[keep]
    return keep, b / b.sum()


def truncation_map(beta, atoms, tau: float):
    """``P_tau(beta, Psi) = (|I|, beta_check, Psi_I)`` (eq. truncation-map); ``atoms`` is ``[q][D]``."""
    keep, bc = prune(beta, tau)
    return keep.size, bc, np.asarray(atoms)[keep]


def coefficient_step(alpha, h, eta: float):
    """``beta = proj_Delta(alpha + eta h)`` with ``h = A^T c`` (eq. coefficient-update)."""
    return project_simplex(np.asarray(alpha, dtype=np.float64) + eta * np.asarray(h, dtype=np.float64))


def reweight(alpha, h, eta: float, tau: float):
    """Coefficient step followed by pruning: returns ``(alpha_out padded to R, keep_idx, R_out)``."""
    beta = coefficient_step(alpha, h, eta)
    keep, bc = prune(beta, tau)
    out = np.zeros(np.asarray(alpha).size)
    out[: keep.size] = bc
    return out, keep.astype(np.int32), int(keep.size)
