"""A small acceptance-safeguarded iteration in the order of the paper's
master-worker algorithm, used by the exact-recovery pin.

Slots: atom steps (eqs. atom-direction, atom-trial), coefficient steps
(eq. coefficient-update with the pruning map) and spectral steps
(eqs. density-proposal ... spectral-selection), each followed by the acceptance
rule (eq. state-acceptance-rule).  Step sizes are searched on the grid
``{2^-j}, j = 0..10``, largest first, keeping the first accepted one.

Readings: the atom to move is chosen cyclically (``r_t = t mod R_t``); slot
``t`` is a spectral step when ``t % t_ref == 0``, a coefficient step when
``t % t_alpha == 0``, otherwise an atom step.
"""
from __future__ import annotations

import numpy as np

from . import born, refactor, simplex

GRID = [2.0 ** (-j) for j in range(11)]


def objective(atoms, weights, settings, f, kind, eps, mu):
    """``J = L(A alpha) + mu R`` (eq. fixed-rank-objective)."""
    p = born.probs_axis(atoms, weights, settings)
    L, g = born.loss_and_sensitivity(p, f, np.asarray(settings).shape[0], kind, eps)
    return L + mu * len(weights), g


def run(atoms, weights, settings, f, kind=born.LOSS_CE, eps=0.0, mu=1e-3, tau=1e-3, tau_acc=1e-10,
        iters=200, t_alpha=5, t_ref=10, L_max=None, n_lanczos=30, rng=None, history=None):
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128).copy()
    w = np.asarray(weights, dtype=np.float64).copy()
    D = atoms.shape[1]
    L_max = L_max or atoms.shape[0]
    rng = rng or np.random.default_rng(0)
    J, g = objective(atoms, w, settings, f, kind, eps, mu)
    for t in range(iters):
        R = w.size
        accepted = None
        if t % t_ref == 0:
            v0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
            for eta in GRID:
                res = refactor.lanczos_refactor(atoms, w, settings, f, kind, eps, eta, mu, tau,
                                                L_max, n_lanczos, v0)
                Jn, gn = objective(res["atoms"], res["weights"], settings, f, kind, eps, mu)
                if Jn <= J - tau_acc:
                    accepted = (res["atoms"], res["weights"], Jn, gn)
                    break
        elif t % t_alpha == 0:
            _, gw = born.gradients_axis(atoms, w, settings, g)
            h = -gw
            for eta in GRID:
                beta = simplex.coefficient_step(w, h, eta)
                keep, bc = simplex.prune(beta, tau)
                Jn, gn = objective(atoms[keep], bc, settings, f, kind, eps, mu)
                if Jn <= J - tau_acc:
                    accepted = (atoms[keep], bc, Jn, gn)
                    break
        else:
            r = t % R
            ga, _ = born.gradients_axis(atoms, w, settings, g)
            d = -born.tangent_project(atoms, ga)[r]
            for eta in GRID:
                trial = atoms[r] + eta * d
                trial = trial / np.linalg.norm(trial)
                new_atoms = atoms.copy()
                new_atoms[r] = trial
                Jn, gn = objective(new_atoms, w, settings, f, kind, eps, mu)
                if Jn <= J - tau_acc:
                    accepted = (new_atoms, w, Jn, gn)
                    break
        if accepted is not None:
            atoms, w, J, g = accepted
            atoms = np.asarray(atoms).copy()
            w = np.asarray(w).copy()
        if history is not None:
            history.append((t, J, w.size, accepted is not None))
    return atoms, w, J
