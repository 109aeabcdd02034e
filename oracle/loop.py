"""An acceptance-safeguarded iteration in the order of the paper's master-worker
algorithm (Algorithm 1), used by the exact-recovery pin and as the reference of the
device-driven iteration.

Slots: atom steps (eqs. atom-direction, atom-trial), coefficient steps
(eq. coefficient-update with the pruning map) and spectral steps
(eqs. density-proposal ... spectral-selection), each followed by the acceptance
rule (eq. state-acceptance-rule) on the objective ``J = L + mu R`` (eq.
fixed-rank-objective).  Step sizes are searched on the grid ``{2^-j}``,
``j = 0..n_grid-1`` (Table sim-parameters), largest first, keeping the first
accepted one.

Readings: the atom to move is chosen cyclically (``r_t = t mod R_t``); slot
``t`` is a spectral step when ``t % t_ref == 0``, a coefficient step when
``t % t_alpha == 0``, otherwise an atom step.  Spectral slot ``k`` (counting
from 0) starts Lanczos from ``v0s[k % len(v0s)]`` when start vectors are given,
else from a fresh complex normal draw of ``rng``.  Stopping (Table
sim-parameters): ``delta`` is the relative objective decrease over the last
``stop_window`` accepted updates (the initial state counts as the first), and
the oracle-call count adds, per slot, one for the gradient product (``G psi``
or ``A^T c``), one per trial for its response and loss, and, per spectral
trial, ``min(n_lanczos, D)`` Lanczos products ``G v`` plus one for the loss.
"""
from __future__ import annotations

import numpy as np

from . import born, refactor, simplex

GRID = [2.0 ** (-j) for j in range(11)]
KIND_RHO, KIND_ALPHA, KIND_PSI = 0, 1, 2


def objective(atoms, weights, settings, f, kind, eps, mu):
    """``J = L(A alpha) + mu R`` (eq. fixed-rank-objective)."""
    p = born.probs_axis(atoms, weights, settings)
    L, g = born.loss_and_sensitivity(p, f, np.asarray(settings).shape[0], kind, eps)
    return L + mu * len(weights), g


def slot_kind(t: int, t_alpha: int, t_ref: int) -> int:
    """Which set of the partition (eq. iteration-partition) slot ``t`` belongs to: the
    spectral set when ``t % t_ref == 0`` (tested first), else the coefficient set when
    ``t % t_alpha == 0``, else the atom set; a period of 0 leaves its set empty."""
    if t_ref > 0 and t % t_ref == 0:
        return KIND_RHO
    if t_alpha > 0 and t % t_alpha == 0:
        return KIND_ALPHA
    return KIND_PSI


def atom_direction(atoms, weights, settings, g, r: int) -> np.ndarray:
    """Atom direction of eq. atom-direction, ``alpha_r (I - psi_r psi_r^*) G psi_r``.

    With ``dL/dpsi_r^* = -alpha_r G psi_r`` (eq. atom-wirtinger-gradient; ``g`` the
    sensitivities ``dL/dp`` of the current state) it is minus the tangent projection
    of the atom gradient (eq. atom-projected-descent-direction)."""
    ga, _ = born.gradients_axis(atoms, weights, settings, g)
    return -born.tangent_project(atoms, ga)[r]


def atom_trial(psi, d, eta: float) -> np.ndarray:
    """Normalised proposed atom ``(psi + eta d) / ||psi + eta d||`` (eq. atom-trial)."""
    trial = np.asarray(psi, dtype=np.complex128) + eta * np.asarray(d, dtype=np.complex128)
    return trial / np.linalg.norm(trial)


def coefficient_direction(atoms, weights, settings, g) -> np.ndarray:
    """``h = A^T c = -dL/dalpha`` (eqs. h_t, weight-gradient)."""
    _, gw = born.gradients_axis(atoms, weights, settings, g)
    return -gw


def coefficient_trial(weights, h, eta: float, tau: float):
    """``P_tau(proj_Delta(alpha + eta h))`` as ``(keep, beta_check)`` (eqs.
    coefficient-update, truncation-map)."""
    beta = simplex.coefficient_step(weights, h, eta)
    return simplex.prune(beta, tau)


def run(atoms, weights, settings, f, kind=born.LOSS_CE, eps=0.0, mu=1e-3, tau=1e-3, tau_acc=1e-10,
        iters=200, t_alpha=5, t_ref=10, L_max=None, n_lanczos=30, rng=None, history=None, v0s=None,
        n_grid=11, stop_window=0, stop_delta=0.0, oracle_budget=0, info=None):
    """Runs up to ``iters`` slots.  ``history`` (a list) receives one tuple per slot:
    ``(t, kind, J_after, R_after, accepted, j_eta or -1)``; ``info`` (a dict) receives
    ``slots``, ``oracle_calls`` and ``stopped`` ('T', 'delta' or 'budget')."""
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128).copy()
    w = np.asarray(weights, dtype=np.float64).copy()
    D = atoms.shape[1]
    L_max = L_max or atoms.shape[0]
    rng = rng or np.random.default_rng(0)
    grid = [2.0 ** (-j) for j in range(n_grid)]
    J, g = objective(atoms, w, settings, f, kind, eps, mu)
    accepted_J = [J]
    n_oracle = 1
    n_spectral = 0
    stopped = "T"
    slots = 0
    for t in range(iters):
        R = w.size
        accepted = None
        j_acc = -1
        sk = slot_kind(t, t_alpha, t_ref)
        if sk == KIND_RHO:
            if v0s is not None:
                v0 = np.asarray(v0s[n_spectral % len(v0s)], dtype=np.complex128)
            else:
                v0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
            n_spectral += 1
            for j, eta in enumerate(grid):
                res = refactor.lanczos_refactor(atoms, w, settings, f, kind, eps, eta, mu, tau,
                                                L_max, n_lanczos, v0)
                Jn, gn = objective(res["atoms"], res["weights"], settings, f, kind, eps, mu)
                n_oracle += min(n_lanczos, D) + 1
                if Jn <= J - tau_acc:
                    accepted = (res["atoms"], res["weights"], Jn, gn)
                    j_acc = j
                    break
        elif sk == KIND_ALPHA:
            h = coefficient_direction(atoms, w, settings, g)
            n_oracle += 1
            for j, eta in enumerate(grid):
                keep, bc = coefficient_trial(w, h, eta, tau)
                Jn, gn = objective(atoms[keep], bc, settings, f, kind, eps, mu)
                n_oracle += 1
                if Jn <= J - tau_acc:
                    accepted = (atoms[keep], bc, Jn, gn)
                    j_acc = j
                    break
        else:
            r = t % R
            d = atom_direction(atoms, w, settings, g, r)
            n_oracle += 1
            for j, eta in enumerate(grid):
                new_atoms = atoms.copy()
                new_atoms[r] = atom_trial(atoms[r], d, eta)
                Jn, gn = objective(new_atoms, w, settings, f, kind, eps, mu)
                n_oracle += 1
                if Jn <= J - tau_acc:
                    accepted = (new_atoms, w, Jn, gn)
                    j_acc = j
                    break
        slots = t + 1
        if accepted is not None:
            atoms, w, J, g = accepted
            atoms = np.asarray(atoms).copy()
            w = np.asarray(w).copy()
            accepted_J.append(J)
        if history is not None:
            history.append((t, sk, J, w.size, accepted is not None, j_acc))
        if oracle_budget > 0 and n_oracle >= oracle_budget:
            stopped = "budget"
            break
        if accepted is not None and stop_window > 0 and len(accepted_J) > stop_window:
            j0 = accepted_J[-stop_window - 1]
            if (j0 - J) / abs(j0) < stop_delta:
                stopped = "delta"
                break
    if info is not None:
        info.update(slots=slots, oracle_calls=n_oracle, stopped=stopped)
    return atoms, w, J
