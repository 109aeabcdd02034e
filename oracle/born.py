"""Born map, losses and gradients of atomic tomography (FP64 oracle).

Definitions followed (paper, problem-formulation and matrix-free sections):

* atomic density ``rho = sum_r alpha_r |psi_r><psi_r|``       (eq. atomic-density)
* Born probabilities ``pi_m = tr(E_m rho)``                    (eq. born-map)
* atom response ``a_m(psi) = <psi|E_m|psi>`` and ``pi = A alpha`` (eqs. atom-response,
  atomic-born-map)
* cross-entropy ``L = -sum_m pihat_m log(pi_m + eps)``          (eq. qst-loss)
* likelihood ratio ``c = pihat / (pi + eps)``                   (eq. likelihood-ratio-vector)
* weight gradient ``-A^T c``                                    (eq. weight-gradient)
* atom Wirtinger gradient ``-alpha_r G psi_r``                  (eq. atom-wirtinger-gradient)
* ``G = sum_m c_m E_m``                                         (eq. negative-gradient-matrix)
* atom step: ``pi~ = pi + alpha_r (a(psi~_r) - a(psi_r))``        (eqs. atom-trial, pi-update)

Interface convention (the paper stacks all settings into one POVM with the
factor ``1/B`` inside ``E_{b,u}``):  arrays handed around here are *per
setting* -- ``p[b, u] = <u|V_b rho V_b^dagger|u>`` and ``f[b, u] = N_{b,u}/N_s``,
each row summing to one -- and the losses act on the stacked vectors
``pi = p / B``, ``pihat = f / B``.  For generality every loss is reduced to the
per-outcome sensitivity ``g[b, u] = dL/dp[b, u]``; the gradients are then

* ``dL/dpsi_r^* = alpha_r sum_b V_b^dagger (g_b * V_b psi_r)``
* ``dL/dalpha_r = sum_{b,u} g[b, u] |(V_b psi_r)_u|^2``

which for cross-entropy equal ``-alpha_r G psi_r`` and ``-(A^T c)_r``.
The least-squares loss ``L = 1/2 ||pi - pihat||^2`` is not in the paper; it is
included as the second loss of the interface.
"""
from __future__ import annotations

import math

import numpy as np

from . import pauli

LOSS_CE, LOSS_LS, LOSS_NONE = 0, 1, 2


# ---------------------------------------------------------------- densities
def density(atoms: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """``rho = Psi diag(alpha) Psi^*`` (eq. atomic-density); ``atoms`` is ``[R][D]``."""
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    rho = np.zeros((atoms.shape[1], atoms.shape[1]), dtype=np.complex128)
    for r in range(atoms.shape[0]):
        rho += w[r] * np.outer(atoms[r], atoms[r].conj())
    return rho


# ---------------------------------------------------------------- forward
def probs_dense(atoms, weights, settings, table=None) -> np.ndarray:
    """Per-setting ``p[b,u] = B tr(E_{b,u} rho)`` from dense POVM effects (n <= 4).
    ``table``: the unitaries named by codes >= 3 (general local settings)."""
    settings = np.asarray(settings)
    B = settings.shape[0]
    E = pauli.povm_elements(settings, table)
    rho = density(atoms, weights)
    D = rho.shape[0]
    p = np.zeros((B, D))
    for b in range(B):
        for u in range(D):
            p[b, u] = B * np.real(np.trace(E[b, u] @ rho))
    return p


def atom_response_dense(atoms, settings, table=None) -> np.ndarray:
    """Stacked atom-response matrix ``A[m, r] = <psi_r|E_m|psi_r>`` (``M = B*D`` rows)."""
    settings = np.asarray(settings)
    E = pauli.povm_elements(settings, table)
    B, D = E.shape[0], E.shape[1]
    atoms = np.asarray(atoms, dtype=np.complex128)
    A = np.zeros((B * D, atoms.shape[0]))
    for b in range(B):
        for u in range(D):
            for r in range(atoms.shape[0]):
                A[b * D + u, r] = np.real(atoms[r].conj() @ E[b, u] @ atoms[r])
    return A


def probs_kron(atoms, weights, settings, table=None) -> np.ndarray:
    """``p[b,u] = sum_r alpha_r |(V_b psi_r)_u|^2`` with dense ``V_b`` (n <= 12)."""
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    p = np.zeros((settings.shape[0], atoms.shape[1]))
    for b in range(settings.shape[0]):
        V = pauli.setting_unitary(settings[b], table)
        for r in range(atoms.shape[0]):
            p[b] += w[r] * np.abs(V @ atoms[r]) ** 2
    return p


def rotate_axis(atoms, codes, table=None) -> np.ndarray:
    """``phi_r = V_b psi_r`` for every atom, per-axis contraction (any n)."""
    return np.stack([pauli.apply_setting_axis(codes, a, table=table) for a in np.asarray(atoms)])


def probs_axis(atoms, weights, settings, rows=None, table=None) -> np.ndarray:
    """``p[b,u]`` by per-axis contraction; ``rows`` restricts to a subset of settings."""
    settings = np.asarray(settings)
    w = np.asarray(weights, dtype=np.float64)
    rows = range(settings.shape[0]) if rows is None else rows
    out = []
    for b in rows:
        phi = rotate_axis(atoms, settings[b], table)
        out.append(np.einsum("r,ru->u", w, np.abs(phi) ** 2))
    return np.asarray(out)


# ---------------------------------------------------------------- atom step (response update)
def atom_response_axis(psi, settings, rows=None, table=None) -> np.ndarray:
    """One-atom response ``a(psi)[b, u] = |(V_b psi)_u|^2`` per setting (eq. atom-response in
    the per-setting layout, i.e. ``B`` times the stacked ``a_m(psi)``)."""
    psi = np.asarray(psi, dtype=np.complex128)
    return probs_axis(psi[None, :], np.ones(1), settings, rows, table=table)


def atom_trial_probs(atoms, weights, settings, r, psi_trial, p_t, rows=None, table=None) -> np.ndarray:
    """Probabilities after atom ``r`` is replaced by ``psi_trial`` (eq. atom-trial), by the
    response update of eq. pi-update: ``p~ = p_t + alpha_r d`` with the response difference
    ``d = a(psi_trial) - a(psi_r)``.  ``p_t`` holds the current probabilities of the rows used."""
    alpha_r = float(np.asarray(weights, dtype=np.float64)[r])
    d = (atom_response_axis(psi_trial, settings, rows, table)
         - atom_response_axis(np.asarray(atoms)[r], settings, rows, table))
    return np.asarray(p_t, dtype=np.float64) + alpha_r * d


def state_error(atoms_a, w_a, atoms_b, w_b) -> float:
    """Relative Frobenius error ``||rho_a - rho_b||_F / ||rho_b||_F`` (the error metric of the
    numerical-test section) from Gram matrices of the atoms, without dense densities:
    ``||sum_r a_r |u_r><u_r| ||_F^2 = sum_{r,r'} a_r a_r' |<u_r|u_r'>|^2``, and the cross term
    likewise."""
    ua = np.asarray(atoms_a, dtype=np.complex128)
    ub = np.asarray(atoms_b, dtype=np.complex128)
    wa = np.asarray(w_a, dtype=np.float64)
    wb = np.asarray(w_b, dtype=np.float64)

    def gram(u, a, v, b):
        return float(a @ (np.abs(u.conj() @ v.T) ** 2) @ b)

    aa, ab, bb = gram(ua, wa, ua, wa), gram(ua, wa, ub, wb), gram(ub, wb, ub, wb)
    return math.sqrt(max(aa - 2.0 * ab + bb, 0.0) / bb)


# ---------------------------------------------------------------- losses
def _sum(x: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    return math.fsum(x) if x.size <= (1 << 20) else float(np.sum(x))


def loss_and_sensitivity(p, f, B: int, kind: int, eps: float):
    """Loss on the stacked vectors ``pi = p/B``, ``pihat = f/B`` and ``g = dL/dp``.

    * CE (eq. qst-loss):  ``L = -sum pihat log(pi + eps)``;
      ``g = -(pihat/(pi+eps))/B = -c/B`` with ``c`` of eq. likelihood-ratio-vector.
      Outcomes with ``pihat = 0`` contribute nothing (``0 log x = 0``).
    * LS:  ``L = 1/2 sum (pi - pihat)^2``;  ``g = (pi - pihat)/B``.
    """
    p = np.asarray(p, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    pi, pih = p / B, f / B
    if kind == LOSS_CE:
        nz = pih > 0
        terms = np.zeros_like(pi)
        terms[nz] = -pih[nz] * np.log(pi[nz] + eps)
        c = np.zeros_like(pi)
        c[nz] = pih[nz] / (pi[nz] + eps)
        return _sum(terms), -c / B
    if kind == LOSS_LS:
        r = pi - pih
        return 0.5 * _sum(r * r), r / B
    raise ValueError("loss kind")


def likelihood_ratio(p, f, B: int, eps: float) -> np.ndarray:
    """``c = pihat / (pi + eps)`` (eq. likelihood-ratio-vector), per setting layout."""
    p = np.asarray(p, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    return (f / B) / (p / B + eps)


# ---------------------------------------------------------------- gradients
def gradients_dense(atoms, weights, settings, g, table=None):
    """Gradients from dense POVM effects (n <= 4), given ``g = dL/dp`` (per setting).

    With ``dL/dpi_m = B g_m``:  ``dL/dpsi_r^* = alpha_r sum_m (B g_m) E_m psi_r`` and
    ``dL/dalpha_r = sum_m (B g_m) <psi_r|E_m|psi_r>``.
    """
    settings = np.asarray(settings)
    E = pauli.povm_elements(settings, table)
    B, D = E.shape[0], E.shape[1]
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    R = atoms.shape[0]
    M = np.zeros((D, D), dtype=np.complex128)
    for b in range(B):
        for u in range(D):
            M += B * g[b, u] * E[b, u]
    ga = np.stack([w[r] * (M @ atoms[r]) for r in range(R)])
    gw = np.array([np.real(atoms[r].conj() @ M @ atoms[r]) for r in range(R)])
    return ga, gw


def gradient_matrix_dense(settings, g, table=None) -> np.ndarray:
    """``G = -grad_rho L = -sum_m (dL/dpi_m) E_m``; for CE this is ``sum_m c_m E_m``
    (eqs. density-gradient, negative-gradient-matrix)."""
    settings = np.asarray(settings)
    E = pauli.povm_elements(settings, table)
    B, D = E.shape[0], E.shape[1]
    G = np.zeros((D, D), dtype=np.complex128)
    for b in range(B):
        for u in range(D):
            G -= B * g[b, u] * E[b, u]
    return G


def gradients_kron(atoms, weights, settings, g, table=None):
    """Same gradients with dense per-setting ``V_b`` (n <= 12)."""
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    R, D = atoms.shape
    ga = np.zeros((R, D), dtype=np.complex128)
    gw = np.zeros(R)
    for b in range(settings.shape[0]):
        V = pauli.setting_unitary(settings[b], table)
        for r in range(R):
            phi = V @ atoms[r]
            ga[r] += w[r] * (V.conj().T @ (g[b] * phi))
            gw[r] += np.sum(g[b] * np.abs(phi) ** 2)
    return ga, gw


def gradients_axis(atoms, weights, settings, g, rows=None, table=None):
    """Same gradients by per-axis contraction; ``rows`` selects a subset of settings
    (``g`` then has one row per selected setting).  The adjoint is a sum over
    settings, so a subset gives the exact partial sum."""
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    rows = list(range(settings.shape[0])) if rows is None else list(rows)
    R, D = atoms.shape
    ga = np.zeros((R, D), dtype=np.complex128)
    gw = np.zeros(R)
    for i, b in enumerate(rows):
        for r in range(R):
            phi = pauli.apply_setting_axis(settings[b], atoms[r], table=table)
            ga[r] += w[r] * pauli.apply_setting_axis(settings[b], g[i] * phi, adjoint=True, table=table)
            gw[r] += np.sum(g[i] * np.abs(phi) ** 2)
    return ga, gw


def apply_gradient_matrix_axis(settings, g, v, table=None) -> np.ndarray:
    """Matrix-free ``G v = -sum_b V_b^dagger (g_b * V_b v)`` (eq. negative-gradient-product)."""
    settings = np.asarray(settings)
    out = np.zeros(np.asarray(v).shape[0], dtype=np.complex128)
    for b in range(settings.shape[0]):
        out -= pauli.apply_setting_axis(settings[b], g[b] * pauli.apply_setting_axis(settings[b], v, table=table),
                                        adjoint=True, table=table)
    return out


def tangent_project(atoms, atom_grad) -> np.ndarray:
    """``(I - psi_r psi_r^*) grad_r`` per atom (tangent space of the complex sphere,
    eq. atom-projected-descent-direction; for CE this is ``-d_r``)."""
    atoms = np.asarray(atoms, dtype=np.complex128)
    atom_grad = np.asarray(atom_grad, dtype=np.complex128)
    out = np.empty_like(atom_grad)
    for r in range(atoms.shape[0]):
        out[r] = atom_grad[r] - atoms[r] * (atoms[r].conj() @ atom_grad[r])
    return out


# ---------------------------------------------------------------- composite
def forward_backward(atoms, weights, settings, f, kind: int, eps: float, tier: str = "axis",
                     grad_p=None, table=None):
    """Loss, per-setting probabilities and both gradients, by the chosen tier.

    If ``grad_p`` is given it is used as ``g`` (generic mode, loss = None).  ``table``
    holds the unitaries of codes >= 3 (general local settings)."""
    settings = np.asarray(settings)
    B = settings.shape[0]
    probs = {"dense": probs_dense, "kron": probs_kron, "axis": probs_axis}[tier](atoms, weights, settings,
                                                                                  table=table)
    if grad_p is None:
        L, g = loss_and_sensitivity(probs, f, B, kind, eps)
    else:
        L, g = None, np.asarray(grad_p, dtype=np.float64)
    grads = {"dense": gradients_dense, "kron": gradients_kron, "axis": gradients_axis}[tier]
    ga, gw = grads(atoms, weights, settings, g, table=table)
    return L, probs, ga, gw
