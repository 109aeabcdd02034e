"""Spectral refactorisation (FP64 oracle): density proposal, Ritz pairs, spectral
candidates and proximal-surrogate selection (algorithm section, update rules for
``t`` in ``T_rho``; Theorem 1).

* density proposal ``S = rho + eta_rho G``                    (eq. density-proposal)
* matrix-free ``S v = sum_r alpha_r psi_r <psi_r|v> + eta_rho G v``  (eq. density-product)
* leading Ritz pairs ``(lambda_l, phi_l)``, ``l = 1..L``, non-increasing  (eq. ritz-pairs)
* candidates ``X^(s) = P_tau(proj_{Delta_s}(lambda_{1..s}), Phi_s)``  (eq. spectral-candidates)
* surrogate ``Q(X) = ||rho_X - S||_F^2 / (2 eta_rho) + mu R``  (eq. proximal-surrogate)
* selection ``s* = argmin_s Q(X^(s))``                        (eq. spectral-selection)

Readings where the paper is silent:

* Lanczos starts from a caller-supplied vector (the random draw is an input),
  uses full re-orthogonalisation (two passes of classical Gram-Schmidt per
  step), runs ``k = min(n_lanczos, D)`` steps and stops early only on an exact
  invariant subspace (``beta_j`` below ``1e-13`` times the running scale).
* Residuals are reported as ``|beta_k y_{k,l}|`` (the standard Lanczos
  residual bound of a Ritz pair).
* ``Q`` is evaluated without dense matrices through the Rayleigh-Ritz
  identity ``phi_l^* S phi_l = lambda_l`` for orthonormal Ritz vectors:
  ``||rho_X - S||^2 = sum beta_l^2 - 2 sum beta_l lambda_l + ||S||^2``; the
  constant ``||S||^2`` is dropped (it does not move the argmin).
* Ties in ``s*`` go to the smallest ``s``.
"""
from __future__ import annotations

import numpy as np

from . import born, simplex


# ---------------------------------------------------------------- dense (Theorem 1)
def density_proposal(rho, G, eta_rho: float):
    """``S = rho + eta_rho G`` (eq. density-proposal)."""
    return np.asarray(rho) + eta_rho * np.asarray(G)


def surrogate_dense(rho_X, S, eta_rho: float, mu: float, R: int) -> float:
    """``Q(X) = ||rho_X - S||_F^2/(2 eta_rho) + mu R`` (eq. proximal-surrogate), dense."""
    d = np.asarray(rho_X) - np.asarray(S)
    return float(np.real(np.vdot(d, d))) / (2.0 * eta_rho) + mu * R


def candidates_from_pairs(lams, vecs, L: int, tau: float):
    """Spectral candidates from the leading pairs (``lams`` non-increasing, ``vecs[l]`` = phi_l)."""
    out = []
    for s in range(1, L + 1):
        beta = simplex.project_simplex(lams[:s])
        keep, bc = simplex.prune(beta, tau)
        out.append(dict(s=s, keep=keep, weights=bc, atoms=np.asarray(vecs)[keep], lams=np.asarray(lams)[keep]))
    return out


def exact_spectral_step(S, L: int, eta_rho: float, mu: float, tau: float):
    """Complete-information spectral step of Theorem 1 (dense ``eigh`` of ``S``).

    Returns ``(chosen, candidates, scores)``; scores use the dense surrogate."""
    lam, U = np.linalg.eigh(np.asarray(S))
    order = np.argsort(lam)[::-1][:L]
    lams, vecs = lam[order], U[:, order].T
    cands = candidates_from_pairs(lams, vecs, L, tau)
    scores = []
    for c in cands:
        rho_X = born.density(c["atoms"], c["weights"])
        scores.append(surrogate_dense(rho_X, S, eta_rho, mu, len(c["keep"])))
    s_star = int(np.argmin(scores))
    return cands[s_star], cands, np.asarray(scores)


# ---------------------------------------------------------------- Lanczos
def lanczos(apply_S, v0, k: int):
    """``k`` steps of Hermitian Lanczos with full re-orthogonalisation.

    Returns ``(a, b, Q)``: diagonal ``a[k']``, off-diagonal ``b[k']`` (``b[j]`` couples
    ``q_j`` and ``q_{j+1}``; ``b[k'-1]`` is the final residual norm) and the basis
    ``Q[k'][D]``; ``k' <= k`` is smaller only on an invariant subspace.
    """
    v0 = np.asarray(v0, dtype=np.complex128)
    q = v0 / np.linalg.norm(v0)
    Q, a, b = [q], [], []
    scale = 0.0
    for j in range(k):
        w = apply_S(Q[j])
        aj = float(np.real(np.vdot(Q[j], w)))
        w = w - aj * Q[j]
        if j > 0:
            w = w - b[j - 1] * Q[j - 1]
        Qm = np.asarray(Q)
        for _ in range(2):
            w = w - Qm.T @ (Qm.conj() @ w)
        bj = float(np.linalg.norm(w))
        a.append(aj)
        b.append(bj)
        scale = max(scale, abs(aj), bj)
        if j + 1 == k or bj <= 1e-13 * max(scale, 1e-300):
            break
        Q.append(w / bj)
    return np.asarray(a), np.asarray(b), np.asarray(Q[: len(a)])


def ritz_pairs(a, b, Q, L: int):
    """Top-``L`` Ritz values (non-increasing), Ritz vectors ``[L][D]`` and residual bounds."""
    k = len(a)
    T = np.diag(a) + np.diag(b[: k - 1], 1) + np.diag(b[: k - 1], -1)
    theta, Y = np.linalg.eigh(T)
    order = np.argsort(theta)[::-1][: min(L, k)]
    theta, Y = theta[order], Y[:, order]
    vecs = (Q.T @ Y).T
    resid = np.abs(b[k - 1] * Y[k - 1, :])
    return theta, vecs, resid


def surrogate_ritz(weights, lams, eta_rho: float, mu: float) -> float:
    """``Q`` via the Rayleigh-Ritz identity, without the constant ``||S||^2/(2 eta_rho)``."""
    w = np.asarray(weights, dtype=np.float64)
    return (float(np.sum(w * w)) - 2.0 * float(np.sum(w * np.asarray(lams)))) / (2.0 * eta_rho) + mu * w.size


def lanczos_refactor(atoms, weights, settings, f, kind: int, eps: float, eta_rho: float, mu: float,
                     tau: float, L_max: int, n_lanczos: int, v0):
    """Matrix-free spectral refactorisation of the current state ``(alpha, Psi)``.

    ``G`` comes from the current probabilities and the data ``f`` (per-setting
    layout); ``v0`` is the Lanczos start vector.  Returns a dict with the Ritz
    values / residuals, per-candidate scores, ``s_star`` (0-based) and the chosen
    candidate's ``atoms``, ``weights`` and rank ``R``.
    """
    settings = np.asarray(settings)
    atoms = np.asarray(atoms, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    B = settings.shape[0]
    D = atoms.shape[1]
    p = born.probs_axis(atoms, w, settings)
    _, g = born.loss_and_sensitivity(p, f, B, kind, eps)

    def apply_S(v):
        low_rank = np.zeros(D, dtype=np.complex128)
        for r in range(atoms.shape[0]):
            low_rank += w[r] * atoms[r] * np.vdot(atoms[r], v)
        return low_rank + eta_rho * born.apply_gradient_matrix_axis(settings, g, v)

    a, b, Q = lanczos(apply_S, v0, min(n_lanczos, D))
    theta, vecs, resid = ritz_pairs(a, b, Q, L_max)
    L = theta.size
    cands = candidates_from_pairs(theta, vecs, L, tau)
    scores = np.array([surrogate_ritz(c["weights"], c["lams"], eta_rho, mu) for c in cands])
    s_star = int(np.argmin(scores))
    ch = cands[s_star]
    return dict(ritz_vals=theta, ritz_resid=resid, q_scores=scores, s_star=s_star,
                atoms=ch["atoms"], weights=ch["weights"], R=len(ch["keep"]), lanczos_steps=len(a))
