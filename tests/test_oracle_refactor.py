"""Pins of the spectral refactorisation: Theorem 1 (i)-(iii) with dense
eigendecompositions, Lanczos = exact spectrum on a full Krylov space, and exact
recovery of a pure state from noiseless, informationally complete data."""
import numpy as np

import synth
from oracle import born, loop, pauli, refactor, simplex


def _state(rng, N, R):
    atoms = synth.haar_atoms(rng, R, 1 << N)
    return atoms, synth.dirichlet_weights(rng, R)


def _random_feasible(rng, D, R):
    atoms = synth.haar_atoms(rng, R, D)
    w = rng.dirichlet(np.ones(R) * rng.choice([0.2, 1.0, 5.0]))
    return born.density(atoms, w)


def _setup(seed, N=3, R=3, kind=born.LOSS_CE):
    rng = synth.make_rng(seed)
    atoms, w = _state(rng, N, R)
    s = synth.all_settings(N)
    truth, wt = _state(rng, N, 2)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), 500)
    p = born.probs_axis(atoms, w, s)
    _, g = born.loss_and_sensitivity(p, f, s.shape[0], kind, 1e-8)
    G = born.gradient_matrix_dense(s, g)
    return rng, atoms, w, s, f, G


def test_theorem1_rank_capped_frobenius_optimality():
    rng, atoms, w, s, f, G = _setup(41)
    D = atoms.shape[1]
    S = refactor.density_proposal(born.density(atoms, w), G, 0.5)
    _, cands, _ = refactor.exact_spectral_step(S, 4, 0.5, 1e-3, 0.0)
    for c in cands:
        best = np.linalg.norm(born.density(c["atoms"], c["weights"]) - S)
        for _ in range(1500):
            rho = _random_feasible(rng, D, int(rng.integers(1, c["s"] + 1)))
            assert np.linalg.norm(rho - S) >= best - 1e-12
        # Local perturbations of the candidate stay feasible and cannot do better.
        for _ in range(300):
            a = c["atoms"] + 0.05 * (rng.standard_normal(c["atoms"].shape) + 1j * rng.standard_normal(c["atoms"].shape))
            a /= np.linalg.norm(a, axis=1, keepdims=True)
            wt = simplex.project_simplex(c["weights"] + 0.05 * rng.standard_normal(c["weights"].size))
            assert np.linalg.norm(born.density(a, wt) - S) >= best - 1e-12


def test_theorem1_selected_candidate_minimises_surrogate():
    rng, atoms, w, s, f, G = _setup(42)
    D = atoms.shape[1]
    eta, mu = 0.3, 2e-3
    S = refactor.density_proposal(born.density(atoms, w), G, eta)
    ch, cands, scores = refactor.exact_spectral_step(S, 4, eta, mu, 0.0)
    q_star = scores.min()
    for _ in range(3000):
        R = int(rng.integers(1, 5))
        a = synth.haar_atoms(rng, R, D)
        wt = rng.dirichlet(np.ones(R))
        q = refactor.surrogate_dense(born.density(a, wt), S, eta, mu, R)
        assert q >= q_star - 1e-12


def test_theorem1_descent_least_squares():
    # LS loss: rho -> L(pi(rho)) has Lipschitz gradient with constant ||Born map||^2; with
    # eta < 1/L the exact proximal step does not increase J (Theorem 1 (iii)).
    rng = synth.make_rng(43)
    N = 2
    s = synth.all_settings(N)
    B = s.shape[0]
    E = pauli.povm_elements(s).reshape(-1, 4, 4)
    X = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    X = X + X.conj().T
    for _ in range(200):  # power iteration on A^* A (rho -> sum_m tr(E_m rho) E_m)
        X = np.einsum("m,mij->ij", np.real(np.einsum("mij,ji->m", E, X)), E)
        X /= np.linalg.norm(X)
    Lip = np.linalg.norm(np.einsum("m,mij->ij", np.real(np.einsum("mij,ji->m", E, X)), E))
    truth, wt = _state(rng, N, 1)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), 200)
    mu = 1e-3
    for trial in range(10):
        atoms, w = _state(rng, N, 3)
        p = born.probs_axis(atoms, w, s)
        L0, g = born.loss_and_sensitivity(p, f, B, born.LOSS_LS, 0.0)
        J0 = L0 + mu * w.size
        eta = 0.9 / Lip
        S = refactor.density_proposal(born.density(atoms, w), born.gradient_matrix_dense(s, g), eta)
        ch, _, _ = refactor.exact_spectral_step(S, 4, eta, mu, 0.0)
        L1, _ = born.loss_and_sensitivity(born.probs_axis(ch["atoms"], ch["weights"], s), f, B, born.LOSS_LS, 0.0)
        J1 = L1 + mu * len(ch["keep"])
        rho1 = born.density(ch["atoms"], ch["weights"])
        bound = J0 - (1 / (2 * eta) - Lip / 2) * np.linalg.norm(rho1 - born.density(atoms, w)) ** 2
        assert J1 <= bound + 1e-12


def test_lanczos_full_space_equals_exact_step():
    rng, atoms, w, s, f, G = _setup(44)
    D = atoms.shape[1]
    eta, mu, tau = 0.4, 1e-3, 1e-3
    v0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    res = refactor.lanczos_refactor(atoms, w, s, f, born.LOSS_CE, 1e-8, eta, mu, tau, 4, D, v0)
    S = refactor.density_proposal(born.density(atoms, w), G, eta)
    lam = np.sort(np.linalg.eigvalsh(S))[::-1][:4]
    assert np.allclose(res["ritz_vals"], lam, atol=1e-10)
    assert np.all(res["ritz_resid"] < 1e-8)
    ch, _, scores = refactor.exact_spectral_step(S, 4, eta, mu, tau)
    const = np.linalg.norm(S) ** 2 / (2 * eta)
    assert np.allclose(res["q_scores"] + const, scores, atol=1e-9)
    assert res["R"] == len(ch["keep"])
    # Atoms match only up to a phase each: compare the densities.
    assert np.allclose(born.density(res["atoms"], res["weights"]), born.density(ch["atoms"], ch["weights"]), atol=1e-9)


def test_exact_recovery_noiseless_pure_state():
    # Noiseless data from a pure state with all 3^N Pauli strings (informationally complete).
    # With the paper's acceptance margin tau_acc = 1e-10 progress stops once a step gains less
    # than the margin (infidelity ~1e-11 here); with tau_acc = 0 the iteration reaches the truth
    # to rounding.  For pure states e_rho = sqrt(2 (1 - |<psi_hat|psi_*>|^2)).
    rng = synth.make_rng(45)
    N = 2
    s = synth.all_settings(N)
    truth, _ = _state(rng, N, 1)
    f = born.probs_axis(truth, [1.0], s)
    atoms, w = _state(rng, N, 2)
    rho_star = born.density(truth, [1.0])
    for tau_acc, max_infid, max_err in ((1e-10, 1e-8, 2e-4), (0.0, 1e-13, 1e-6)):
        out_atoms, out_w, J = loop.run(atoms, w, s, f, kind=born.LOSS_CE, eps=0.0, mu=1e-3, tau_acc=tau_acc,
                                       iters=80, t_ref=4, t_alpha=3, rng=synth.make_rng(1))
        rho_hat = born.density(out_atoms, out_w)
        e_rho = np.linalg.norm(rho_hat - rho_star) / np.linalg.norm(rho_star)
        assert out_w.size == 1
        assert 1 - abs(np.vdot(out_atoms[0], truth[0])) ** 2 < max_infid
        assert e_rho < max_err


def test_lanczos_basis_orthonormal_and_tridiagonal():
    # Hermitian matrix with a clustered spectrum: without re-orthogonalisation the Lanczos
    # basis loses orthogonality after a few converged Ritz values.  Pins Q Q^* = I and
    # Q S Q^* = T, and that the extreme Ritz values converge to the true extremes.
    rng = synth.make_rng(46)
    D, k = 256, 30
    lam = np.concatenate([[3.0, 2.9, 2.85], rng.uniform(-1, 1, D - 3)])
    U, _ = np.linalg.qr(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)))
    S = (U * lam) @ U.conj().T
    v0 = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    a, b, Q = refactor.lanczos(lambda v: S @ v, v0, k)
    assert len(a) == k
    assert np.abs(Q.conj() @ Q.T - np.eye(k)).max() < 1e-12
    T = np.diag(a) + np.diag(b[: k - 1], 1) + np.diag(b[: k - 1], -1)
    assert np.abs(Q.conj() @ S @ Q.T - T).max() < 1e-12
    theta, vecs, resid = refactor.ritz_pairs(a, b, Q, 3)
    assert abs(theta[0] - 3.0) < 1e-8
    for l in range(3):
        assert abs(np.linalg.norm(S @ vecs[l] - theta[l] * vecs[l]) - resid[l]) < 1e-10
