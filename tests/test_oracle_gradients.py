"""Pins of the oracle's adjoint (atom Wirtinger gradient, weight gradient,
density-level gradient) against finite differences, closed forms and the
dense POVM definition."""
import numpy as np
import pytest

import synth
from oracle import born, pauli


def _instance(seed, N, R, B, shots=2000, exhaustive=False):
    rng = synth.make_rng(seed)
    D = 1 << N
    truth = synth.haar_atoms(rng, 2, D)
    wt = synth.dirichlet_weights(rng, 2)
    s = synth.all_settings(N) if exhaustive else synth.random_settings(rng, B, N)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), shots)
    atoms = synth.haar_atoms(rng, R, D)
    w = synth.dirichlet_weights(rng, R)
    return atoms, w, s, f, rng


def _loss(atoms, w, s, f, kind, eps):
    p = born.probs_axis(atoms, w, s)
    return born.loss_and_sensitivity(p, f, s.shape[0], kind, eps)[0]


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_atom_gradient_central_fd(kind):
    atoms, w, s, f, rng = _instance(21, 5, 3, 12)
    eps = 1e-8
    L, _, ga, gw = born.forward_backward(atoms, w, s, f, kind, eps, tier="axis")
    h = 1e-6
    for r in range(atoms.shape[0]):
        d = rng.standard_normal(atoms.shape[1]) + 1j * rng.standard_normal(atoms.shape[1])
        ap, am = atoms.copy(), atoms.copy()
        ap[r] += h * d
        am[r] -= h * d
        fd = (_loss(ap, w, s, f, kind, eps) - _loss(am, w, s, f, kind, eps)) / (2 * h)
        an = 2 * np.real(np.vdot(ga[r], d))  # dL = 2 Re <dL/dpsi^*, delta>
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-12) + 1e-12, (r, fd, an)


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_weight_gradient_central_fd(kind):
    atoms, w, s, f, _ = _instance(22, 4, 3, 10)
    eps = 1e-8
    _, _, _, gw = born.forward_backward(atoms, w, s, f, kind, eps, tier="axis")
    h = 1e-6
    for r in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[r] += h
        wm[r] -= h
        fd = (_loss(atoms, wp, s, f, kind, eps) - _loss(atoms, wm, s, f, kind, eps)) / (2 * h)
        assert abs(fd - gw[r]) <= 1e-7 * abs(gw[r]) + 1e-12


def test_tiers_agree_and_match_dense_definitions():
    atoms, w, s, f, _ = _instance(23, 3, 2, 0, exhaustive=True)
    eps = 1e-8
    res = {t: born.forward_backward(atoms, w, s, f, born.LOSS_CE, eps, tier=t) for t in ("dense", "kron", "axis")}
    for t in ("kron", "axis"):
        assert abs(res[t][0] - res["dense"][0]) < 1e-13
        assert np.allclose(res[t][2], res["dense"][2], atol=1e-13)
        assert np.allclose(res[t][3], res["dense"][3], atol=1e-13)
    # CE: dL/dalpha = -A^T c and dL/dpsi^* = -alpha_r G psi_r with G = sum c_m E_m.
    B = s.shape[0]
    p = res["dense"][1]
    c = born.likelihood_ratio(p, f, B, eps).reshape(-1)
    A = born.atom_response_dense(atoms, s)
    assert np.allclose(res["dense"][3], -(A.T @ c), atol=1e-13)
    E = pauli.povm_elements(s).reshape(-1, 8, 8)
    G = np.einsum("m,mij->ij", c, E)
    for r in range(atoms.shape[0]):
        assert np.allclose(res["dense"][2][r], -w[r] * (G @ atoms[r]), atol=1e-13)
    _, g = born.loss_and_sensitivity(p, f, B, born.LOSS_CE, eps)
    assert np.allclose(born.gradient_matrix_dense(s, g), G, atol=1e-13)
    # Matrix-free G v equals the dense product.
    v = atoms[0] + 0.3j * atoms[1]
    assert np.allclose(born.apply_gradient_matrix_axis(s, g, v), G @ v, atol=1e-13)


def test_adjoint_closed_forms_any_n():
    rng = synth.make_rng(24)
    N, R, B = 10, 2, 7
    D = 1 << N
    atoms = synth.haar_atoms(rng, R, D)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, N)
    # g = 1: sum_b V_b^dagger V_b = B I, so dL/dpsi_r^* = alpha_r B psi_r; dL/dalpha_r = B ||psi_r||^2.
    ga, gw = born.gradients_axis(atoms, w, s, np.ones((B, D)))
    for r in range(R):
        assert np.allclose(ga[r], w[r] * B * atoms[r], atol=1e-12)
        assert abs(gw[r] - B) < 1e-11
    # g = (-1)^{u_j}: V^dagger diag(1,-1) V = sigma, so the gradient is alpha_r sum_b sigma^(j)_{s_bj} psi_r.
    j = 3
    sign = np.array([1.0 - 2.0 * ((u >> (N - 1 - j)) & 1) for u in range(D)])
    ga, _ = born.gradients_axis(atoms, w, s, np.tile(sign, (B, 1)))
    for r in range(R):
        want = np.zeros(D, dtype=np.complex128)
        t = atoms[r].reshape((2,) * N)
        for b in range(B):
            op = pauli.SIGMA[int(s[b, j])]
            want += np.moveaxis(np.tensordot(op, t, axes=([1], [j])), 0, j).reshape(-1)
        assert np.allclose(ga[r], w[r] * want, atol=1e-12)
    # Dot-product test <V x, y> = <x, V^dagger y>.
    x = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    y = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    for b in range(B):
        lhs = np.vdot(pauli.apply_setting_axis(s[b], x), y)
        rhs = np.vdot(x, pauli.apply_setting_axis(s[b], y, adjoint=True))
        assert abs(lhs - rhs) < 1e-11


def test_stationarity_at_noiseless_truth():
    # f = p exactly, CE with eps = 0: c = 1 wherever p > 0, so G = I and dL/dpsi_r^* = -alpha_r psi_r;
    # the tangent part vanishes.  LS with f = p: both gradients vanish.
    rng = synth.make_rng(25)
    N, R = 3, 2
    atoms = synth.haar_atoms(rng, R, 1 << N)
    w = synth.dirichlet_weights(rng, R)
    s = synth.all_settings(N)
    p = born.probs_axis(atoms, w, s)
    _, _, ga, gw = born.forward_backward(atoms, w, s, p, born.LOSS_CE, 0.0)
    for r in range(R):
        assert np.allclose(ga[r], -w[r] * atoms[r], atol=1e-13)
    assert np.allclose(born.tangent_project(atoms, ga), 0, atol=1e-13)
    assert np.allclose(gw, -1.0, atol=1e-13)  # -A^T c with c = 1 and columns of A on the simplex
    _, _, ga, gw = born.forward_backward(atoms, w, s, p, born.LOSS_LS, 0.0)
    assert np.allclose(ga, 0, atol=1e-15) and np.allclose(gw, 0, atol=1e-15)


def test_cross_entropy_minimised_at_data():
    # Gibbs: for eps = 0, sum_u f log p <= sum_u f log f, so the CE loss over each setting's
    # simplex is minimised at p = f (catches sign / placement mistakes in the loss).
    rng = synth.make_rng(26)
    B, D = 5, 16
    f = rng.dirichlet(np.ones(D), size=B)
    L0, _ = born.loss_and_sensitivity(f, f, B, born.LOSS_CE, 0.0)
    for _ in range(20):
        q = rng.dirichlet(np.ones(D), size=B)
        L, _ = born.loss_and_sensitivity(q, f, B, born.LOSS_CE, 0.0)
        assert L >= L0 - 1e-15
    L0, g0 = born.loss_and_sensitivity(f, f, B, born.LOSS_LS, 0.0)
    assert L0 == 0.0 and not g0.any()
