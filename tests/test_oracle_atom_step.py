"""Pins of the oracle's atom-step response update (eqs. atom-trial, pi-update):
p~ = p_t + alpha_r (a(psi~) - a(psi_r)).  Checked against a full recomputation of the
replaced mixture by the dense-unitary tier (a different route), against exact identities
and against closed forms -- never against itself."""
import numpy as np

import synth
from oracle import born


def _case(seed, n, R, B):
    rng = synth.make_rng(seed)
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex128)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    trial = synth.haar_atoms(rng, 1, 1 << n, dtype=np.complex128)[0]
    return atoms, w, s, trial


def test_update_equals_full_recomputation():
    # the incremental form must reproduce the replaced mixture's Born map, computed here
    # with dense per-setting unitaries (probs_kron), not the per-axis contraction
    for seed, (n, R, B) in enumerate([(3, 2, 9), (5, 4, 7), (7, 3, 5)]):
        atoms, w, s, trial = _case(100 + seed, n, R, B)
        p_t = born.probs_kron(atoms, w, s)
        for r in range(R):
            got = born.atom_trial_probs(atoms, w, s, r, trial, p_t)
            rep = atoms.copy()
            rep[r] = trial
            ref = born.probs_kron(rep, w, s)
            assert np.max(np.abs(got - ref)) < 1e-13, (n, r)


def test_same_atom_leaves_probabilities_unchanged():
    # d = a(psi_r) - a(psi_r) is exactly zero in floating point
    atoms, w, s, _ = _case(120, 6, 3, 8)
    p_t = born.probs_axis(atoms, w, s)
    for r in range(3):
        assert np.array_equal(born.atom_trial_probs(atoms, w, s, r, atoms[r], p_t), p_t)


def test_response_rows_sum_to_the_squared_norm():
    # V_b is unitary: every row of a(psi) sums to ||psi||^2, also for an unnormalised psi
    rng = synth.make_rng(130)
    s = synth.random_settings(rng, 11, 6)
    psi = 1.7 * synth.haar_atoms(rng, 1, 64, dtype=np.complex128)[0]
    a = born.atom_response_axis(psi, s)
    assert np.allclose(a.sum(axis=1), 1.7 ** 2, rtol=0, atol=1e-13)
    assert (a >= 0).all()


def test_closed_form_basis_state_trial():
    # psi~ = |0...0>: all-Z gives the point mass at u = 0, all-X the uniform row 1/D; with
    # p_t from a product state |+>^n (uniform under all-Z, point mass under all-X) the
    # update is written out by hand.
    n, D = 4, 16
    plus = np.full(D, 0.25, dtype=np.complex128)
    zero = np.zeros(D, dtype=np.complex128)
    zero[0] = 1.0
    s = np.array([[2] * n, [0] * n], dtype=np.uint8)
    atoms = np.stack([plus, zero])
    w = np.array([0.25, 0.75])
    p_t = np.zeros((2, D))
    p_t[0] = 0.25 / D
    p_t[0, 0] += 0.75
    p_t[1] = 0.75 / D
    p_t[1, 0] += 0.25
    assert np.allclose(born.probs_axis(atoms, w, s), p_t, atol=1e-15)
    got = born.atom_trial_probs(atoms, w, s, 0, zero, p_t)  # replace |+>^n by |0...0>
    want = np.zeros((2, D))
    want[0, 0] = 1.0        # both atoms are |0...0>: point mass under all-Z
    want[1] = 1.0 / D       # and uniform under all-X
    assert np.allclose(got, want, atol=1e-15)


def test_update_is_linear_in_the_weight():
    # p~ - p_t scales with alpha_r and flips sign when the two atoms trade places
    atoms, w, s, trial = _case(140, 5, 3, 6)
    p_t = born.probs_axis(atoms, w, s)
    d1 = born.atom_trial_probs(atoms, w, s, 1, trial, p_t) - p_t
    w2 = w.copy()
    w2[1] *= 3.0
    d3 = born.atom_trial_probs(atoms, w2, s, 1, trial, p_t) - p_t
    assert np.allclose(d3, 3.0 * d1, atol=1e-14)
    rep = atoms.copy()
    rep[1] = trial
    back = born.atom_trial_probs(rep, w, s, 1, atoms[1], p_t) - p_t
    assert np.allclose(back, -d1, atol=1e-14)


def test_state_error_gram_form_matches_dense():
    # the Gram form against dense densities and the Frobenius norm (numpy), plus closed forms
    rng = synth.make_rng(150)
    for n, Ra, Rb in ((3, 2, 3), (5, 4, 1), (6, 1, 1)):
        ua = synth.haar_atoms(rng, Ra, 1 << n)
        ub = synth.haar_atoms(rng, Rb, 1 << n)
        wa = synth.dirichlet_weights(rng, Ra)
        wb = synth.dirichlet_weights(rng, Rb)
        ra, rb = born.density(ua, wa), born.density(ub, wb)
        want = np.linalg.norm(ra - rb) / np.linalg.norm(rb)
        assert abs(born.state_error(ua, wa, ub, wb) - want) < 1e-12
        assert born.state_error(ua, wa, ua, wa) < 1e-7
    e0 = np.eye(4, dtype=np.complex128)
    assert abs(born.state_error(e0[:1], [1.0], e0[1:2], [1.0]) - np.sqrt(2.0)) < 1e-15  # orthogonal pure states
