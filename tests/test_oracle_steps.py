"""Pins of the oracle's update steps away from stationarity: the tangent projection
(eq. atom-projected-descent-direction), the atom direction and trial curve (eqs.
atom-direction, atom-trial), the coefficient direction (eqs. h_t,
coefficient-update) and the slot schedule (eq. iteration-partition, Algorithm 1).

The directions are pinned by first-order calculus rather than by their formulas: along
the oracle's own trial curve the objective must fall at the rate the gradient
predicts (a wrong sign makes it rise, a wrong conjugation moves the curve off the
tangent space), measured by central finite differences of the FP64 objective."""
import numpy as np
import pytest

import synth
from oracle import born, loop


def _problem(seed, n=4, R=3, B=20, shots=500):
    rng = synth.make_rng(seed)
    s = synth.random_settings(rng, B, n)
    truth = synth.haar_atoms(rng, 2, 1 << n)
    wt = synth.dirichlet_weights(rng, 2)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), shots).astype(np.float64)
    atoms = synth.haar_atoms(rng, R, 1 << n)
    w = synth.dirichlet_weights(rng, R)
    return atoms, w, s, f, rng


def _J(atoms, w, s, f, kind, eps, mu=1e-3):
    return loop.objective(atoms, w, s, f, kind, eps, mu)[0]


def test_tangent_projection_on_random_vectors():
    rng = synth.make_rng(301)
    R, D = 4, 32
    atoms = synth.haar_atoms(rng, R, D)
    g = rng.standard_normal((R, D)) + 1j * rng.standard_normal((R, D))
    t = born.tangent_project(atoms, g)
    for r in range(R):
        # orthogonal to its own atom (the inner product <psi, g> is complex here)
        assert abs(np.vdot(g[r], atoms[r]).imag) > 1e-2
        assert abs(np.vdot(atoms[r], t[r])) < 1e-13
        # the removed part is along psi_r: g - t is a multiple of psi_r
        c = np.vdot(atoms[r], g[r] - t[r])
        assert np.allclose(g[r] - t[r], c * atoms[r], atol=1e-13)
    # idempotent
    assert np.allclose(born.tangent_project(atoms, t), t, atol=1e-13)
    # a complex multiple of the atom projects to zero; a vector orthogonal to it is kept
    c = 0.7 - 1.3j
    assert np.allclose(born.tangent_project(atoms, c * atoms), 0.0, atol=1e-13)
    assert np.allclose(born.tangent_project(atoms, t), t, atol=1e-13)
    # the dense projector (I - psi psi^*) as a matrix gives the same vector
    for r in range(R):
        P = np.eye(D) - np.outer(atoms[r], atoms[r].conj())
        assert np.allclose(P @ g[r], t[r], atol=1e-13)


def test_tangent_projection_of_a_non_stationary_gradient():
    atoms, w, s, f, _ = _problem(302)
    _, _, ga, _ = born.forward_backward(atoms, w, s, f, born.LOSS_CE, 1e-8)
    t = born.tangent_project(atoms, ga)
    for r in range(atoms.shape[0]):
        assert np.linalg.norm(t[r]) > 1e-3 * np.linalg.norm(ga[r])  # far from stationarity
        assert abs(np.vdot(atoms[r], t[r])) < 1e-13 * np.linalg.norm(ga[r])


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_atom_direction_descends_at_the_predicted_rate(kind):
    # Along psi(eta) = (psi + eta d)/||psi + eta d|| with d orthogonal to a unit psi,
    # dpsi/deta = d at eta = 0, so dJ/deta = 2 Re <dL/dpsi^*, d> = -2 ||d||^2 when
    # d = -(I - psi psi^*) dL/dpsi^*.
    atoms, w, s, f, _ = _problem(303)
    eps = 1e-8
    _, g = loop.objective(atoms, w, s, f, kind, eps, 1e-3)
    h = 1e-5
    for r in range(atoms.shape[0]):
        d = loop.atom_direction(atoms, w, s, g, r)
        assert abs(np.vdot(atoms[r], d)) < 1e-12 * np.linalg.norm(d)
        ap, am = atoms.copy(), atoms.copy()
        ap[r] = loop.atom_trial(atoms[r], d, h)
        am[r] = loop.atom_trial(atoms[r], d, -h)
        assert abs(np.linalg.norm(ap[r]) - 1.0) < 1e-14
        fd = (_J(ap, w, s, f, kind, eps) - _J(am, w, s, f, kind, eps)) / (2 * h)
        want = -2.0 * np.linalg.norm(d) ** 2
        assert want < 0
        assert abs(fd - want) <= 1e-6 * abs(want), (r, fd, want)


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_coefficient_direction_descends_at_the_predicted_rate(kind):
    # For alpha inside the simplex and small eta, proj(alpha + eta h) = alpha + eta (h - mean h),
    # so dJ/deta = <dL/dalpha, h - mean h> = -||h - mean h||^2 with h = -dL/dalpha.
    atoms, w, s, f, _ = _problem(304, R=4)
    eps, tau = 1e-8, 1e-3
    assert w.min() > 10 * tau
    _, g = loop.objective(atoms, w, s, f, kind, eps, 1e-3)
    hv = loop.coefficient_direction(atoms, w, s, g)
    step = 1e-6
    vals = []
    for eta in (step, -step):
        keep, bc = loop.coefficient_trial(w, hv, eta, tau)
        assert keep.size == w.size
        vals.append(_J(atoms[keep], bc, s, f, kind, eps))
    fd = (vals[0] - vals[1]) / (2 * step)
    want = -np.linalg.norm(hv - hv.mean()) ** 2
    assert want < 0
    assert abs(fd - want) <= 1e-6 * abs(want), (fd, want)


def test_run_takes_the_atom_and_coefficient_steps_of_the_step_functions():
    # One atom slot (t = 1, atom r = 1) after one coefficient slot (t = 0): the state the
    # driver accepts is the step functions' trial at the accepted grid index, and J falls.
    atoms, w, s, f, _ = _problem(305)
    eps, mu, tau = 1e-8, 1e-3, 1e-3
    hist = []
    a2, w2, J2 = loop.run(atoms, w, s, f, kind=born.LOSS_CE, eps=eps, mu=mu, tau=tau, iters=2, t_alpha=2,
                          t_ref=0, history=hist)
    assert [h[1] for h in hist] == [loop.KIND_ALPHA, loop.KIND_PSI]
    assert all(h[4] for h in hist), hist
    J0, g0 = loop.objective(atoms, w, s, f, born.LOSS_CE, eps, mu)
    keep, bc = loop.coefficient_trial(w, loop.coefficient_direction(atoms, w, s, g0), 2.0 ** -hist[0][5], tau)
    a1, w1 = atoms[keep], bc
    J1, g1 = loop.objective(a1, w1, s, f, born.LOSS_CE, eps, mu)
    assert J1 < J0 and abs(J1 - hist[0][2]) < 1e-13 * abs(J1)
    r = 1 % w1.size
    want = a1.copy()
    want[r] = loop.atom_trial(a1[r], loop.atom_direction(a1, w1, s, g1, r), 2.0 ** -hist[1][5])
    assert np.allclose(a2, want, atol=1e-14) and np.allclose(w2, w1, atol=0)
    assert J2 < J1


def test_slot_schedule_written_out():
    # eq. iteration-partition with the reading of Algorithm 1 used here: spectral slots every
    # t_ref (tested first), coefficient slots every t_alpha, atom slots otherwise.
    S, C, A = loop.KIND_RHO, loop.KIND_ALPHA, loop.KIND_PSI
    want_5_10 = [S, A, A, A, A, C, A, A, A, A, S, A, A, A, A, C, A, A, A, A, S, A]
    assert [loop.slot_kind(t, 5, 10) for t in range(22)] == want_5_10
    want_2_3 = [S, A, C, S, C, A, S, A, C, S]
    assert [loop.slot_kind(t, 2, 3) for t in range(10)] == want_2_3
    assert [loop.slot_kind(t, 0, 0) for t in range(4)] == [A, A, A, A]
    assert [loop.slot_kind(t, 3, 0) for t in range(7)] == [C, A, A, C, A, A, C]
    assert [loop.slot_kind(t, 0, 4) for t in range(5)] == [S, A, A, A, S]
    # the three sets partition the slots
    kinds = [loop.slot_kind(t, 5, 10) for t in range(100)]
    assert kinds.count(S) == 10 and kinds.count(C) == 10 and kinds.count(A) == 80
