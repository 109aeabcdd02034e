"""Pins of the oracle's general local product measurements (codes >= 3 name the caller's
2x2 unitaries): Pauli matrices put in the table reproduce the Pauli codes, the dense-effect,
dense-unitary and per-axis tiers agree, the effects of every setting resolve the identity,
and both gradients match central finite differences."""
import numpy as np
import pytest

import synth
from oracle import born, pauli


def _general(seed, N, R, B, K=3, shots=2000):
    rng = synth.make_rng(seed)
    table = synth.haar_unitaries_2x2(rng, K)
    s = synth.random_general_settings(rng, B, N, K)
    truth = synth.haar_atoms(rng, 2, 1 << N)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, synth.dirichlet_weights(rng, 2), s, table=table), shots)
    atoms = synth.haar_atoms(rng, R, 1 << N)
    w = synth.dirichlet_weights(rng, R)
    return atoms, w, s, f, table, rng


def test_pauli_matrices_in_the_table_reproduce_pauli_codes():
    rng = synth.make_rng(300)
    N, R, B = 5, 3, 9
    table = np.stack([pauli.single(c) for c in (pauli.X, pauli.Y, pauli.Z)])
    s = synth.random_settings(rng, B, N)
    atoms = synth.haar_atoms(rng, R, 1 << N)
    w = synth.dirichlet_weights(rng, R)
    f = synth.multinomial_freqs(rng, born.probs_axis(atoms, w, s), 1000)
    ref = born.forward_backward(atoms, w, s, f, born.LOSS_CE, 1e-8)
    got = born.forward_backward(atoms, w, (s + 3).astype(np.uint8), f, born.LOSS_CE, 1e-8, table=table)
    assert abs(got[0] - ref[0]) < 1e-13
    for a, b in zip(got[1:], ref[1:]):
        assert np.allclose(a, b, atol=1e-14)


def test_tiers_agree_with_dense_effects():
    atoms, w, s, f, table, _ = _general(301, 3, 2, 12)
    res = {t: born.forward_backward(atoms, w, s, f, born.LOSS_CE, 1e-8, tier=t, table=table)
           for t in ("dense", "kron", "axis")}
    for t in ("kron", "axis"):
        assert abs(res[t][0] - res["dense"][0]) < 1e-13
        for k in (1, 2, 3):
            assert np.allclose(res[t][k], res["dense"][k], atol=1e-13)


def test_effects_resolve_the_identity_and_rows_sum_to_one():
    atoms, w, s, _, table, _ = _general(302, 3, 3, 7)
    E = pauli.povm_elements(s, table)
    B, D = E.shape[0], E.shape[1]
    for b in range(B):
        assert np.allclose(E[b].sum(axis=0), np.eye(D) / B, atol=1e-14)
    p = born.probs_axis(atoms, w, s, table=table)
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_gradients_central_fd(kind):
    atoms, w, s, f, table, rng = _general(303, 4, 3, 8)
    eps = 1e-8

    def loss(a, ww):
        p = born.probs_axis(a, ww, s, table=table)
        return born.loss_and_sensitivity(p, f, s.shape[0], kind, eps)[0]

    _, _, ga, gw = born.forward_backward(atoms, w, s, f, kind, eps, table=table)
    h = 1e-6
    for r in range(atoms.shape[0]):
        d = rng.standard_normal(atoms.shape[1]) + 1j * rng.standard_normal(atoms.shape[1])
        ap, am = atoms.copy(), atoms.copy()
        ap[r] += h * d
        am[r] -= h * d
        fd = (loss(ap, w) - loss(am, w)) / (2 * h)
        an = 2 * np.real(np.vdot(ga[r], d))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-12) + 1e-12, (r, fd, an)
        wp, wm = w.copy(), w.copy()
        wp[r] += h
        wm[r] -= h
        fdw = (loss(atoms, wp) - loss(atoms, wm)) / (2 * h)
        assert abs(fdw - gw[r]) <= 1e-7 * abs(gw[r]) + 1e-12
