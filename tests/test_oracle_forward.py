"""Pins of the oracle's forward map (Born probabilities) against closed forms,
invariants, hand-derived fixtures and brute force -- never against itself."""
import os

import numpy as np
import pytest

import synth
from oracle import born, pauli

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CODE = {"X": 0, "Y": 1, "Z": 2}


def _kron_states(*vs):
    out = np.ones(1, dtype=np.complex128)
    for v in vs:
        out = np.kron(out, np.asarray(v, dtype=np.complex128))
    return out


def test_single_qubit_rotations_diagonalise_paulis():
    # V^dagger diag(1,-1) V must be the Pauli observable itself: this fixes both the
    # matrices and the outcome labelling (bit 0 <-> +1 eigenvector).
    for c in (pauli.X, pauli.Y, pauli.Z):
        V = pauli.single(c)
        assert np.allclose(V @ V.conj().T, np.eye(2), atol=1e-15)
        assert np.allclose(V.conj().T @ np.diag([1.0, -1.0]) @ V, pauli.SIGMA[c], atol=1e-15)


def test_golden_single_qubit_bloch():
    rows = np.loadtxt(os.path.join(GOLD, "single_qubit_bloch.txt"))
    for th, ph, px, py, pz in rows:
        psi = np.array([[np.cos(th / 2), np.exp(1j * ph) * np.sin(th / 2)]])
        for code, want in ((0, px), (1, py), (2, pz)):
            s = np.array([[code]], dtype=np.uint8)
            for tier in (born.probs_dense, born.probs_kron, born.probs_axis):
                p = tier(psi, [1.0], s)
                assert abs(p[0, 0] - want) < 1e-14 and abs(p[0, 1] - (1 - want)) < 1e-14


def test_golden_bell_ghz_product():
    s2 = 1 / np.sqrt(2)
    states = {
        "bell": np.array([s2, 0, 0, s2], dtype=np.complex128),
        "ghz3": np.array([s2, 0, 0, 0, 0, 0, 0, s2], dtype=np.complex128),
        "prod": _kron_states([1, 0], [s2, s2], [s2, 1j * s2]),
    }
    with open(os.path.join(GOLD, "bell_ghz.txt")) as fh:
        lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(lines) >= 9
    for ln in lines:
        psi = states[ln[1]][None, :]
        s = np.array([[CODE[ch] for ch in ln[2]]], dtype=np.uint8)
        want = np.array([float(x) for x in ln[3:]])
        for tier in (born.probs_dense, born.probs_kron, born.probs_axis):
            assert np.allclose(tier(psi, [1.0], s)[0], want, atol=1e-14), (ln, tier)


def test_ghz_closed_forms_large_n():
    # GHZ_N under all-X: uniform 2^(1-N) on even parity; under all-Z: 1/2 on 0^N and 1^N.
    for N in (5, 8, 11):
        D = 1 << N
        psi = np.zeros(D, dtype=np.complex128)
        psi[0] = psi[-1] = 1 / np.sqrt(2)
        px = born.probs_axis(psi[None], [1.0], np.zeros((1, N), dtype=np.uint8))[0]
        par = np.array([bin(u).count("1") % 2 for u in range(D)])
        assert np.allclose(px, np.where(par == 0, 2.0 ** (1 - N), 0.0), atol=1e-14)
        pz = born.probs_axis(psi[None], [1.0], np.full((1, N), 2, dtype=np.uint8))[0]
        want = np.zeros(D)
        want[0] = want[-1] = 0.5
        assert np.allclose(pz, want, atol=1e-14)


def test_plus_i_under_all_y_and_bit_order():
    # |+i>^N under all-Y gives u = 0 with probability 1 (fixes V_Y's outcome-0 row).
    N = 6
    plus_i = np.array([1, 1j]) / np.sqrt(2)
    psi = _kron_states(*([plus_i] * N))
    p = born.probs_axis(psi[None], [1.0], np.ones((1, N), dtype=np.uint8))[0]
    assert abs(p[0] - 1) < 1e-14
    # Product of distinct single-qubit states under all-Z factorises with qubit 0 = MSB.
    rng = synth.make_rng(3)
    singles = [rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(N)]
    singles = [v / np.linalg.norm(v) for v in singles]
    psi = _kron_states(*singles)
    p = born.probs_axis(psi[None], [1.0], np.full((1, N), 2, dtype=np.uint8))[0]
    for u in range(1 << N):
        bits = [(u >> (N - 1 - j)) & 1 for j in range(N)]
        want = np.prod([abs(singles[j][bits[j]]) ** 2 for j in range(N)])
        assert abs(p[u] - want) < 1e-14


def test_eigenstate_gives_certain_outcome():
    rng = synth.make_rng(7)
    N = 7
    s = synth.random_settings(rng, 4, N)
    for b in range(4):
        u = int(rng.integers(0, 1 << N))
        e = np.zeros(1 << N, dtype=np.complex128)
        e[u] = 1
        psi = pauli.apply_setting_axis(s[b], e, adjoint=True)  # V_b^dagger e_u
        p = born.probs_axis(psi[None], [1.0], s[b:b + 1])[0]
        assert abs(p[u] - 1) < 1e-13


def test_invariants_and_tiers_agree():
    rng = synth.make_rng(11)
    for N, R in ((2, 2), (3, 3), (4, 2)):
        D = 1 << N
        atoms = synth.haar_atoms(rng, R, D)
        w = synth.dirichlet_weights(rng, R)
        s = synth.all_settings(N)
        pd = born.probs_dense(atoms, w, s)
        pk = born.probs_kron(atoms, w, s)
        pa = born.probs_axis(atoms, w, s)
        assert np.allclose(pd, pk, atol=1e-13) and np.allclose(pd, pa, atol=1e-13)
        assert (pd > -1e-15).all()
        assert np.allclose(pd.sum(axis=1), 1.0, atol=1e-13)
        # The combined POVM sums to the identity.
        E = pauli.povm_elements(s)
        assert np.allclose(E.sum(axis=(0, 1)), np.eye(D), atol=1e-13)
        # rho is PSD with unit trace and rank <= R.
        rho = born.density(atoms, w)
        ev = np.linalg.eigvalsh(rho)
        assert ev.min() > -1e-14 and abs(np.trace(rho) - 1) < 1e-14
        assert (ev > 1e-12).sum() <= R
        # Linearity pi = A alpha (stacked, p = B pi).
        A = born.atom_response_dense(atoms, s)
        assert np.allclose(A @ w * s.shape[0], pd.reshape(-1), atol=1e-13)
        # Every atom response lies on the simplex.
        assert np.allclose(A.sum(axis=0), 1.0, atol=1e-13)


def test_tiers_agree_n10_and_phase_invariance():
    rng = synth.make_rng(12)
    N, R, B = 9, 3, 6
    atoms = synth.haar_atoms(rng, R, 1 << N)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, N)
    pk = born.probs_kron(atoms, w, s)
    pa = born.probs_axis(atoms, w, s)
    assert np.allclose(pk, pa, atol=1e-13)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(R, 1)))
    assert np.allclose(born.probs_axis(atoms * ph, w, s), pa, atol=1e-13)


def test_brute_force_trace_formula():
    # Brute force with no Kronecker machinery: build V_b entry by entry from the
    # per-qubit matrices, p = sum_r alpha_r |sum_v V[u,v] psi_r[v]|^2.
    rng = synth.make_rng(13)
    N, R = 3, 2
    D = 1 << N
    atoms = synth.haar_atoms(rng, R, D)
    w = synth.dirichlet_weights(rng, R)
    s = synth.all_settings(N)
    ref = np.zeros((s.shape[0], D))
    for b in range(s.shape[0]):
        V = np.ones((D, D), dtype=np.complex128)
        for u in range(D):
            for v in range(D):
                for j in range(N):
                    bu, bv = (u >> (N - 1 - j)) & 1, (v >> (N - 1 - j)) & 1
                    V[u, v] *= pauli.single(s[b, j])[bu, bv]
        for r in range(R):
            ref[b] += w[r] * np.abs(V @ atoms[r]) ** 2
    assert np.allclose(born.probs_dense(atoms, w, s), ref, atol=1e-14)
    assert np.allclose(born.probs_axis(atoms, w, s), ref, atol=1e-14)


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_loss_values_by_hand(kind):
    # Two settings, two outcomes each: evaluate the stacked-vector losses by hand.
    p = np.array([[0.25, 0.75], [0.6, 0.4]])
    f = np.array([[0.5, 0.5], [1.0, 0.0]])
    B, eps = 2, 1e-3
    L, g = born.loss_and_sensitivity(p, f, B, kind, eps)
    if kind == born.LOSS_CE:
        want = -(0.25 * np.log(0.125 + eps) + 0.25 * np.log(0.375 + eps) + 0.5 * np.log(0.3 + eps))
        assert abs(L - want) < 1e-15
        assert abs(g[1, 1]) == 0.0  # pihat = 0 outcome
        assert abs(g[0, 0] - (-(0.25 / (0.125 + eps)) / 2)) < 1e-15
    else:
        r = (p - f) / B
        assert abs(L - 0.5 * np.sum(r * r)) < 1e-15
        assert np.allclose(g, r / B)
