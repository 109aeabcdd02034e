"""Pauli-string measurement descriptors (numerical-test section, Pauli design).

A setting is a string ``s_b in {X, Y, Z}^N``; its product basis rotation is
``V_b = V_{s_b,1} (x) ... (x) V_{s_b,N}``, where each single-qubit ``V`` maps
the Pauli eigenbasis to the computational basis.  The paper does not print
the three matrices; the readings used here (and recorded as such) are

* ``V_Z = I``;
* ``V_X = H = (1/sqrt2) [[1, 1], [1, -1]]``  (rows are <+| and <-|);
* ``V_Y = H S^dagger = (1/sqrt2) [[1, -i], [1, i]]``  (rows are <+i| and <-i|);

so outcome bit 0 is the +1 eigenvector.  Qubit ``j`` (0-based; qubit 0 is the
leftmost Kronecker factor) is bit ``N-1-j`` of both the amplitude index and
the outcome index -- i.e. axis ``j`` of a C-ordered ``(2,)*N`` reshape.

General local product measurements (the measurement-action section allows any
local or tensor-product POVM given by its descriptors): a code ``c >= 3`` names
the caller's unitary ``table[c - 3]`` (a 2x2 complex matrix applied before the
computational-basis readout), so a setting is still one code per qubit.
"""
from __future__ import annotations

import numpy as np

X, Y, Z = 0, 1, 2

_S2 = 1.0 / np.sqrt(2.0)
V_SINGLE = {
    X: np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) * _S2,
    Y: np.array([[1.0, -1.0j], [1.0, 1.0j]], dtype=np.complex128) * _S2,
    Z: np.eye(2, dtype=np.complex128),
}

# The Pauli observables themselves (used by pins: V^dagger diag(1,-1) V = sigma).
SIGMA = {
    X: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    Y: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    Z: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def single(code: int, table=None) -> np.ndarray:
    """2x2 rotation for one code: X=0, Y=1, Z=2, or ``table[code - 3]`` for ``code >= 3``."""
    code = int(code)
    if code <= Z:
        return V_SINGLE[code]
    return np.asarray(table, dtype=np.complex128)[code - 3]


def setting_unitary(codes, table=None) -> np.ndarray:
    """Dense ``V_b = kron(V_{s_0}, ..., V_{s_{N-1}})`` (D x D); qubit 0 is the leftmost factor."""
    V = np.ones((1, 1), dtype=np.complex128)
    for c in codes:
        V = np.kron(V, single(c, table))
    return V


def apply_setting_axis(codes, vec: np.ndarray, adjoint: bool = False, table=None) -> np.ndarray:
    """``V_b vec`` (or ``V_b^dagger vec``) by contracting each 2x2 along its own axis.

    ``vec`` has length ``2^N``; it is viewed as a ``(2,)*N`` tensor whose axis ``j``
    is qubit ``j``.
    """
    N = len(codes)
    t = np.asarray(vec, dtype=np.complex128).reshape((2,) * N)
    for j, c in enumerate(codes):
        if int(c) == Z:
            continue
        U = single(c, table)
        if adjoint:
            U = U.conj().T
        t = np.moveaxis(np.tensordot(U, t, axes=([1], [j])), 0, j)
    return t.reshape(-1)


def povm_elements(settings, table=None) -> np.ndarray:
    """All effects ``E_{b,u} = (1/B) V_b^dagger |u><u| V_b`` as a ``[B][D][D][D]`` array.

    Only for tiny ``N`` (dense tier).
    """
    settings = np.asarray(settings)
    B, N = settings.shape
    D = 1 << N
    E = np.zeros((B, D, D, D), dtype=np.complex128)
    for b in range(B):
        V = setting_unitary(settings[b], table)
        for u in range(D):
            w = V[u, :].conj()  # V_b^dagger e_u
            E[b, u] = np.outer(w, w.conj()) / B
    return E
