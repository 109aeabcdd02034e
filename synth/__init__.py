"""Seeded synthetic inputs for the atomic-tomography hot path.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic (no basis rotation, no Born probabilities, no loss).
Both the FP64 oracle tests and the GPU tests / benchmark take their inputs
from here, so the two sides see bit-identical data.

Recipes follow the paper's numerical-test section (ground truth, Pauli
design and data generation):

* atoms ``psi = xi / ||xi||`` with ``xi ~ CN(0, I_D)`` (real and imaginary
  parts i.i.d. ``N(0, 1/2)``);
* weights ``alpha ~ Dirichlet(1)``, sorted non-increasing;
* Pauli strings drawn i.i.d. uniform over ``{X, Y, Z}`` per qubit, encoded
  as ``uint8`` codes X=0, Y=1, Z=2;
* frequencies ``f_{b,u} = N_{b,u} / N_s`` from ``N_s`` multinomial shots of a
  given per-setting distribution (the distribution itself is computed by the
  caller, e.g. by the oracle).

For workloads too large to push through the oracle (n = 20) the
frequencies come from a Porter-Thomas stand-in: each setting's outcome
distribution is a Dirichlet-weighted mixture of i.i.d. exponential
profiles -- the law of ``|<u|V psi>|^2`` for Haar-random atoms -- followed by
Poisson shot noise.  The stand-in is drawn here, never from the GPU path.
"""
from __future__ import annotations

import itertools

import numpy as np

PAULI_X, PAULI_Y, PAULI_Z = 0, 1, 2


def make_rng(seed: int) -> np.random.Generator:
    """PCG64 generator from a SeedSequence of ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))


def haar_atoms(rng: np.random.Generator, R: int, D: int, dtype=np.complex128) -> np.ndarray:
    """``[R][D]`` unit-norm atoms, ``xi ~ CN(0, I)`` normalised (ground-truth recipe)."""
    re = rng.standard_normal((R, D))
    im = rng.standard_normal((R, D))
    xi = (re + 1j * im) * np.sqrt(0.5)
    nrm = np.sqrt(np.sum(np.abs(xi) ** 2, axis=1, keepdims=True))
    return (xi / nrm).astype(dtype)


def dirichlet_weights(rng: np.random.Generator, R: int, sort: bool = True) -> np.ndarray:
    """``[R]`` float64 weights on the simplex, ``Dirichlet(1)``, non-increasing if ``sort``."""
    w = rng.dirichlet(np.ones(R))
    if sort:
        w = np.sort(w)[::-1].copy()
    return w.astype(np.float64)


def random_settings(rng: np.random.Generator, B: int, N: int) -> np.ndarray:
    """``[B][N]`` uint8 Pauli codes, i.i.d. uniform over X/Y/Z, duplicates allowed."""
    return rng.integers(0, 3, size=(B, N), dtype=np.uint8)


def all_settings(N: int) -> np.ndarray:
    """All ``3^N`` Pauli strings, setting ``b = sum_j code_j 3^(N-1-j)`` (qubit 0 most significant)."""
    rows = list(itertools.product(range(3), repeat=N))
    return np.asarray(rows, dtype=np.uint8).reshape(len(rows), N)


def multinomial_freqs(rng: np.random.Generator, probs: np.ndarray, shots: int) -> np.ndarray:
    """``[B][D]`` float32 frequencies ``N_{b,u}/N_s`` from ``shots`` draws of each row of ``probs``."""
    probs = np.asarray(probs, dtype=np.float64)
    out = np.empty(probs.shape, dtype=np.float32)
    for b in range(probs.shape[0]):
        q = np.clip(probs[b], 0.0, None)
        q = q / q.sum()
        out[b] = (rng.multinomial(int(shots), q) / float(shots)).astype(np.float32)
    return out


def porter_thomas_freqs(rng: np.random.Generator, B: int, D: int, weights: np.ndarray,
                        shots: int) -> np.ndarray:
    """Stand-in frequencies ``[B][D]`` float32 for large ``D`` (numpy; moderate sizes only).

    Per setting: ``q = sum_r w_r e_r / D`` with ``e_r ~ Exp(1)`` i.i.d. per outcome,
    then ``N_u ~ Poisson(shots * q_u)`` and ``f = N / shots``.
    """
    out = np.empty((B, D), dtype=np.float32)
    w = np.asarray(weights, dtype=np.float64)
    for b in range(B):
        q = np.zeros(D)
        for r in range(w.shape[0]):
            q += w[r] * rng.exponential(1.0, size=D)
        q /= q.sum()
        out[b] = (rng.poisson(shots * q) / float(shots)).astype(np.float32)
    return out


def porter_thomas_freqs_torch(seed: int, B: int, D: int, weights, shots: int, device):
    """Same stand-in as :func:`porter_thomas_freqs`, drawn with torch's seeded generator on
    ``device`` (used where ``B*D`` is in the billions).  Returns a ``[B][D]`` float32 tensor."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    w = torch.as_tensor(np.asarray(weights, dtype=np.float32), device=device)
    out = torch.empty((B, D), dtype=torch.float32, device=device)
    rows = max(1, (1 << 26) // D)
    for b0 in range(0, B, rows):
        b1 = min(B, b0 + rows)
        q = torch.zeros((b1 - b0, D), dtype=torch.float32, device=device)
        for r in range(w.shape[0]):
            e = torch.empty((b1 - b0, D), dtype=torch.float32, device=device).exponential_(1.0, generator=gen)
            q.add_(e, alpha=float(w[r]))
        q.div_(q.sum(dim=1, keepdim=True))
        cnt = torch.poisson(q * float(shots), generator=gen)
        out[b0:b1] = cnt / float(shots)
    return out


def haar_unitaries_2x2(rng: np.random.Generator, K: int) -> np.ndarray:
    """K Haar-random 2x2 unitaries ``[K][2][2]`` complex128 (QR of a complex Gaussian with the
    phases of R's diagonal moved into Q): single-qubit readout rotations of general local
    settings."""
    z = rng.standard_normal((K, 2, 2)) + 1j * rng.standard_normal((K, 2, 2))
    out = np.empty_like(z)
    for k in range(K):
        q, r = np.linalg.qr(z[k])
        out[k] = q * (np.diag(r) / np.abs(np.diag(r)))
    return out


def random_general_settings(rng: np.random.Generator, B: int, N: int, K: int) -> np.ndarray:
    """Settings ``[B][N]`` uint8 with codes uniform over the three Pauli bases and ``K`` table
    entries (codes ``3 .. 3+K-1``)."""
    return rng.integers(0, 3 + K, size=(B, N)).astype(np.uint8)


def dense_to_csr(f: np.ndarray):
    """``(rowptr int64 [B+1], index int32 [nnz], values float32 [nnz])`` of the non-zero entries of a
    ``[B][D]`` frequency array, outcomes ascending within each row."""
    f = np.asarray(f, dtype=np.float32)
    rows, cols = np.nonzero(f)
    rowptr = np.zeros(f.shape[0] + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr).astype(np.int64), cols.astype(np.int32), f[rows, cols].astype(np.float32)


def poisson_freqs_torch(seed: int, probs, shots: int):
    """Frequencies ``Poisson(shots * p) / shots`` of given per-setting probabilities ``probs``
    (a device tensor ``[B][D]``), drawn with torch's seeded generator on the same device: the
    large-count stand-in for multinomial sampling where ``B*D`` is large."""
    import torch

    gen = torch.Generator(device=probs.device)
    gen.manual_seed(int(seed))
    return (torch.poisson(probs.float().clamp_min(0.0) * float(shots), generator=gen) / float(shots)).float()


# Workload shapes (number of qubits, atoms, settings, shots) used by tests and the benchmark.
WORKLOADS = {
    "n4_r2_all81": dict(n=4, R=2, B=81, shots=1000, R_true=2, exhaustive=True),
    "n10_r4_b200": dict(n=10, R=4, B=200, shots=10_000, R_true=4),
    "n14_r8_b1000": dict(n=14, R=8, B=1000, shots=100_000, R_true=4),
    "n20_r16_b2000": dict(n=20, R=16, B=2000, shots=1_000_000, R_true=4),
}


def uneven_batch_shapes(rng: np.random.Generator, count: int = 64):
    """Shapes of ``count`` independent instances: n ~ U{6..12}, R ~ U{1..8}, B ~ U{50..500}."""
    n = rng.integers(6, 13, size=count)
    R = rng.integers(1, 9, size=count)
    B = rng.integers(50, 501, size=count)
    return [dict(n=int(a), R=int(b), B=int(c)) for a, b, c in zip(n, R, B)]
