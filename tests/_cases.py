"""Shared helpers for the GPU parity tests: seeded instances (same bits on both
sides) and norm-wise error measures."""
from __future__ import annotations

import numpy as np

import synth
from oracle import born


def rel(a, b) -> float:
    """Norm-wise relative error ||a - b|| / ||b||."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def close(a, b, tol) -> bool:
    """Norm-wise relative error <= tol, and every element within tol * max|b| (element-wise check
    that stays meaningful for the near-zero outcomes of Porter-Thomas distributed probabilities)."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return rel(a, b) <= tol and bool(np.all(np.abs(a - b) <= tol * scale))


def make_case(seed: int, n: int, R: int, B: int, shots: int = 10_000, complex_dtype=np.complex64,
              exhaustive: bool = False, R_true: int = 2, freqs: bool = True):
    """Model atoms/weights, settings and multinomial frequencies of a random truth.

    Returns numpy arrays (atoms in ``complex_dtype``; the oracle upcasts the same values)."""
    rng = synth.make_rng(seed)
    D = 1 << n
    s = synth.all_settings(n) if exhaustive else synth.random_settings(rng, B, n)
    f = None
    if freqs:
        truth = synth.haar_atoms(rng, R_true, D)
        wt = synth.dirichlet_weights(rng, R_true)
        f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), shots)
    atoms = synth.haar_atoms(rng, R, D, dtype=complex_dtype)
    w = synth.dirichlet_weights(rng, R)
    return dict(atoms=atoms, weights=w, settings=s, freqs=f)


def to_device(case, dev):
    import torch

    from paper_2607_19577_amd import api

    return api.Instance(torch.from_numpy(case["atoms"]).to(dev), torch.from_numpy(case["weights"]).to(dev),
                        torch.from_numpy(case["settings"]).to(dev),
                        None if case["freqs"] is None else torch.from_numpy(case["freqs"]).to(dev))


def oracle(case, kind=born.LOSS_CE, eps=1e-8, tier="axis", grad_p=None, rows=None):
    atoms = case["atoms"].astype(np.complex128)
    s = case["settings"] if rows is None else case["settings"][rows]
    f = None if case["freqs"] is None else case["freqs"].astype(np.float64)
    if f is not None and rows is not None:
        f = f[rows]
    return born.forward_backward(atoms, case["weights"], s, f, kind, eps, tier=tier, grad_p=grad_p)
