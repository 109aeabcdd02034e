"""Pins of the simplex projection and pruning map: KKT conditions, brute-force
support enumeration, idempotence and the strict-threshold rule."""
import itertools

import numpy as np

import synth
from oracle import simplex


def _brute_projection(v):
    # Enumerate every support S; on S the minimiser of ||x - v||^2 subject to sum x = 1 is
    # v_S - (sum v_S - 1)/|S|; keep the feasible (non-negative) candidate of least distance.
    best, arg = np.inf, None
    n = v.size
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            S = list(S)
            x = np.zeros(n)
            x[S] = v[S] - (v[S].sum() - 1.0) / k
            if (x >= -1e-15).all():
                d = np.sum((x - v) ** 2)
                if d < best:
                    best, arg = d, x
    return arg


def test_projection_matches_brute_force_and_kkt():
    rng = synth.make_rng(31)
    for n in range(1, 9):
        for _ in range(25):
            v = rng.standard_normal(n) * rng.choice([0.1, 1.0, 5.0])
            x = simplex.project_simplex(v)
            assert np.allclose(x, _brute_projection(v), atol=1e-12)
            assert abs(x.sum() - 1) < 1e-12 and (x >= 0).all()
            # KKT: x = max(v - theta, 0) for one theta.
            pos = x > 0
            theta = (v[pos] - x[pos]).mean()
            assert np.allclose(x, np.maximum(v - theta, 0), atol=1e-12)


def test_projection_idempotent_on_simplex():
    rng = synth.make_rng(32)
    for n in (1, 3, 10, 64):
        x = rng.dirichlet(np.ones(n))
        assert np.allclose(simplex.project_simplex(x), x, atol=1e-14)


def test_prune_strict_threshold_and_renormalise():
    beta = np.array([0.5, 1e-3, 0.2, 0.299, 0.001])
    keep, bc = simplex.prune(beta, 1e-3)
    assert list(keep) == [0, 2, 3]  # strict '>' drops entries equal to tau
    assert abs(bc.sum() - 1) < 1e-15
    assert np.allclose(bc, beta[[0, 2, 3]] / beta[[0, 2, 3]].sum())
    keep, bc = simplex.prune(np.array([0.2, 0.3, 0.5]), 0.9)
    assert list(keep) == [2] and bc[0] == 1.0


def test_reweight_padding_and_indices():
    alpha = np.array([0.4, 0.3, 0.2, 0.1])
    h = np.array([1.0, 0.0, -2.0, 0.5])
    out, keep, R = simplex.reweight(alpha, h, 0.5, 1e-3)
    beta = simplex.project_simplex(alpha + 0.5 * h)
    assert R == (beta > 1e-3).sum() and list(keep) == list(np.nonzero(beta > 1e-3)[0])
    assert np.allclose(out[:R], beta[keep] / beta[keep].sum()) and not out[R:].any()
