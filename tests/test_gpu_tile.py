"""GPU parity of the MFMA tile paths (16x16 complex Kronecker tiles of four qubits,
FP16 or BF16 operands, FP32 accumulation) against the FP64 oracle.

Tolerance 1e-2 (norm-wise, and element-wise scaled by the largest reference element)
for probabilities, loss, atom and weight gradients.  The BF16 path splits each
amplitude into two BF16 parts and is checked at 1e-4 as well; the FP16 path scales
each 16x16 block before rounding and is checked at 3e-3.  At the full n=20, R=16
shape every path is compared with the oracle on three sampled settings.

The staged butterfly path with BF16 intermediates (FP32 arithmetic, the setting-batch
amplitudes X and W stored in BF16) is checked at 1e-2, including several batches,
batched small instances and the full n=20, R=16 shape on sampled settings.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import born
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL_TILE = 1e-2
TIGHT = {"PATH_TILE_F16": 3e-3, "PATH_TILE_BF16": 1e-4}


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _run(h, case, path, kind=born.LOSS_CE):
    from paper_2607_19577_amd import api

    inst = to_device(case, DEV)
    probs, _ = api.qst_forward(h, [inst], want_probs=True, path=path)
    lt, ag, wg = api.qst_backward(h, [inst], loss=kind, eps=1e-8, path=path)
    torch.cuda.synchronize()
    return float(lt[0]), probs[0].cpu().numpy(), ag[0].cpu().numpy(), wg[0].cpu().numpy()


@pytest.mark.parametrize("path_name", ["PATH_TILE_F16", "PATH_TILE_BF16"])
@pytest.mark.parametrize("n,R,B", [
    (4, 2, 81),    # below 2^8 amplitudes: per-qubit passes only
    (8, 2, 5),     # two tile groups
    (10, 4, 20),   # two groups and two single qubits
    (13, 3, 6),    # three groups and one single qubit
    (16, 5, 3),    # four groups
])
def test_tile_path_matches_oracle(h, path_name, n, R, B):
    from paper_2607_19577_amd import api

    path = getattr(api, path_name)
    case = make_case(900 + n, n, R, B, shots=5000, exhaustive=(n == 4))
    L, p, ga, gw = _run(h, case, path)
    Lr, pr, gar, gwr = oracle(case, born.LOSS_CE, 1e-8, tier="axis")
    tol = TIGHT[path_name] if n >= 8 else 1e-5
    assert abs(L - Lr) <= tol * abs(Lr), (L, Lr)
    assert close(p, pr, tol), rel(p, pr)
    for r in range(R):
        assert close(ga[r], gar[r], tol), (r, rel(ga[r], gar[r]))
    assert close(gw, gwr, tol), rel(gw, gwr)
    assert tol <= TOL_TILE


@pytest.mark.parametrize("path_name", ["PATH_TILE_F16", "PATH_TILE_BF16"])
def test_tile_path_least_squares(h, path_name):
    from paper_2607_19577_amd import api

    case = make_case(950, 11, 3, 9, shots=5000)
    L, p, ga, gw = _run(h, case, getattr(api, path_name), kind=born.LOSS_LS)
    Lr, pr, gar, gwr = oracle(case, born.LOSS_LS, 1e-8, tier="axis")
    tol = TIGHT[path_name]
    assert abs(L - Lr) <= tol * abs(Lr), (L, Lr)
    for r in range(3):
        assert close(ga[r], gar[r], tol), (r, rel(ga[r], gar[r]))


@pytest.fixture(scope="module")
def n20_sample():
    """n=20, R=16 on three settings with Porter-Thomas frequencies, and the oracle's results."""
    rng = synth.make_rng(960)
    n, R, B = 20, 16, 3
    case = dict(atoms=synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64), weights=synth.dirichlet_weights(rng, R),
                settings=synth.random_settings(rng, B, n))
    case["freqs"] = synth.porter_thomas_freqs(rng, B, 1 << n, synth.dirichlet_weights(rng, 4), 1_000_000)
    return case, oracle(case, born.LOSS_CE, 1e-8, tier="axis")


def _check_n20(h, n20_sample, path, tol, atoms_checked=(0, 5, 15)):
    case, (Lr, pr, gar, gwr) = n20_sample
    L, p, ga, gw = _run(h, case, path)
    assert abs(L - Lr) <= tol * abs(Lr), (L, Lr)
    assert close(p, pr, tol), rel(p, pr)
    for r in atoms_checked:
        assert close(ga[r], gar[r], tol), (r, rel(ga[r], gar[r]))
    assert close(gw, gwr, tol), rel(gw, gwr)


@pytest.mark.parametrize("path_name", ["PATH_TILE_F16", "PATH_TILE_BF16"])
def test_tile_path_full_size_subset(h, n20_sample, path_name):
    """n=20, R=16 on three settings: the tile path against the oracle."""
    from paper_2607_19577_amd import api

    print("tile n=20 subset", path_name, flush=True)
    _check_n20(h, n20_sample, getattr(api, path_name), TIGHT[path_name])


# ---------------------------------------------------------------- FP32 butterflies with BF16 intermediates
TOL_BF16X = 1e-2


@pytest.mark.parametrize("n,R,B,spb", [
    (6, 3, 9, 0),      # whole state in one chunk: W in BF16, settings summed from BF16
    (12, 5, 17, 0),    # tile stages with one high bit
    (15, 16, 11, 4),   # tile stages, several batches
    (17, 3, 9, 2),     # n_lo = 12, five batches
])
def test_bf16_intermediates_match_oracle(h, n, R, B, spb):
    from paper_2607_19577_amd import api

    case = make_case(970 + n, n, R, B, shots=5000)
    inst = to_device(case, DEV)
    inst.settings_per_batch = spb
    probs, _ = api.qst_forward(h, [inst], want_probs=True, path=api.PATH_BUTTERFLY_BF16)
    lt, ag, wg = api.qst_backward(h, [inst], loss=born.LOSS_CE, eps=1e-8, path=api.PATH_BUTTERFLY_BF16)
    torch.cuda.synchronize()
    Lr, pr, gar, gwr = oracle(case, born.LOSS_CE, 1e-8, tier="axis")
    assert abs(float(lt[0]) - Lr) <= TOL_BF16X * abs(Lr)
    assert close(probs[0].cpu().numpy(), pr, TOL_BF16X), rel(probs[0].cpu().numpy(), pr)
    g = ag[0].cpu().numpy()
    for r in range(R):
        assert close(g[r], gar[r], TOL_BF16X), (r, rel(g[r], gar[r]))
    assert close(wg[0].cpu().numpy(), gwr, TOL_BF16X), rel(wg[0].cpu().numpy(), gwr)


def test_bf16_intermediates_batched_instances(h):
    """Several small instances in one call (one launch per step) on the BF16-intermediate path."""
    from paper_2607_19577_amd import api

    cases = [make_case(980 + i, 7, R, B, shots=5000) for i, (R, B) in enumerate([(2, 5), (5, 7), (8, 3)])]
    insts = [to_device(c, DEV) for c in cases]
    lt, ag, wg = api.qst_backward(h, insts, loss=born.LOSS_CE, eps=1e-8, path=api.PATH_BUTTERFLY_BF16)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        Lr, _, gar, gwr = oracle(c, born.LOSS_CE, 1e-8)
        assert abs(float(lt[i]) - Lr) <= TOL_BF16X * abs(Lr)
        g = ag[i].cpu().numpy()
        for r in range(g.shape[0]):
            assert close(g[r], gar[r], TOL_BF16X), (i, r, rel(g[r], gar[r]))


def test_bf16_intermediates_full_size_subset(h, n20_sample):
    """n=20, R=16 on three settings against the oracle."""
    from paper_2607_19577_amd import api

    print("bf16 intermediates n=20 subset", flush=True)
    _check_n20(h, n20_sample, api.PATH_BUTTERFLY_BF16, TOL_BF16X)
