"""GPU parity of sparse (CSR) frequencies through the C ABI: loss, probabilities and both
gradients against the FP64 oracle on the same (dense-expanded) data, on one-chunk states, the
staged path, the plain and tile paths, batched instances and general settings; sparse and
dense storage of the same data give the same results; malformed index data stay inside the
arrays (entries outside a chunk are dropped)."""
import numpy as np
import pytest
import torch

import synth
from oracle import born
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _sparse_inst(case, dev=DEV):
    inst = to_device(case, dev)
    rp, ix, vals = synth.dense_to_csr(case["freqs"])
    inst.freqs = None
    inst.freqs_csr = (torch.from_numpy(rp).to(dev), torch.from_numpy(ix).to(dev), torch.from_numpy(vals).to(dev))
    return inst


def test_csr_round_trip():
    rng = synth.make_rng(1700)
    f = synth.multinomial_freqs(rng, np.full((5, 64), 1 / 64), 20).astype(np.float32)
    rp, ix, vals = synth.dense_to_csr(f)
    back = np.zeros_like(f)
    for b in range(5):
        back[b, ix[rp[b]:rp[b + 1]]] = vals[rp[b]:rp[b + 1]]
    assert np.array_equal(back, f) and (np.diff(ix[rp[0]:rp[1]]) > 0).all()


@pytest.mark.parametrize("n,R,B,shots", [
    (3, 2, 9, 5),      # one chunk, few shots
    (6, 3, 7, 20),
    (12, 4, 6, 40),    # one chunk, 12 low bits
    (15, 3, 5, 200),   # staged
    (17, 5, 3, 500),   # staged, two register layouts in the tile stages
])
@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_sparse_matches_oracle(h, n, R, B, shots, kind):
    from paper_2607_19577_amd import api

    case = make_case(1710 + n, n, R, B, shots=shots)
    assert (case["freqs"] > 0).mean() < 0.5  # sparse data indeed
    inst = _sparse_inst(case)
    lt, ag, wg = api.qst_backward(h, [inst], loss=kind, eps=1e-8)
    _, lf = api.qst_forward(h, [inst], want_probs=False, loss=kind, eps=1e-8)
    torch.cuda.synchronize()
    L, _, ga, gw = oracle(case, kind, 1e-8)
    assert abs(float(lt[0]) - L) <= 1e-5 * abs(L), (float(lt[0]), L)
    assert abs(float(lf[0]) - L) <= 1e-5 * abs(L)
    g = ag[0].cpu().numpy()
    for r in range(R):
        assert close(g[r], ga[r], 1e-5), (r, rel(g[r], ga[r]))
    assert close(wg[0].cpu().numpy(), gw, 1e-5)


@pytest.mark.parametrize("n", [9, 16])
def test_sparse_equals_dense_storage(h, n):
    from paper_2607_19577_amd import api

    case = make_case(1730 + n, n, 3, 5, shots=300)
    dense, sparse = to_device(case, DEV), _sparse_inst(case)
    # the same kernels for both storages: an explicit batch size keeps the dense instance on the
    # staged (or one-chunk fused) path that sparse data takes
    dense.settings_per_batch = sparse.settings_per_batch = 5
    a = api.qst_backward(h, [dense], loss=api.LOSS_CE, eps=1e-8)
    b = api.qst_backward(h, [sparse], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    assert torch.equal(a[1][0], b[1][0])
    assert abs(float(a[0][0]) - float(b[0][0])) <= 1e-12 * abs(float(a[0][0]))
    torch.testing.assert_close(a[2][0], b[2][0], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("path_name", ["PATH_PLAIN_F32", "PATH_TILE_BF16"])
def test_sparse_on_pass_paths(h, path_name):
    from paper_2607_19577_amd import api

    case = make_case(1740, 10, 3, 4, shots=100)
    inst = _sparse_inst(case)
    lt, ag, _ = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=getattr(api, path_name))
    torch.cuda.synchronize()
    L, _, ga, _ = oracle(case, born.LOSS_CE, 1e-8)
    tol = 1e-5 if path_name == "PATH_PLAIN_F32" else 1e-4
    assert abs(float(lt[0]) - L) <= tol * abs(L)
    for r in range(3):
        assert close(ag[0][r].cpu().numpy(), ga[r], tol)


def test_sparse_in_batched_call(h):
    from paper_2607_19577_amd import api

    cases = [make_case(1750 + i, 6, R, B, shots=30) for i, (R, B) in enumerate([(2, 5), (3, 7), (1, 4), (4, 6)])]
    insts = [_sparse_inst(c) if i % 2 == 0 else to_device(c, DEV) for i, c in enumerate(cases)]
    lt, ag, wg = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        L, _, ga, gw = oracle(c, born.LOSS_CE, 1e-8)
        assert abs(float(lt[i]) - L) <= 1e-5 * abs(L), i
        for r in range(ga.shape[0]):
            assert close(ag[i][r].cpu().numpy(), ga[r], 1e-5), (i, r)


def test_sparse_with_general_settings(h):
    from paper_2607_19577_amd import api

    rng = synth.make_rng(1760)
    n, R, B = 14, 3, 5
    table = synth.haar_unitaries_2x2(rng, 2)
    s = synth.random_general_settings(rng, B, n, 2)
    truth = synth.haar_atoms(rng, 1, 1 << n)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, [1.0], s, table=table), 200).astype(np.float32)
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    rp, ix, vals = synth.dense_to_csr(f)
    inst = api.Instance(torch.from_numpy(atoms).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(s).to(DEV),
                        unitaries=torch.from_numpy(table).to(DEV),
                        freqs_csr=(torch.from_numpy(rp).to(DEV), torch.from_numpy(ix).to(DEV),
                                   torch.from_numpy(vals).to(DEV)))
    lt, ag, _ = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    L, _, ga, _ = born.forward_backward(atoms.astype(np.complex128), w, s, f.astype(np.float64), born.LOSS_CE, 1e-8,
                                        table=table)
    assert abs(float(lt[0]) - L) <= 1e-5 * abs(L)
    for r in range(R):
        assert close(ag[0][r].cpu().numpy(), ga[r], 1e-5)


def test_malformed_index_data_stay_in_bounds(h):
    """Unsorted rows and outcomes beyond D: the call completes with finite results (entries that
    fall outside their chunk are dropped; every read stays inside the given arrays)."""
    from paper_2607_19577_amd import api

    case = make_case(1770, 13, 2, 4, shots=100)
    inst = _sparse_inst(case)
    rp, ix, vals = inst.freqs_csr
    ix = ix.flip(0).contiguous()
    ix[::7] = 1 << 20  # beyond D
    inst.freqs_csr = (rp, ix, vals)
    lt, ag, _ = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    assert torch.isfinite(lt).all() and torch.isfinite(torch.view_as_real(ag[0])).all()
