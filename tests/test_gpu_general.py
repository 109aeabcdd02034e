"""GPU parity of general local product measurements (settings codes >= 3 name the caller's
2x2 unitaries) through the C ABI, against the FP64 oracle's per-axis tier with the same
table: probabilities, loss (CE and LS), atom and weight gradients at 1e-5, from one-chunk
states to the staged path and a sampled subset at n=20.  Plus: Pauli matrices in the table
give the Pauli path's results, and codes beyond the table raise the device flag."""
import numpy as np
import pytest
import torch

import synth
from oracle import born, pauli
from tests._cases import close, rel

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _case(seed, n, R, B, K=3, shots=5000):
    rng = synth.make_rng(seed)
    table = synth.haar_unitaries_2x2(rng, K)
    s = synth.random_general_settings(rng, B, n, K)
    truth = synth.haar_atoms(rng, 2, 1 << n)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, synth.dirichlet_weights(rng, 2), s, table=table), shots)
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    return dict(atoms=atoms, weights=w, settings=s, freqs=f.astype(np.float32), table=table)


def _inst(c):
    from paper_2607_19577_amd import api

    return api.Instance(torch.from_numpy(c["atoms"]).to(DEV), torch.from_numpy(c["weights"]).to(DEV),
                        torch.from_numpy(c["settings"]).to(DEV), torch.from_numpy(c["freqs"]).to(DEV),
                        unitaries=torch.from_numpy(c["table"]).to(DEV))


@pytest.mark.parametrize("n,R,B", [
    (1, 2, 5),     # one qubit
    (3, 2, 9),     # one chunk
    (7, 3, 11),
    (12, 4, 6),    # one chunk, 12 low bits
    (15, 3, 5),    # staged: 12 low, 3 high bits
    (17, 5, 3),    # staged: 11 low, 6 high bits (two register layouts in the tile stages)
])
@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_general_settings_match_oracle(h, n, R, B, kind):
    from paper_2607_19577_amd import api

    c = _case(1600 + n, n, R, B)
    inst = _inst(c)
    probs, _ = api.qst_forward(h, [inst], want_probs=True)
    lt, ag, wg = api.qst_backward(h, [inst], loss=kind, eps=1e-8)
    torch.cuda.synchronize()
    L, p, ga, gw = born.forward_backward(c["atoms"].astype(np.complex128), c["weights"], c["settings"],
                                         c["freqs"].astype(np.float64), kind, 1e-8, table=c["table"])
    assert close(probs[0].cpu().numpy(), p, 1e-5), rel(probs[0].cpu().numpy(), p)
    assert abs(float(lt[0]) - L) <= 1e-5 * abs(L), (float(lt[0]), L)
    g = ag[0].cpu().numpy()
    for r in range(R):
        assert close(g[r], ga[r], 1e-5), (r, rel(g[r], ga[r]))
    assert close(wg[0].cpu().numpy(), gw, 1e-5), rel(wg[0].cpu().numpy(), gw)


def test_pauli_table_equals_pauli_codes(h):
    from paper_2607_19577_amd import api

    rng = synth.make_rng(1650)
    n, R, B = 14, 4, 7
    s = synth.random_settings(rng, B, n)
    atoms = torch.from_numpy(synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)).to(DEV)
    w = torch.from_numpy(synth.dirichlet_weights(rng, R)).to(DEV)
    f = torch.from_numpy(synth.porter_thomas_freqs(rng, B, 1 << n, synth.dirichlet_weights(rng, 2), 10_000)
                         .astype(np.float32)).to(DEV)
    table = torch.from_numpy(np.stack([pauli.single(k) for k in (pauli.X, pauli.Y, pauli.Z)])).to(DEV)
    pa = api.Instance(atoms, w, torch.from_numpy(s).to(DEV), f)
    ge = api.Instance(atoms, w, torch.from_numpy((s + 3).astype(np.uint8)).to(DEV), f, unitaries=table)
    ref = api.qst_backward(h, [pa], loss=api.LOSS_CE, eps=1e-8)
    got = api.qst_backward(h, [ge], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    assert abs(float(got[0][0]) - float(ref[0][0])) <= 1e-5 * abs(float(ref[0][0]))
    assert close(got[1][0].cpu().numpy(), ref[1][0].cpu().numpy(), 1e-5)
    assert close(got[2][0].cpu().numpy(), ref[2][0].cpu().numpy(), 1e-5)


def test_general_full_size_subset(h):
    """n = 20, R = 4 (staged: 12 low, 8 high bits) on four settings against the oracle."""
    from paper_2607_19577_amd import api

    c = _case(1660, 20, 4, 4, shots=100_000)
    inst = _inst(c)
    probs, _ = api.qst_forward(h, [inst], want_probs=True)
    lt, ag, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    L, p, ga, gw = born.forward_backward(c["atoms"].astype(np.complex128), c["weights"], c["settings"],
                                         c["freqs"].astype(np.float64), born.LOSS_CE, 1e-8, table=c["table"])
    assert close(probs[0].cpu().numpy(), p, 1e-5), rel(probs[0].cpu().numpy(), p)
    assert abs(float(lt[0]) - L) <= 1e-5 * abs(L)
    g = ag[0].cpu().numpy()
    for r in range(4):
        assert close(g[r], ga[r], 1e-5), (r, rel(g[r], ga[r]))
    assert close(wg[0].cpu().numpy(), gw, 1e-5)


def test_code_beyond_the_table_raises_the_flag(h):
    from paper_2607_19577_amd import api

    c = _case(1670, 6, 2, 4, K=2)
    c["settings"][1, 3] = 3 + 2  # one past the table
    api.qst_forward(h, [_inst(c)], want_probs=True)
    torch.cuda.synchronize()
    with pytest.raises(api.QSTError, match="NUMERIC"):
        api.qst_forward(h, [_inst(c)], want_probs=True)
    torch.cuda.synchronize()
    api.qst_forward(h, [_inst(_case(1671, 6, 2, 4))], want_probs=True)  # the flag was cleared


def test_non_unitary_table_entry_raises_the_flag(h):
    """The kernels apply each table entry in rotation form, which needs a unitary: an entry off
    unitarity by more than 1e-6 is flagged (and acts as the identity); the flag is then cleared."""
    from paper_2607_19577_amd import api

    c = _case(1672, 6, 2, 4, K=2)
    c["settings"][2, 1] = 3 + 1
    bad = c["table"].copy()
    bad[1] *= 1.001  # columns no longer of unit norm
    inst = api.Instance(torch.from_numpy(c["atoms"]).to(DEV), torch.from_numpy(c["weights"]).to(DEV),
                        torch.from_numpy(c["settings"]).to(DEV), torch.from_numpy(c["freqs"]).to(DEV),
                        unitaries=torch.from_numpy(bad).to(DEV))
    api.qst_forward(h, [inst], want_probs=True)
    torch.cuda.synchronize()
    with pytest.raises(api.QSTError, match="not unitary"):
        api.qst_forward(h, [_inst(c)], want_probs=True)
    torch.cuda.synchronize()
    api.qst_forward(h, [_inst(c)], want_probs=True)  # the flag was cleared


def test_autograd_with_general_settings_and_sparse_data(h):
    """torch.autograd through the general-settings forward (caller's dL/dp) and the fused loss on
    sparse frequencies, against the oracle's gradients (torch's complex gradient is twice the
    conjugate-Wirtinger one)."""
    from paper_2607_19577_amd.autograd import born_map, fused_loss

    c = _case(1680, 8, 3, 6, shots=60)
    a = torch.from_numpy(c["atoms"]).to(DEV).requires_grad_(True)
    w = torch.from_numpy(c["weights"]).to(DEV).requires_grad_(True)
    s = torch.from_numpy(c["settings"]).to(DEV)
    table = torch.from_numpy(c["table"]).to(DEV)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(3)
    cw = torch.randn((6, 256), generator=gen, device=DEV)
    (born_map(a, w, s, h, unitaries=table) * cw).sum().backward()
    torch.cuda.synchronize()
    gar, gwr = born.gradients_axis(c["atoms"].astype(np.complex128), c["weights"], c["settings"],
                                   cw.cpu().numpy().astype(np.float64), table=c["table"])
    ga = a.grad.cpu().numpy() / 2
    for r in range(3):
        assert close(ga[r], gar[r], 1e-5), (r, rel(ga[r], gar[r]))
    assert close(w.grad.cpu().numpy(), gwr, 1e-5)
    a.grad = None
    w.grad = None
    rp, ix, vals = synth.dense_to_csr(c["freqs"])
    csr = (torch.from_numpy(rp).to(DEV), torch.from_numpy(ix).to(DEV), torch.from_numpy(vals).to(DEV))
    L = fused_loss(a, w, s, csr, h, unitaries=table)
    L.backward()
    torch.cuda.synchronize()
    Lr, _, gar, gwr = born.forward_backward(c["atoms"].astype(np.complex128), c["weights"], c["settings"],
                                            c["freqs"].astype(np.float64), born.LOSS_CE, 1e-8, table=c["table"])
    assert abs(float(L.detach()) - Lr) <= 1e-5 * abs(Lr)
    ga = a.grad.cpu().numpy() / 2
    for r in range(3):
        assert close(ga[r], gar[r], 1e-5), (r, rel(ga[r], gar[r]))
    assert close(w.grad.cpu().numpy(), gwr, 1e-5)


def test_atom_trial_and_solve_with_general_settings(h):
    """The atom-step update and the iteration carry the unitary table through every call."""
    from paper_2607_19577_amd import api

    c = _case(1690, 9, 3, 8, shots=3000)
    inst = _inst(c)
    p_t = born.probs_axis(c["atoms"].astype(np.complex128), c["weights"], c["settings"], table=c["table"])
    trial = synth.haar_atoms(synth.make_rng(1691), 1, 512, dtype=np.complex64)[0]
    probs, lt = api.qst_atom_trial(h, inst, 1, torch.from_numpy(trial).to(DEV),
                                   torch.from_numpy(p_t.astype(np.float32)).to(DEV), loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    pr = born.atom_trial_probs(c["atoms"].astype(np.complex128), c["weights"], c["settings"], 1,
                               trial.astype(np.complex128), p_t.astype(np.float32).astype(np.float64),
                               table=c["table"])
    assert close(probs.cpu().numpy(), pr, 1e-5), rel(probs.cpu().numpy(), pr)
    v0s = torch.from_numpy(synth.haar_atoms(synth.make_rng(1692), 2, 512, dtype=np.complex128)).to(DEV)
    prm = api.SolveParams(max_slots=25, t_alpha=5, t_ref=10, rank_max=4, n_lanczos=12, stop_window=0,
                          oracle_budget=0)
    res = api.qst_solve(h, inst, prm, v0s)
    hist = res["history"]
    assert hist[:, 4].sum() >= 3
    a = res["atoms"].cpu().numpy().astype(np.complex128)
    wv = res["weights"].cpu().numpy()
    p = born.probs_axis(a, wv, c["settings"], table=c["table"])
    L, _ = born.loss_and_sensitivity(p, c["freqs"].astype(np.float64), 8, born.LOSS_CE, 1e-8)
    assert abs(L + prm.mu * res["rank"] - hist[-1, 2]) <= 1e-5 * abs(hist[-1, 2])
