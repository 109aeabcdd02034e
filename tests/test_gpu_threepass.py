"""GPU parity of the schedules for more than ten bits above the low stage, and of ranks above 16.

When the index bits above the low stage are more than one tile of 2^14 amplitudes holds with at
most 2^10 rows (n = 21 at R = 16, or n = 20 at R = 17..32, whose low stage takes nine bits), the
staged path either gives the low stage n - 10 bits with its atoms looped in one work-group (two
sweeps over X; Pauli settings and dense data) or adds a middle tile pass in place on the
setting-batch intermediates X and W (general settings, sparse data).  Ranks above 16 also reach
the low stage with six to eight low bits, the on-chip passes (n = 11..14) and the fused slices
(R 2^n <= 2^14).  Every case is compared with the FP64 oracle (norm-wise and element-wise
scaled, 1e-5 in FP32, 1e-2 with BF16 intermediates) on the same seeded inputs, or, where the
oracle would take minutes, with closed forms of the adjoint that hold at any size.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import born, pauli
from tests._cases import close, rel

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL32 = 1e-5


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _case(seed, n, R, B, shots=100_000):
    rng = synth.make_rng(seed)
    D = 1 << n
    atoms = synth.haar_atoms(rng, R, D, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    f = synth.porter_thomas_freqs(rng, B, D, synth.dirichlet_weights(rng, 3), shots)
    return dict(atoms=atoms, weights=w, settings=s, freqs=f)


def _inst(case, S=0, unitaries=None):
    from paper_2607_19577_amd import api

    return api.Instance(torch.from_numpy(case["atoms"]).to(DEV), torch.from_numpy(case["weights"]).to(DEV),
                        torch.from_numpy(case["settings"]).to(DEV), torch.from_numpy(case["freqs"]).to(DEV),
                        settings_per_batch=S, unitaries=unitaries)


def _gpu(h, inst, path=None, loss=None):
    from paper_2607_19577_amd import api

    path = api.PATH_BUTTERFLY_F32 if path is None else path
    loss = api.LOSS_CE if loss is None else loss
    probs, _ = api.qst_forward(h, [inst], want_probs=True, path=path)
    lt, ag, wg = api.qst_backward(h, [inst], loss=loss, eps=1e-8, path=path)
    torch.cuda.synchronize()
    return float(lt[0]), probs[0].cpu().numpy(), ag[0].cpu().numpy(), wg[0].cpu().numpy()


def _oracle(case):
    return born.forward_backward(case["atoms"].astype(np.complex128), case["weights"], case["settings"],
                                 case["freqs"].astype(np.float64), born.LOSS_CE, 1e-8, tier="axis")


def _check(got, ref, tol, what):
    L, p, ga, gw = got
    Lr, pr, gar, gwr = ref
    assert abs(L - Lr) <= tol * abs(Lr), (what, "loss", L, Lr)
    assert close(p, pr, tol), (what, "probs", rel(p, pr))
    for r in range(ga.shape[0]):
        assert close(ga[r], gar[r], tol), (what, "atom_grad", r, rel(ga[r], gar[r]))
    assert close(gw, gwr, tol), (what, "weight_grad", rel(gw, gwr))


def test_three_pass_n20_r17_against_the_oracle(h):
    """n=20, R=17 (nine low bits would leave eleven above them): the two-sweep low stage over ten
    bits with dense frequencies, and the middle pass (five bits, top pass of six) with the same
    frequencies in CSR form; two settings in two batches of one."""
    case = _case(9101, 20, 17, 2)
    ref = _oracle(case)
    _check(_gpu(h, _inst(case, S=1)), ref, TOL32, "n=20 R=17 two-sweep low stage")
    _check(_gpu(h, _sparse(_inst(case, S=1))), ref, TOL32, "n=20 R=17 middle pass (sparse data)")


def _sparse(inst):
    rp, ix, vals = synth.dense_to_csr(inst.freqs.cpu().numpy())
    inst.freqs = None
    inst.freqs_csr = (torch.from_numpy(rp).to(DEV), torch.from_numpy(ix).to(DEV), torch.from_numpy(vals).to(DEV))
    return inst


def test_two_sweep_low_stage_equals_the_middle_pass(h):
    """n=21, R=16, six settings in batches of four: the two-sweep low stage (dense data) and the
    middle pass (the same data in CSR form) give the same loss, probabilities and gradients to
    rounding, for the CE and LS losses, in FP32 and (CE) with BF16 intermediates (1e-2)."""
    from paper_2607_19577_amd import api

    case = _case(9105, 21, 16, 6, shots=20_000)
    for path, tol, loss in ((api.PATH_BUTTERFLY_F32, TOL32, api.LOSS_CE), (api.PATH_BUTTERFLY_F32, TOL32, api.LOSS_LS),
                            (api.PATH_BUTTERFLY_BF16, 1e-2, api.LOSS_CE)):
        a = _gpu(h, _inst(case, S=4), path=path, loss=loss)
        b = _gpu(h, _sparse(_inst(case, S=4)), path=api.PATH_BUTTERFLY_F32, loss=loss)
        _check(a, b, tol, f"two sweeps vs middle pass, path {path}, loss {loss}")


def test_two_sweep_low_stage_n22_against_the_oracle(h):
    """n=22, R=16: the two-sweep low stage over twelve bits (128 threads per atom), one setting,
    against the oracle."""
    case = _case(9106, 22, 16, 1)
    _check(_gpu(h, _inst(case)), _oracle(case), TOL32, "n=22 R=16 two-sweep low stage")


def test_three_pass_equals_two_pass_with_a_zero_weight_atom(h):
    """R=17 with the last atom at weight zero describes the R=16 state (three passes against two):
    same loss, probabilities, weight gradients of the first 16 atoms and atom gradients, and the
    seventeenth atom's gradient is alpha_17 (= 0) times its adjoint."""
    case = _case(9102, 20, 16, 24)
    extra = synth.haar_atoms(synth.make_rng(9103), 1, 1 << 20, dtype=np.complex64)
    w17 = np.concatenate([case["weights"], [0.0]])
    case17 = dict(atoms=np.concatenate([case["atoms"], extra]), weights=w17, settings=case["settings"],
                  freqs=case["freqs"])
    L16, p16, ga16, gw16 = _gpu(h, _inst(case))
    L17, p17, ga17, gw17 = _gpu(h, _inst(case17))
    assert abs(L17 - L16) <= TOL32 * abs(L16)
    assert close(p17, p16, TOL32), rel(p17, p16)
    assert close(gw17[:16], gw16, TOL32), rel(gw17[:16], gw16)
    for r in range(16):
        assert close(ga17[r], ga16[r], TOL32), (r, rel(ga17[r], ga16[r]))
    assert np.abs(ga17[16]).max() == 0.0


@pytest.mark.parametrize("n,R", [(21, 16), (22, 4), (22, 16), (23, 8), (24, 2)])
def test_beyond_twenty_qubits_closed_forms(h, n, R):
    """n=21..24: the two-sweep low stage over 11 to 14 bits (R = 16, 16, 8, 2) and two plain tile
    passes (n=22 at R=4): sensitivity g = 1 gives alpha_r B psi_r
    and B ||psi_r||^2 (V^dagger V = 1 per setting); g = (-1)^{u_j} gives alpha_r sum_b
    sigma^(j)_{s_bj} psi_r for qubit j, one in each pass; a Z-only setting's probabilities are
    sum_r alpha_r |psi_r|^2; and every setting's probabilities sum to sum_r alpha_r ||psi_r||^2."""
    from paper_2607_19577_amd import api

    B = 6
    D = 1 << n
    rng = synth.make_rng(9200 + n)
    atoms = synth.haar_atoms(rng, R, D, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    s[0, :] = 2  # all Z
    inst = api.Instance(torch.from_numpy(atoms).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(s).to(DEV),
                        torch.ones((B, D), dtype=torch.float32, device=DEV) / D)
    psi = atoms.astype(np.complex128)
    probs, _ = api.qst_forward(h, [inst], want_probs=True)
    ones = torch.ones((B, D), dtype=torch.float32, device=DEV)
    _, ag, wg = api.qst_backward(h, [inst], grad_p=[ones])
    torch.cuda.synchronize()
    p = probs[0].cpu().numpy()
    want0 = (w[:, None] * np.abs(psi) ** 2).sum(axis=0)
    assert close(p[0], want0, TOL32), rel(p[0], want0)
    tot = float((w * (np.abs(psi) ** 2).sum(axis=1)).sum())
    assert np.allclose(p.astype(np.float64).sum(axis=1), tot, rtol=1e-5)
    got = ag[0].cpu().numpy()
    for r in (0, R - 1):
        assert close(got[r], w[r] * B * psi[r], TOL32), rel(got[r], w[r] * B * psi[r])
    assert close(wg[0].cpu().numpy(), B * (np.abs(psi) ** 2).sum(axis=1), TOL32)
    del ones
    # one qubit in each pass of the geometry (low stage, middle or top)
    for j in (0, n // 2, n - 1):
        bit = n - 1 - j
        sign = 1.0 - 2.0 * ((torch.arange(D, device=DEV) >> bit) & 1).float()
        _, ag, _ = api.qst_backward(h, [inst], grad_p=[sign.expand(B, D).contiguous()])
        torch.cuda.synchronize()
        got = ag[0].cpu().numpy()
        counts = [int((s[:, j] == c).sum()) for c in (0, 1, 2)]
        r = R // 2
        t = psi[r].reshape((2,) * n)
        want = np.zeros(D, dtype=np.complex128)
        for c in (0, 1, 2):
            want += counts[c] * np.moveaxis(np.tensordot(pauli.SIGMA[c], t, axes=([1], [j])), 0, j).reshape(-1)
        assert close(got[r], w[r] * want, TOL32), (j, rel(got[r], w[r] * want))


def test_three_pass_general_settings_and_bf16(h):
    """The middle pass with general local settings (the Pauli matrices as a table: the Pauli
    result to rounding) and with BF16 intermediates (1e-2 of the FP32 three-pass result)."""
    from paper_2607_19577_amd import api

    case = _case(9301, 20, 17, 5)
    ref = _gpu(h, _inst(case))
    table = torch.from_numpy(np.stack([pauli.single(k) for k in (pauli.X, pauli.Y, pauli.Z)])).to(DEV)
    gen = dict(case, settings=(case["settings"] + 3).astype(np.uint8))
    got = _gpu(h, _inst(gen, unitaries=table))
    _check(got, ref, TOL32, "general settings, three passes")
    got16 = _gpu(h, _inst(case), path=api.PATH_BUTTERFLY_BF16)
    _check(got16, ref, 1e-2, "BF16 intermediates, three passes")


@pytest.mark.parametrize("n,R", [(8, 64), (12, 40), (15, 256), (16, 100)])
def test_ranks_above_sixteen_against_the_oracle(h, n, R):
    """Fused slices (n=8, R=64: R 2^n = 2^14), on chip (n=12, R=40, atoms in turn), the staged low
    stage with six low bits (n=15, R=256) and with seven (n=16, R=100), against the oracle."""
    case = _case(9400 + n, n, R, 2)
    _check(_gpu(h, _inst(case)), _oracle(case), TOL32, f"n={n} R={R}")


def _pauli_on_qubit(psi, n, j, code):
    """sigma_code on qubit j (index bit n-1-j) of a device vector, with torch only."""
    v = psi.reshape(1 << j, 2, 1 << (n - 1 - j))
    if code == 2:  # Z
        return torch.cat([v[:, :1], -v[:, 1:]], dim=1).reshape(-1)
    if code == 0:  # X
        return torch.cat([v[:, 1:], v[:, :1]], dim=1).reshape(-1)
    return torch.cat([-1j * v[:, 1:], 1j * v[:, :1]], dim=1).reshape(-1)  # Y


@pytest.mark.parametrize("n", [26, 28])
def test_largest_states_closed_forms_on_device(h, n):
    """n=26 and n=28 at R=1 (the largest states one 4 GiB buffer range holds: three passes, the
    low stage over fourteen bits, a middle pass of six or seven and a top pass of six or seven),
    three settings, the first all Z.  Closed forms evaluated with torch on the device: the all-Z
    probabilities alpha |psi|^2; every setting's probabilities sum to alpha ||psi||^2; g = 1
    gives alpha B psi; g = (-1)^{u_j} gives alpha sum_b sigma^(j)_{s_bj} psi for one qubit in
    each pass."""
    from paper_2607_19577_amd import api

    B, D = 3, 1 << n
    gen = torch.Generator(device=DEV).manual_seed(9500 + n)
    psi = torch.complex(torch.randn(D, generator=gen, device=DEV), torch.randn(D, generator=gen, device=DEV))
    psi = (psi / torch.linalg.vector_norm(psi)).to(torch.complex64).reshape(1, D)
    w = torch.tensor([0.75], dtype=torch.float64, device=DEV)
    s = synth.random_settings(synth.make_rng(9500 + n), B, n)
    s[0, :] = 2
    inst = api.Instance(psi, w, torch.from_numpy(s).to(DEV), torch.full((B, D), 1.0 / D, device=DEV))
    probs, _ = api.qst_forward(h, [inst], want_probs=True)
    torch.cuda.synchronize()
    p = probs[0]
    a2 = (psi[0].real.double() ** 2 + psi[0].imag.double() ** 2)
    want0 = 0.75 * a2
    assert float(torch.linalg.vector_norm(p[0].double() - want0) / torch.linalg.vector_norm(want0)) <= TOL32
    tot = 0.75 * float(a2.sum())
    assert torch.allclose(p.double().sum(dim=1), torch.full((B,), tot, dtype=torch.float64, device=DEV), rtol=1e-5)
    del probs, p
    ones = torch.ones((B, D), dtype=torch.float32, device=DEV)
    _, ag, _ = api.qst_backward(h, [inst], grad_p=[ones])
    torch.cuda.synchronize()
    want = 0.75 * B * psi[0].to(torch.complex128)
    assert float(torch.linalg.vector_norm(ag[0][0].to(torch.complex128) - want) / torch.linalg.vector_norm(want)) <= TOL32
    del ones, ag
    for j in (0, n // 2, n - 1):
        bit = n - 1 - j
        sign = 1.0 - 2.0 * ((torch.arange(D, device=DEV) >> bit) & 1).float()
        _, ag, _ = api.qst_backward(h, [inst], grad_p=[sign.expand(B, D).contiguous()])
        torch.cuda.synchronize()
        want = torch.zeros(D, dtype=torch.complex128, device=DEV)
        p64 = psi[0].to(torch.complex128)
        for b in range(B):
            want += _pauli_on_qubit(p64, n, j, int(s[b, j]))
        want *= 0.75
        got = ag[0][0].to(torch.complex128)
        assert float(torch.linalg.vector_norm(got - want) / torch.linalg.vector_norm(want)) <= TOL32, j
        del ag, sign, want, got, p64
