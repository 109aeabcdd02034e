"""GPU parity of the on-chip path (states of 2^11 .. 2^14 amplitudes whose atoms do not all
fit one low-stage work-group: every (setting, atom) rotation on chip, the atoms looped in
the forward pass, the adjoint summed over slices of settings) against the FP64 oracle.

Shapes span one to four vectors per work-group, ragged atom tiles and setting groups, one
and many slices; the n=14, R=8, B=1000 workload is checked at its full size on sampled
settings and through closed forms of the adjoint (g = 1 and g = (-1)^(u_j))."""
import numpy as np
import pytest
import torch

from oracle import born, pauli
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-5


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _say(*a):
    print("onchip:", *a, flush=True)


def _check_all(h, case, kind, what, tangent=False):
    from paper_2607_19577_amd import api

    inst = to_device(case, DEV)
    _say(what)
    probs, lf = api.qst_forward(h, [inst], want_probs=True, loss=kind, eps=1e-8)
    lt, ag, wg = api.qst_backward(h, [inst], loss=kind, eps=1e-8, project_tangent=tangent)
    torch.cuda.synchronize()
    Lr, pr, gar, gwr = oracle(case, kind, 1e-8, tier="axis")
    if tangent:
        gar = born.tangent_project(case["atoms"].astype(np.complex128), gar)
    assert abs(float(lf[0]) - Lr) <= TOL * abs(Lr), (what, "forward loss")
    assert abs(float(lt[0]) - Lr) <= TOL * abs(Lr), (what, "loss")
    assert close(probs[0].cpu().numpy(), pr, TOL), (what, "probs", rel(probs[0].cpu().numpy(), pr))
    ga = ag[0].cpu().numpy()
    for r in range(ga.shape[0]):
        assert close(ga[r], gar[r], TOL), (what, "atom_grad", r, rel(ga[r], gar[r]))
    assert close(wg[0].cpu().numpy(), gwr, TOL), (what, "weight_grad")


@pytest.mark.parametrize("n,R,B", [
    (11, 9, 7),    # four atoms per work-group (one wavefront each), three tiles with a ragged one
    (11, 16, 3),
    (12, 6, 13),   # two vectors per work-group, two settings per forward item
    (13, 3, 9),    # one vector of four wavefronts
    (14, 2, 5),    # 512 threads, one vector
    (14, 8, 3),
])
def test_onchip_shapes_ce(h, n, R, B):
    case = make_case(900 + 7 * n + R, n, R, B, shots=5000)
    _check_all(h, case, born.LOSS_CE, f"CE n={n} R={R} B={B}")


def test_onchip_ls_and_tangent(h):
    case = make_case(931, 13, 4, 6, shots=2000)
    _check_all(h, case, born.LOSS_LS, "LS n=13 R=4 B=6")
    case = make_case(932, 14, 3, 4, shots=2000)
    _check_all(h, case, born.LOSS_CE, "CE tangent n=14 R=3 B=4", tangent=True)


def test_onchip_one_setting_one_slice(h):
    # B = 1: one slice, the adjoint written straight into the gradient
    case = make_case(933, 14, 3, 1, shots=2000)
    _check_all(h, case, born.LOSS_CE, "CE n=14 R=3 B=1")


def test_onchip_generic_sensitivity(h):
    from paper_2607_19577_amd import api

    case = make_case(934, 12, 7, 5, freqs=False)
    rng = np.random.default_rng(934)
    gp = rng.standard_normal((5, 1 << 12)).astype(np.float32)
    _say("grad_p n=12 R=7 B=5")
    inst = to_device(case, DEV)
    _, ag, wg = api.qst_backward(h, [inst], grad_p=[torch.from_numpy(gp).to(DEV)])
    torch.cuda.synchronize()
    _, _, gar, gwr = oracle(case, grad_p=gp.astype(np.float64))
    ga = ag[0].cpu().numpy()
    for r in range(7):
        assert close(ga[r], gar[r], TOL), ("atom_grad", r, rel(ga[r], gar[r]))
    assert close(wg[0].cpu().numpy(), gwr, TOL)


def test_onchip_base_probabilities(h):
    # p = base + sum_r alpha_r |V psi_r|^2: probabilities, loss and gradients act on that p
    from paper_2607_19577_amd import api

    case = make_case(935, 14, 2, 4, shots=3000)
    rng = np.random.default_rng(935)
    base = (rng.random((4, 1 << 14)) * 1e-4).astype(np.float32)
    inst = to_device(case, DEV)
    inst.probs_base = torch.from_numpy(base).to(DEV)
    _say("base n=14 R=2 B=4")
    probs, lf = api.qst_forward(h, [inst], want_probs=True, loss=api.LOSS_CE, eps=1e-8)
    lt, ag, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8)
    torch.cuda.synchronize()
    atoms = case["atoms"].astype(np.complex128)
    s, f = case["settings"], case["freqs"].astype(np.float64)
    p = born.probs_axis(atoms, case["weights"], s) + base.astype(np.float64)
    L, g = born.loss_and_sensitivity(p, f, 4, born.LOSS_CE, 1e-8)
    gar, gwr = born.gradients_axis(atoms, case["weights"], s, g)
    assert close(probs[0].cpu().numpy(), p, TOL)
    assert abs(float(lf[0]) - L) <= TOL * abs(L) and abs(float(lt[0]) - L) <= TOL * abs(L)
    ga = ag[0].cpu().numpy()
    for r in range(2):
        assert close(ga[r], gar[r], TOL), ("atom_grad", r, rel(ga[r], gar[r]))
    assert close(wg[0].cpu().numpy(), gwr, TOL)


def test_onchip_full_n14_r8_b1000(h):
    """n=14, R=8, B=1000 at full size: probabilities of sampled settings against the oracle, and
    the adjoint against its closed forms for g = 1 (sum_b V_b^dagger V_b = B I) and
    g = (-1)^(u_j) (single-qubit Pauli action on qubit j)."""
    from paper_2607_19577_amd import api

    n, R, B = 14, 8, 1000
    D = 1 << n
    case = make_case(936, n, R, B, freqs=False)
    inst = to_device(case, DEV)
    _say("full n=14 R=8 B=1000 forward")
    probs, _ = api.qst_forward(h, [inst], want_probs=True)
    torch.cuda.synchronize()
    rows = [0, 1, 377, 640, 999]
    pr = born.probs_axis(case["atoms"].astype(np.complex128), case["weights"], case["settings"], rows=rows)
    pg = probs[0].cpu().numpy()[rows]
    assert close(pg, pr, TOL), rel(pg, pr)
    del probs
    atoms = case["atoms"].astype(np.complex128)
    w = case["weights"]
    _say("full n=14 R=8 B=1000 adjoint, g = 1")
    ones = torch.ones((B, D), dtype=torch.float32, device=DEV)
    _, ag, wg = api.qst_backward(h, [inst], grad_p=[ones])
    torch.cuda.synchronize()
    ga = ag[0].cpu().numpy()
    for r in range(R):
        assert close(ga[r], w[r] * B * atoms[r], TOL), ("g=1", r, rel(ga[r], w[r] * B * atoms[r]))
    assert close(wg[0].cpu().numpy(), B * np.sum(np.abs(atoms) ** 2, axis=1), TOL)
    j = 5
    sign = np.array([1.0 - 2.0 * ((u >> (n - 1 - j)) & 1) for u in range(D)], dtype=np.float32)
    _say("full n=14 R=8 B=1000 adjoint, g = (-1)^u_j")
    gsgn = torch.from_numpy(sign).to(DEV).expand(B, D).contiguous()
    _, ag, _ = api.qst_backward(h, [inst], grad_p=[gsgn])
    torch.cuda.synchronize()
    ga = ag[0].cpu().numpy()
    counts = np.bincount(case["settings"][:, j].astype(np.int64), minlength=3)
    op = sum(counts[c] * pauli.SIGMA[c] for c in range(3))
    for r in range(R):
        t = atoms[r].reshape((2,) * n)
        want = w[r] * np.moveaxis(np.tensordot(op, t, axes=([1], [j])), 0, j).reshape(-1)
        assert close(ga[r], want, TOL), ("sign", r, rel(ga[r], want))


def test_onchip_multi_instance_call(h):
    """Several on-chip instances of different n in one call (one launch of each pass per n),
    beside a staged and a one-chunk instance, each equal to the oracle."""
    from paper_2607_19577_amd import api

    cases = [make_case(940 + i, n, R, B, shots=3000)
             for i, (n, R, B) in enumerate([(12, 5, 6), (14, 2, 3), (12, 8, 4), (11, 12, 5), (9, 3, 7), (15, 2, 3)])]
    insts = [to_device(c, DEV) for c in cases]
    _say("multi-instance call")
    lt, ag, wg = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        Lr, _, gar, gwr = oracle(c, born.LOSS_CE, 1e-8)
        gar = born.tangent_project(c["atoms"].astype(np.complex128), gar)
        assert abs(float(lt[i]) - Lr) <= TOL * abs(Lr), (i, "loss")
        ga = ag[i].cpu().numpy()
        for r in range(ga.shape[0]):
            assert close(ga[r], gar[r], TOL), (i, r, rel(ga[r], gar[r]))
        assert close(wg[i].cpu().numpy(), gwr, TOL), (i, "weight_grad")
