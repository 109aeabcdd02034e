"""GPU parity of the boundary steps and the integration surfaces against the oracle.

* simplex reweight + pruning (eq. coefficient-update, eq. truncation-map): FP64,
  compared to the sort-based oracle projection to 1e-13 with identical keep sets;
* spectral refactorisation (eq. density-proposal .. eq. spectral-selection): the
  library's Lanczos against the oracle's with the same start vector -- FP64 path
  to 1e-9 (Ritz values, scores, weights, chosen density), FP32 path to 1e-5 on
  the leading Ritz values; at k = D the Ritz values are the exact spectrum of S;
* torch.autograd: gradcheck of the FP64 Born map, and the fused loss against
  the oracle;
* the plain per-qubit path against the oracle (1e-5);
* hipGraph capture of backward + reweight, replayed with eager work in between,
  every replay equal to the eager result bit for bit.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import born, refactor, simplex
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


# ---------------------------------------------------------------- a9: reweight
REWEIGHT_CASES = [
    # (seed, R, eta, tau)
    (1, 1, 0.5, 0.0),
    (2, 2, 0.5, 1e-3),
    (3, 5, -0.5, 1e-3),
    (4, 16, 0.3, 1e-2),
    (5, 16, 5.0, 0.05),
    (6, 64, 0.1, 1e-3),
    (7, 8, 0.5, 0.99),     # nothing above tau: the largest weight is kept alone
    (8, 300, 0.02, 1e-4),  # several waves of the single work-group
]


@pytest.mark.parametrize("seed,R,eta,tau", REWEIGHT_CASES)
def test_reweight_matches_oracle(h, seed, R, eta, tau):
    from paper_2607_19577_amd import api

    rng = synth.make_rng(seed)
    alpha = synth.dirichlet_weights(rng, R)
    hv = rng.standard_normal(R)
    out, keep, rout = api.qst_reweight_simplex(h, torch.from_numpy(alpha).to(DEV), torch.from_numpy(hv).to(DEV),
                                               eta, tau)
    torch.cuda.synchronize()
    ro, ko, Ro = simplex.reweight(alpha, hv, eta, tau)
    Rg = int(rout.cpu()[0])
    assert Rg == Ro
    np.testing.assert_array_equal(keep.cpu().numpy()[:Rg], ko)
    assert np.all(keep.cpu().numpy()[Rg:] == -1)
    np.testing.assert_allclose(out.cpu().numpy(), ro, rtol=0, atol=1e-13)
    assert abs(out.cpu().numpy()[:Rg].sum() - 1.0) < 1e-13


def test_reweight_ties_and_identity(h):
    """h = 0 and eta = 0: the projection of a simplex point is itself (idempotence)."""
    from paper_2607_19577_amd import api

    alpha = np.full(6, 1.0 / 6)
    out, keep, rout = api.qst_reweight_simplex(h, torch.from_numpy(alpha).to(DEV),
                                               torch.zeros(6, dtype=torch.float64, device=DEV), 0.0, 0.0)
    torch.cuda.synchronize()
    assert int(rout.cpu()[0]) == 6
    np.testing.assert_array_equal(keep.cpu().numpy(), np.arange(6))
    np.testing.assert_allclose(out.cpu().numpy(), alpha, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- a10: refactor
def _dense_rho(atoms, weights):
    a = np.asarray(atoms, dtype=np.complex128)
    return (a.T * np.asarray(weights)) @ a.conj()


def _run_refactor(h, case, path, L_max, k, v0, eta_rho=0.5, mu=1e-3, tau=1e-3, eps=1e-8):
    from paper_2607_19577_amd import api

    inst = to_device(case, DEV)
    out = api.qst_refactor(h, inst, api.LOSS_CE, eps, eta_rho, mu, tau, L_max, k,
                           torch.from_numpy(v0).to(DEV), path=path)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def _oracle_refactor(case, L_max, k, v0, eta_rho=0.5, mu=1e-3, tau=1e-3, eps=1e-8):
    return refactor.lanczos_refactor(case["atoms"].astype(np.complex128), case["weights"], case["settings"],
                                     case["freqs"].astype(np.float64), born.LOSS_CE, eps, eta_rho, mu, tau, L_max, k,
                                     v0)


def test_refactor_exact_spectrum_small(h):
    """n=3, all 27 settings, k = D: the Ritz values are the top of the exact spectrum of S."""
    from paper_2607_19577_amd import api

    case = make_case(301, 3, 2, 27, shots=1000, complex_dtype=np.complex128, exhaustive=True)
    v0 = synth.make_rng(302).standard_normal(8) + 1j * synth.make_rng(303).standard_normal(8)
    L = 4
    got = _run_refactor(h, case, api.PATH_BUTTERFLY_F64, L, 8, v0)
    # dense S = rho + eta G (Theorem 1 setting)
    atoms = case["atoms"]
    p = born.probs_dense(atoms, case["weights"], case["settings"])
    _, g = born.loss_and_sensitivity(p, case["freqs"].astype(np.float64), 27, born.LOSS_CE, 1e-8)
    S = refactor.density_proposal(born.density(atoms, case["weights"]), born.gradient_matrix_dense(case["settings"], g),
                                  0.5)
    lam = np.sort(np.linalg.eigvalsh(S))[::-1][:L]
    np.testing.assert_allclose(got["ritz_vals"][:L], lam, rtol=0, atol=1e-10 * max(1.0, abs(lam[0])))
    ref = _oracle_refactor(case, L, 8, v0)
    assert int(got["s_star"][0]) == ref["s_star"]
    assert int(got["R"][0]) == ref["R"]
    np.testing.assert_allclose(got["q_scores"][:L], ref["q_scores"], rtol=1e-9, atol=1e-12)
    R = ref["R"]
    np.testing.assert_allclose(got["weights"][:R], ref["weights"], rtol=0, atol=1e-10)
    rg = _dense_rho(got["atoms"][:R], got["weights"][:R])
    ro = _dense_rho(ref["atoms"], ref["weights"])
    assert np.linalg.norm(rg - ro) <= 1e-8 * np.linalg.norm(ro)


@pytest.mark.parametrize("path_name,tol", [("PATH_BUTTERFLY_F64", 1e-9), ("PATH_BUTTERFLY_F32", 1e-5)])
def test_refactor_lanczos_matches_oracle(h, path_name, tol):
    """n=8, R=3, B=40, k=24 Lanczos steps with the same start vector as the oracle."""
    from paper_2607_19577_amd import api

    path = getattr(api, path_name)
    cdt = np.complex128 if path == api.PATH_BUTTERFLY_F64 else np.complex64
    case = make_case(311, 8, 3, 40, shots=10_000, complex_dtype=cdt)
    rng = synth.make_rng(312)
    v0 = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    L = 5
    got = _run_refactor(h, case, path, L, 24, v0)
    ref = _oracle_refactor(case, L, 24, v0)
    lead = 2 if path == api.PATH_BUTTERFLY_F32 else L  # leading (converged) Ritz values for FP32 operators
    np.testing.assert_allclose(got["ritz_vals"][:lead], ref["ritz_vals"][:lead], rtol=tol, atol=0)
    if path == api.PATH_BUTTERFLY_F64:
        assert int(got["s_star"][0]) == ref["s_star"]
        assert int(got["R"][0]) == ref["R"]
        np.testing.assert_allclose(got["q_scores"][:L], ref["q_scores"], rtol=tol, atol=0)
        R = ref["R"]
        np.testing.assert_allclose(got["weights"][:R], ref["weights"], rtol=0, atol=tol)
        rg = _dense_rho(got["atoms"][:R], got["weights"][:R])
        ro = _dense_rho(ref["atoms"], ref["weights"])
        assert np.linalg.norm(rg - ro) <= 10 * tol * np.linalg.norm(ro)


# ---------------------------------------------------------------- autograd
def test_gradcheck_born_map_fp64(h):
    from paper_2607_19577_amd import api
    from paper_2607_19577_amd.autograd import born_map

    case = make_case(401, 3, 2, 4, complex_dtype=np.complex128, freqs=False)
    a = torch.from_numpy(case["atoms"]).to(DEV).requires_grad_(True)
    w = torch.from_numpy(case["weights"]).to(DEV).requires_grad_(True)
    s = torch.from_numpy(case["settings"]).to(DEV)
    fn = lambda aa, ww: born_map(aa, ww, s, h, api.PATH_BUTTERFLY_F64)  # noqa: E731
    assert torch.autograd.gradcheck(fn, (a, w), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_fused_loss_autograd_matches_oracle(h, kind):
    from paper_2607_19577_amd.autograd import fused_loss

    case = make_case(402, 7, 3, 12)
    inst = to_device(case, DEV)
    a = inst.atoms.clone().requires_grad_(True)
    w = inst.weights.clone().requires_grad_(True)
    L = fused_loss(a, w, inst.settings, inst.freqs, h, loss=kind, eps=1e-8)
    (3.0 * L).backward()
    torch.cuda.synchronize()
    Lr, _, gar, gwr = oracle(case, kind, 1e-8)
    assert abs(float(L.detach()) - Lr) <= 1e-5 * abs(Lr)
    # torch's complex gradient is twice the conjugate-Wirtinger gradient
    ga = a.grad.cpu().numpy() / (2 * 3.0)
    gw = w.grad.cpu().numpy() / 3.0
    for r in range(ga.shape[0]):
        assert close(ga[r], gar[r], 1e-5), (r, rel(ga[r], gar[r]))
    assert close(gw, gwr, 1e-5), rel(gw, gwr)


# ---------------------------------------------------------------- plain path
@pytest.mark.parametrize("n,R,B", [(3, 2, 5), (9, 4, 7), (13, 3, 4)])
def test_plain_path_matches_oracle(h, n, R, B):
    from paper_2607_19577_amd import api

    case = make_case(500 + n, n, R, B)
    inst = to_device(case, DEV)
    probs, _ = api.qst_forward(h, [inst], want_probs=True, path=api.PATH_PLAIN_F32)
    lt, ag, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=api.PATH_PLAIN_F32)
    torch.cuda.synchronize()
    Lr, pr, gar, gwr = oracle(case, born.LOSS_CE, 1e-8)
    assert abs(float(lt[0]) - Lr) <= 1e-5 * abs(Lr)
    assert close(probs[0].cpu().numpy(), pr, 1e-5)
    g = ag[0].cpu().numpy()
    for r in range(R):
        assert close(g[r], gar[r], 1e-5), (r, rel(g[r], gar[r]))
    assert close(wg[0].cpu().numpy(), gwr, 1e-5)


# ---------------------------------------------------------------- hipGraph capture
@pytest.mark.parametrize("n,R,B", [(12, 4, 30), (16, 4, 12)])
def test_graph_capture_replay(h, n, R, B):
    """backward (CE, tangent projection) + reweight captured once, replayed three times
    with unrelated eager work in between; each replay equals the eager result exactly."""
    from paper_2607_19577_amd import api

    case = make_case(600 + n, n, R, B)
    inst = to_device(case, DEV)
    api.qst_plan(h, [inst])

    def step():
        lt, ag, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
        out, keep, rout = api.qst_reweight_simplex(h, inst.weights, -wg[0], 0.5, 1e-3)
        return [lt, ag[0], wg[0], out, keep, rout]

    ref = [t.clone() for t in step()]
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        h.set_stream(side)
        step()  # warm-up on a side stream, as torch asks before a capture
    h.set_stream(torch.cuda.current_stream())
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        h.set_stream(torch.cuda.current_stream())
        outs = step()
    h.set_stream(torch.cuda.current_stream())

    small = to_device(make_case(700 + n, 6, 2, 5), DEV)
    for rep in range(3):
        # eager work between replays: other tensors and another (smaller) instance on the same handle
        x = torch.randn(256, 256, device=DEV)
        _ = (x @ x).sum()
        api.qst_forward(h, [small], want_probs=True)
        torch.cuda.synchronize()
        for t in outs:
            t.zero_() if t.dtype != torch.int32 else t.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip(outs, ref):
            assert torch.equal(got, want), (rep, got.dtype)
