"""GPU runs of the rank-adaptive iteration (Algorithm 1, qst_solve) and of the Gram-form
state error (qst_state_error), through the C ABI.

* FP64 path against the oracle's driver on the same inputs (same start vectors): the same
  slot kinds, acceptances, grid indices, ranks and oracle-call count, J to 1e-9 and the final
  density to 1e-8 (Ritz vectors carry arbitrary phases, so densities are compared).
* FP32 path: J never increases, each accepted slot decreases it by at least tau_acc, and the
  oracle's objective of the returned state equals the reported final J to 1e-5.
* Stopping rules; exact recovery of a pure state from noiseless data.
* State error against the oracle (1e-6 FP32 atoms, 1e-12 FP64).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import born, loop

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


def _problem(seed, n, R, B, shots=2000, complex_dtype=np.complex128, R_true=2):
    rng = synth.make_rng(seed)
    s = synth.random_settings(rng, B, n)
    truth = synth.haar_atoms(rng, R_true, 1 << n)
    wt = synth.dirichlet_weights(rng, R_true)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), shots).astype(np.float32)
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=complex_dtype)
    w = np.full(R, 1.0 / R)
    v0s = synth.haar_atoms(rng, 2, 1 << n, dtype=np.complex128)
    return atoms, w, s, f, v0s


def _inst(atoms, w, s, f):
    from paper_2607_19577_amd import api

    return api.Instance(torch.from_numpy(atoms).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(s).to(DEV),
                        torch.from_numpy(f).to(DEV))


@pytest.mark.parametrize("n,R,B,slots,t_alpha,t_ref", [(3, 3, 18, 40, 4, 9), (4, 4, 30, 36, 5, 10)])
def test_solve_f64_matches_oracle_driver(h, n, R, B, slots, t_alpha, t_ref):
    from paper_2607_19577_amd import api

    atoms, w, s, f, v0s = _problem(1500 + n, n, R, B)
    prm = api.SolveParams(max_slots=slots, t_alpha=t_alpha, t_ref=t_ref, rank_max=R, n_lanczos=12, stop_window=0,
                          oracle_budget=0, eps=1e-8)
    res = api.qst_solve(h, _inst(atoms, w, s, f), prm, torch.from_numpy(v0s).to(DEV), path=api.PATH_BUTTERFLY_F64)
    hist, info = [], {}
    oa, ow, oJ = loop.run(atoms, w, s, f.astype(np.float64), kind=born.LOSS_CE, eps=1e-8, mu=prm.mu, tau=prm.tau,
                          tau_acc=prm.tau_acc, iters=slots, t_alpha=t_alpha, t_ref=t_ref, L_max=R, n_lanczos=12,
                          v0s=list(v0s), history=hist, info=info)
    gh = res["history"]
    assert res["slots"] == info["slots"] == slots
    assert any(x[4] for x in hist), "nothing accepted: the case does not exercise the driver"
    for k, (t, kind, J, Rk, acc, j) in enumerate(hist):
        g = gh[k]
        assert (int(g[0]), int(g[1]), int(g[3]), bool(g[4]), int(g[5])) == (t, kind, Rk, acc, j), (k, g, hist[k])
        assert abs(g[2] - J) <= 1e-9 * abs(J), (k, g[2], J)
    assert res["oracle_calls"] == info["oracle_calls"]
    assert res["rank"] == ow.size
    rho_g = born.density(res["atoms"].cpu().numpy(), res["weights"].cpu().numpy())
    assert np.abs(rho_g - born.density(oa, ow)).max() < 1e-8


def test_solve_f32_monotone_and_consistent(h):
    from paper_2607_19577_amd import api

    n, R, B = 8, 4, 40
    atoms, w, s, f, v0s = _problem(1520, n, R, B, shots=5000, complex_dtype=np.complex64)
    prm = api.SolveParams(max_slots=45, t_alpha=5, t_ref=20, rank_max=6, n_lanczos=20, stop_window=0,
                          oracle_budget=0, eps=1e-8)
    res = api.qst_solve(h, _inst(atoms, w, s, f), prm, torch.from_numpy(v0s).to(DEV))
    hist = res["history"]
    Jprev = None
    for t, kind, J, Rk, acc, j in hist:
        if Jprev is not None:
            assert (J <= Jprev - prm.tau_acc) if acc else (J == Jprev)
        Jprev = J
    assert hist[:, 4].sum() >= 5
    a = res["atoms"].cpu().numpy().astype(np.complex128)
    wv = res["weights"].cpu().numpy()
    assert np.allclose(np.linalg.norm(a, axis=1), 1.0, atol=1e-5)
    Jo, _ = loop.objective(a, wv, s, f.astype(np.float64), born.LOSS_CE, 1e-8, prm.mu)
    assert abs(Jo - hist[-1, 2]) <= 1e-5 * abs(Jo), (Jo, hist[-1, 2])


def test_solve_stopping_rules(h):
    from paper_2607_19577_amd import api

    atoms, w, s, f, v0s = _problem(1530, 3, 3, 18)
    inst = _inst(atoms, w, s, f)
    v0 = torch.from_numpy(v0s).to(DEV)
    res = api.qst_solve(h, inst, api.SolveParams(max_slots=200, rank_max=3, n_lanczos=8, oracle_budget=40,
                                                 stop_window=0), v0, path=api.PATH_BUTTERFLY_F64)
    assert res["stopped"] == "budget" and res["oracle_calls"] >= 40 and res["slots"] < 200
    res = api.qst_solve(h, inst, api.SolveParams(max_slots=200, rank_max=3, n_lanczos=8, oracle_budget=0,
                                                 stop_window=3, stop_delta=10.0), v0, path=api.PATH_BUTTERFLY_F64)
    assert res["stopped"] == "delta" and res["history"][:, 4].sum() == 3


def test_solve_exact_recovery_pure_state(h):
    """Noiseless data of a pure state, all 3^N settings: the iteration prunes to one atom and
    reaches the truth (FP64 path; the data are stored in FP32)."""
    from paper_2607_19577_amd import api

    rng = synth.make_rng(1540)
    n = 2
    s = synth.all_settings(n)
    truth = synth.haar_atoms(rng, 1, 1 << n)
    f = born.probs_axis(truth, [1.0], s).astype(np.float32)
    atoms = synth.haar_atoms(rng, 2, 1 << n)
    w = np.array([0.5, 0.5])
    v0s = synth.haar_atoms(rng, 3, 1 << n)
    prm = api.SolveParams(max_slots=80, t_alpha=3, t_ref=4, rank_max=2, n_lanczos=30, stop_window=0, oracle_budget=0,
                          eps=0.0, tau_acc=0.0)
    res = api.qst_solve(h, _inst(atoms, w, s, f), prm, torch.from_numpy(v0s).to(DEV), path=api.PATH_BUTTERFLY_F64)
    assert res["rank"] == 1
    psi = res["atoms"][0].cpu().numpy()
    assert 1 - abs(np.vdot(psi, truth[0])) ** 2 < 1e-6
    e = api.qst_state_error(h, res["atoms"], res["weights"], torch.from_numpy(truth).to(DEV),
                            torch.ones(1, dtype=torch.float64, device=DEV), path=api.PATH_BUTTERFLY_F64)
    assert e < 2e-3


@pytest.mark.parametrize("cdt,path_name,tol", [(np.complex64, "PATH_BUTTERFLY_F32", 1e-6),
                                               (np.complex128, "PATH_BUTTERFLY_F64", 1e-12)])
def test_state_error_matches_oracle(h, cdt, path_name, tol):
    from paper_2607_19577_amd import api

    rng = synth.make_rng(1550)
    for n, Ra, Rb in ((4, 3, 2), (12, 5, 4)):
        ua = synth.haar_atoms(rng, Ra, 1 << n, dtype=cdt)
        ub = synth.haar_atoms(rng, Rb, 1 << n, dtype=cdt)
        wa = synth.dirichlet_weights(rng, Ra)
        wb = synth.dirichlet_weights(rng, Rb)
        e = api.qst_state_error(h, torch.from_numpy(ua).to(DEV), torch.from_numpy(wa).to(DEV),
                                torch.from_numpy(ub).to(DEV), torch.from_numpy(wb).to(DEV),
                                path=getattr(api, path_name))
        want = born.state_error(ua, wa, ub, wb)
        assert abs(e - want) <= tol * want, (n, e, want)
