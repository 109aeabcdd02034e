"""Pins of the oracle's iteration driver (Algorithm 1 order): the acceptance rule holds on
every recorded slot, the oracle-call count equals the per-slot tally rebuilt from the history,
and the two stopping rules of Table sim-parameters end the run where they should."""
import numpy as np

import synth
from oracle import born, loop


def _problem(seed, n=3, R=3, B=18):
    rng = synth.make_rng(seed)
    s = synth.random_settings(rng, B, n)
    truth = synth.haar_atoms(rng, 2, 1 << n)
    wt = synth.dirichlet_weights(rng, 2)
    f = synth.multinomial_freqs(rng, born.probs_axis(truth, wt, s), 2000)
    atoms = synth.haar_atoms(rng, R, 1 << n)
    w = np.full(R, 1.0 / R)
    v0s = [synth.haar_atoms(rng, 1, 1 << n)[0] for _ in range(2)]
    return atoms, w, s, f, v0s


def _tally(history, n_grid, n_lanczos, D):
    # 1 for the initial objective; per slot: gradient product + one per trial (atom,
    # coefficient), or (Lanczos products + 1) per trial (spectral)
    calls = 1
    for _, kind, _, _, acc, j in history:
        trials = j + 1 if acc else n_grid
        if kind == loop.KIND_RHO:
            calls += trials * (min(n_lanczos, D) + 1)
        else:
            calls += 1 + trials
    return calls


def test_history_obeys_acceptance_and_the_count_is_the_tally():
    atoms, w, s, f, v0s = _problem(200)
    hist, info = [], {}
    tau_acc = 1e-10
    loop.run(atoms, w, s, f, kind=born.LOSS_CE, eps=1e-8, mu=1e-3, tau_acc=tau_acc, iters=30, t_alpha=4, t_ref=9,
             n_lanczos=6, v0s=v0s, history=hist, info=info)
    J_prev = None
    for t, kind, J, R, acc, j in hist:
        assert kind == loop.slot_kind(t, 4, 9)
        if J_prev is not None:
            assert (J <= J_prev - tau_acc) if acc else (J == J_prev)
        J_prev = J
    assert info["slots"] == 30 and info["stopped"] == "T"
    assert info["oracle_calls"] == _tally(hist, 11, 6, 8)


def test_stopping_rules():
    atoms, w, s, f, v0s = _problem(201)
    hist, info = [], {}
    loop.run(atoms, w, s, f, eps=1e-8, iters=200, t_alpha=5, t_ref=50, n_lanczos=8, v0s=v0s, history=hist,
             info=info, oracle_budget=40)
    assert info["stopped"] == "budget" and info["oracle_calls"] >= 40
    assert _tally(hist[:-1], 11, 8, 8) < 40  # the slot before the last had not reached it
    hist, info = [], {}
    loop.run(atoms, w, s, f, eps=1e-8, iters=200, t_alpha=5, t_ref=50, n_lanczos=8, v0s=v0s, history=hist,
             info=info, stop_window=3, stop_delta=10.0)  # any decrease is below 10: stop at 3 accepted
    assert info["stopped"] == "delta"
    assert sum(1 for h in hist if h[4]) == 3 and hist[-1][4]
