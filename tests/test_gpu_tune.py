"""The autotuner (qst_plan with autotune) and pinned implementation choices (qst_plan_choice).

* Tuning one shape records a choice (tuned = 1, with the chosen and the default candidate's
  times); the tuned call gives the same bits as a fresh handle with that choice pinned, and
  agrees with an untuned handle to rounding (1e-5 norm-wise; different kernels associate the
  sums differently, so equal bits are not expected across choices) and with the oracle.
* A later handle on the same device reuses the process-wide choice without timing again.
* Every kind of kernels pinned at a shape where all apply matches the oracle.
* Tuning a multi-instance call keeps a routing policy; the tuned call matches the oracle and
  replays from a graph bit for bit.
* The order in which the low stage stores its output for the adjoint tile stage (w_row_bits)
  moves values, not sums: every order gives the same bits."""
import numpy as np
import pytest
import torch

from oracle import born
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-5


def _bw(h, insts):
    from paper_2607_19577_amd import api

    out = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=False)
    torch.cuda.synchronize()
    return out


def _vs_oracle(case, got, i=0):
    Lr, _, gar, gwr = oracle(case, born.LOSS_CE, 1e-8)
    assert abs(float(got[0][i]) - Lr) <= TOL * abs(Lr)
    ga = got[1][i].cpu().numpy()
    for r in range(ga.shape[0]):
        assert close(ga[r], gar[r], TOL), (r, rel(ga[r], gar[r]))
    assert close(got[2][i].cpu().numpy(), gwr, TOL)


def test_autotune_one_shape(tmp_path):
    from paper_2607_19577_amd import api

    case = make_case(1201, 14, 8, 64, shots=5000)
    inst = to_device(case, DEV)
    print("tune: n=14 R=8 B=64", flush=True)
    with api.Handle(0) as h1, api.Handle(0) as h2, api.Handle(0) as h3:
        api.qst_plan(h1, [inst], autotune=True)
        c = api.qst_plan_choice(h1, inst)
        assert c["tuned"] == 1 and c["best_ms"] > 0 and c["default_ms"] > 0, c
        assert c["best_ms"] <= c["default_ms"], c
        a = _bw(h1, [inst])
        pin = {k: c[k] for k in ("kind", "settings_per_batch", "tile_bits_fwd", "tile_bits_adj",
                                 "values_per_thread_log2", "w_row_bits", "x_row_bits")}
        got = api.qst_plan_choice(h2, inst, set_to=pin)
        assert got["kind"] == c["kind"] and got["tuned"] == 0
        b = _bw(h2, [inst])
        assert torch.equal(a[0], b[0]) and torch.equal(a[1][0], b[1][0]) and torch.equal(a[2][0], b[2][0])
        u = _bw(h3, [inst])
        assert api.qst_plan_choice(h3, inst)["kind"] == -1
        for r in range(8):
            assert rel(a[1][0][r].cpu().numpy(), u[1][0][r].cpu().numpy()) <= TOL, r
        _vs_oracle(case, a)
    with api.Handle(0) as h4:  # the process-wide cache: same choice, no new timing
        api.qst_plan(h4, [inst], autotune=True)
        c4 = api.qst_plan_choice(h4, inst)
        assert c4 == c, (c4, c)


@pytest.mark.parametrize("kind,lv,n", [(0, 0, 12), (1, 5, 12), (1, 4, 13), (1, 4, 14), (1, 5, 14), (2, 0, 12)])
def test_every_kind_matches_oracle(kind, lv, n):
    from paper_2607_19577_amd import api

    case = make_case(1210 + kind * 7 + lv + n, n, 16384 >> n, 24, shots=5000)  # R 2^n = 2^14: every kind applies
    inst = to_device(case, DEV)
    print("pinned kind", kind, "logv", lv, flush=True)
    with api.Handle(0) as h:
        api.qst_plan_choice(h, inst, set_to={"kind": kind, "values_per_thread_log2": lv})
        a = _bw(h, [inst])
        b = _bw(h, [inst])
        assert torch.equal(a[1][0], b[1][0])
        _vs_oracle(case, a)


def test_autotune_call_policy_and_graph():
    from paper_2607_19577_amd import api

    shapes = [(12, 6, 40), (11, 8, 30), (11, 3, 50), (9, 5, 60), (12, 2, 20), (10, 7, 25)]
    cases = [make_case(1230 + i, n, R, B, shots=3000) for i, (n, R, B) in enumerate(shapes)]
    insts = [to_device(c, DEV) for c in cases]
    print("tune: call of six instances", flush=True)
    with api.Handle(0) as h:
        api.qst_plan(h, insts, autotune=True)
        ref = _bw(h, insts)
        for i, c in enumerate(cases):
            _vs_oracle(c, ref, i)
        ref = [ref[0].clone(), [t.clone() for t in ref[1]], [t.clone() for t in ref[2]]]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            h.set_stream(side)
            api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8)
        h.set_stream(torch.cuda.current_stream())
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.set_stream(torch.cuda.current_stream())
            out = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8)
        h.set_stream(torch.cuda.current_stream())
        for rep in range(3):
            api.qst_forward(h, insts[:2], want_probs=True)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out[0], ref[0]), rep
            for x, y in zip(out[1], ref[1]):
                assert torch.equal(x, y), rep


@pytest.mark.parametrize("n,kind", [(19, "f32"), (19, "bf16"), (19, "general"), (21, "f32"), (21, "bf16")])
def test_w_layouts_give_the_same_bits(n, kind):
    """n=19, R=16 (tiles of 2^9 rows by 32 columns, so the orders of X and W matter) and n=21,
    R=16 (the two-sweep low stage over eleven bits, tiles of 2^10 rows by 16 columns), three
    batches of 16 settings: W in plain order (rows 2^n_lo apart) and with rows 2^5 (the default
    here), 2^6 and 2^8 apart, each with X in plain order or rows 2^6 (the default) or 2^5
    apart, give equal losses, probabilities and gradients, on the FP32 path, with BF16
    intermediates and with general local settings."""
    from paper_2607_19577_amd import api
    import synth

    rng = synth.make_rng(1250 + n)
    R, B = 16, 40
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_general_settings(rng, B, n, 2) if kind == "general" else synth.random_settings(rng, B, n)
    f = synth.porter_thomas_freqs(rng, B, 1 << n, synth.dirichlet_weights(rng, 3), 20000)
    unitaries = torch.from_numpy(synth.haar_unitaries_2x2(rng, 2)).to(DEV) if kind == "general" else None
    inst = api.Instance(torch.from_numpy(atoms).to(DEV), torch.from_numpy(w).to(DEV), torch.from_numpy(s).to(DEV),
                        torch.from_numpy(f).to(DEV), unitaries=unitaries)
    path = api.PATH_BUTTERFLY_BF16 if kind == "bf16" else api.PATH_BUTTERFLY_F32
    ref = None
    n_lo = n - 10 if n > 20 else 10
    for wb, xb in ((n_lo, n_lo), (5, 6), (6, 5), (8, n_lo)):
        print("w_row_bits", wb, "x_row_bits", xb, kind, flush=True)
        with api.Handle(0) as h:
            api.qst_plan_choice(h, inst, path=path, set_to={"kind": 0, "settings_per_batch": 16, "w_row_bits": wb,
                                                           "x_row_bits": xb})
            probs, _ = api.qst_forward(h, [inst], want_probs=True, path=path)
            got = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=path)
            torch.cuda.synchronize()
            out = (probs[0].cpu(), float(got[0][0]), got[1][0].cpu(), got[2][0].cpu())
        if ref is None:
            ref = out
            continue
        assert torch.equal(out[0], ref[0]) and out[1] == ref[1], wb
        assert torch.equal(out[2], ref[2]) and torch.equal(out[3], ref[3]), wb
