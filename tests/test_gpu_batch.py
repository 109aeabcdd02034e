"""GPU parity of multi-instance calls: instances of uneven n, R and B run as one launch
of each pass per class of equal n (any number of instances, from one instance table in
device memory), mixed with instances that take the staged path one by one.

* every instance of a batched call matches the FP64 oracle (1e-5, FP32 path);
* a batched call matches one-at-a-time calls: probabilities bit for bit, loss and weight
  gradient to 1e-12 (FP64 sums of per-item partials), atom gradients to 1e-6 norm-wise
  (FP32 sums over slices of settings whose size follows the launch's total work; 1e-5 after
  the tangent projection);
* the uneven 64-instance workload (n in 6..12, R in 1..8, B in 50..500) against
  one-at-a-time calls, and captured in a graph and replayed.
"""
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


def _shapes():
    rng = synth.make_rng(811)
    shapes = [(5, int(rng.integers(1, 9)), int(rng.integers(3, 13))) for _ in range(17)]  # 16 + 1 in one group
    shapes += [(7, int(rng.integers(1, 9)), int(rng.integers(3, 13))) for _ in range(3)]
    shapes += [(13, 3, 4)]  # high bits: staged path inside the same call
    return shapes


@pytest.fixture(scope="module")
def uneven():
    return [make_case(820 + i, n, R, B, shots=5000) for i, (n, R, B) in enumerate(_shapes())]


@pytest.mark.parametrize("tangent", [False, True])
def test_batched_call_matches_oracle(h, uneven, tangent):
    from paper_2607_19577_amd import api

    insts = [to_device(c, DEV) for c in uneven]
    lt, ag, wg = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=tangent)
    torch.cuda.synchronize()
    for i, c in enumerate(uneven):
        Lr, _, gar, gwr = oracle(c, born.LOSS_CE, 1e-8)
        if tangent:
            gar = born.tangent_project(c["atoms"].astype(np.complex128), gar)
        assert abs(float(lt[i]) - Lr) <= 1e-5 * abs(Lr), (i, float(lt[i]), Lr)
        g = ag[i].cpu().numpy()
        for r in range(g.shape[0]):
            assert close(g[r], gar[r], 1e-5), (i, r, rel(g[r], gar[r]))
        assert close(wg[i].cpu().numpy(), gwr, 1e-5), (i, rel(wg[i].cpu().numpy(), gwr))


def test_batched_call_matches_single_calls(h, uneven):
    from paper_2607_19577_amd import api

    insts = [to_device(c, DEV) for c in uneven]
    probs, lf = api.qst_forward(h, insts, want_probs=True, loss=api.LOSS_LS, eps=0.0)
    lt, ag, wg = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8)
    for i, inst in enumerate(insts):
        p1, l1f = api.qst_forward(h, [inst], want_probs=True, loss=api.LOSS_LS, eps=0.0)
        l1, a1, w1 = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8)
        assert torch.equal(probs[i], p1[0]), i
        assert rel(ag[i].cpu().numpy(), a1[0].cpu().numpy()) <= 1e-6, i
        assert abs(float(lf[i]) - float(l1f[0])) <= 1e-12 * abs(float(l1f[0])), i
        assert abs(float(lt[i]) - float(l1[0])) <= 1e-12 * abs(float(l1[0])), i
        torch.testing.assert_close(wg[i], w1[0], rtol=1e-12, atol=1e-300)


def test_batched_generic_sensitivity(h, uneven):
    """The autograd route (caller's dL/dp) through a batched call equals single calls."""
    from paper_2607_19577_amd import api

    insts = [to_device(c, DEV) for c in uneven[:6]]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(5)
    gps = [torch.randn((c.settings.shape[0], 1 << c.settings.shape[1]), generator=gen, device=DEV) for c in insts]
    _, ag, wg = api.qst_backward(h, insts, grad_p=gps)
    for i, inst in enumerate(insts):
        _, a1, w1 = api.qst_backward(h, [inst], grad_p=[gps[i]])
        assert rel(ag[i].cpu().numpy(), a1[0].cpu().numpy()) <= 1e-6, i
        torch.testing.assert_close(wg[i], w1[0], rtol=1e-12, atol=1e-300)


@pytest.fixture(scope="module")
def uneven64():
    rng = synth.make_rng(4004)
    out = []
    for k, sh in enumerate(synth.uneven_batch_shapes(rng, 64)):
        n, R, B = sh["n"], sh["R"], sh["B"]
        r = synth.make_rng(5000 + k)
        atoms = synth.haar_atoms(r, R, 1 << n, dtype=np.complex64)
        w = synth.dirichlet_weights(r, R)
        s = synth.random_settings(r, B, n)
        f = synth.porter_thomas_freqs(r, B, 1 << n, synth.dirichlet_weights(r, min(R, 4)), 10_000)
        out.append(dict(atoms=atoms, weights=w, settings=s, freqs=f))
    return out


def test_uneven64_batched_matches_single(h, uneven64):
    from paper_2607_19577_amd import api

    insts = [to_device(c, DEV) for c in uneven64]
    lt, ag, wg = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
    for i, inst in enumerate(insts):
        l1, a1, w1 = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
        assert abs(float(lt[i]) - float(l1[0])) <= 1e-12 * abs(float(l1[0])), i
        torch.testing.assert_close(wg[i], w1[0], rtol=1e-12, atol=1e-300)
        # the settings are summed in slices whose size follows the launch's total work; after the
        # tangent projection removes most of each gradient, the FP32 bar (1e-5) applies
        for r in range(ag[i].shape[0]):
            assert rel(ag[i][r].cpu().numpy(), a1[0][r].cpu().numpy()) <= 1e-5, (i, r)


def test_uneven64_graph_replay(h, uneven64):
    from paper_2607_19577_amd import api

    insts = [to_device(c, DEV) for c in uneven64]
    api.qst_plan(h, insts)
    ref = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
    ref = [ref[0].clone()] + [[t.clone() for t in ref[1]], [t.clone() for t in ref[2]]]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        h.set_stream(side)
        api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
    h.set_stream(torch.cuda.current_stream())
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.set_stream(torch.cuda.current_stream())
        out = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)
    h.set_stream(torch.cuda.current_stream())
    for rep in range(3):
        api.qst_forward(h, insts[:3], want_probs=True)
        torch.cuda.synchronize()
        out[0].zero_()
        for t in out[1] + out[2]:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]), rep
        for a, b in zip(out[1], ref[1]):
            assert torch.equal(a, b), rep
        for a, b in zip(out[2], ref[2]):
            assert torch.equal(a, b), rep
