"""The no-allocation backward (qst_backward_static, whose scratch is a fixed device array)
against qst_backward through the C ABI: two calls in a row, the second smaller, each equal
to qst_backward's results bit for bit (same kernels and batch sizes), and a call that needs
more scratch than the array holds is refused before anything runs."""
import numpy as np
import pytest
import torch

import synth
from paper_2607_19577_amd import api


def _inst(seed, n, R, B, S=0, dev="cuda:0"):
    rng = synth.make_rng(seed)
    D = 1 << n
    atoms = torch.from_numpy(synth.haar_atoms(rng, R, D, dtype=np.complex64)).to(dev)
    w = torch.from_numpy(synth.dirichlet_weights(rng, R)).to(dev)
    s = torch.from_numpy(synth.random_settings(rng, B, n)).to(dev)
    f = synth.porter_thomas_freqs_torch(seed + 1, B, D, synth.dirichlet_weights(rng, 2), 10_000, torch.device(dev))
    return api.Instance(atoms, w, s, f, settings_per_batch=S)


def _both(h, insts, tangent):
    ref = api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=tangent)
    got = api.qst_backward_static(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=tangent)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got):
    assert torch.equal(ref[0], got[0])
    for a, b in zip(ref[1], got[1]):
        assert torch.equal(a, b)
    for a, b in zip(ref[2], got[2]):
        assert torch.equal(a, b)


@pytest.mark.gpu
def test_static_backward_equals_backward_twice_then_refuses_oversize():
    print("no-alloc: staged n=15 R=6 B=24 S=8 with one-chunk n=9 R=3 B=20, then n=10 R=2 B=7", flush=True)
    with api.Handle(0) as h:
        big = [_inst(501, 15, 6, 24, S=8), _inst(502, 9, 3, 20), _inst(503, 9, 5, 13)]
        ref, got = _both(h, big, tangent=True)
        _same(ref, got)
        # the second call is smaller: the scratch keeps the first call's contents, which must not leak in
        small = [_inst(504, 10, 2, 7)]
        ref, got = _both(h, small, tangent=False)
        _same(ref, got)
        # a shape whose one setting of intermediates exceeds the array is refused, nothing enqueued
        n = 20
        huge = api.Instance(torch.zeros((16, 1 << n), dtype=torch.complex64, device="cuda:0"),
                            torch.full((16,), 1 / 16, dtype=torch.float64, device="cuda:0"),
                            torch.zeros((2, n), dtype=torch.uint8, device="cuda:0"),
                            torch.zeros((2, 1 << n), dtype=torch.float32, device="cuda:0"))
        with pytest.raises(api.QSTError) as e:
            api.qst_backward_static(h, [huge], loss=api.LOSS_CE)
        assert e.value.status == 2 and "bytes of scratch" in str(e.value)
        # the handle still works after the refusal
        ref, got = _both(h, small, tangent=True)
        _same(ref, got)
