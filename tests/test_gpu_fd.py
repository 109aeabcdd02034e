"""Central finite-difference check of both gradients at the n=10, R=4, B=200 workload
(eqs. atom-wirtinger-gradient and weight-gradient), on the FP64 path (whole state on chip):
along random directions, [L(x + h d) - L(x - h d)] / 2h from the library's own loss must
equal the directional derivative of its gradient, 2 Re <dL/dpsi^*, d> for atoms and
<dL/dalpha, d> for weights, to about 1e-7 relative (the FD truncation and rounding error
at h = 1e-5 in FP64).  The gradients themselves are compared with the oracle too."""
import numpy as np
import pytest
import torch

from oracle import born
from tests._cases import close, make_case, oracle, rel, to_device

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def h():
    from paper_2607_19577_amd import api

    with api.Handle(0) as hd:
        yield hd


@pytest.mark.parametrize("kind", [born.LOSS_CE, born.LOSS_LS])
def test_central_fd_n10_r4_b200_fp64(h, kind):
    from paper_2607_19577_amd import api

    print("fd: n=10 R=4 B=200 FP64 kind", kind, flush=True)
    case = make_case(1101, 10, 4, 200, shots=10_000, complex_dtype=np.complex128, R_true=4)
    inst = to_device(case, DEV)
    path = api.PATH_BUTTERFLY_F64
    lt, ag, wg = api.qst_backward(h, [inst], loss=kind, eps=1e-8, path=path)
    torch.cuda.synchronize()
    ga, gw = ag[0].cpu().numpy(), wg[0].cpu().numpy()
    Lr, _, gar, gwr = oracle(case, kind, 1e-8, tier="axis")
    assert abs(float(lt[0]) - Lr) <= 1e-12 * abs(Lr)
    for r in range(4):
        assert close(ga[r], gar[r], 1e-12), (r, rel(ga[r], gar[r]))
    assert close(gw, gwr, 1e-12)

    def loss_at(atoms, w):
        x = api.Instance(torch.from_numpy(atoms).to(DEV), torch.from_numpy(w).to(DEV), inst.settings, inst.freqs)
        _, lv = api.qst_forward(h, [x], want_probs=False, loss=kind, eps=1e-8, path=path)
        return float(lv[0])

    rng = np.random.default_rng(1102)
    step = 1e-5
    atoms, w = case["atoms"], case["weights"]
    for _ in range(3):
        d = rng.standard_normal(atoms.shape) + 1j * rng.standard_normal(atoms.shape)
        d /= np.linalg.norm(d)
        fd = (loss_at(atoms + step * d, w) - loss_at(atoms - step * d, w)) / (2 * step)
        an = 2.0 * float(np.sum(np.real(np.conj(ga) * d)))
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)
        dw = rng.standard_normal(w.shape)
        dw /= np.linalg.norm(dw)
        fd = (loss_at(atoms, w + step * dw) - loss_at(atoms, w - step * dw)) / (2 * step)
        an = float(np.dot(gw, dw))
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)
