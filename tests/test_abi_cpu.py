"""The C-ABI library loads on a CPU host, exports every entry point that
include/qst.h declares, and its argument validation behaves as documented
(validation-only handle: nothing is launched)."""
import ctypes
import os
import re

import pytest

from paper_2607_19577_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qst_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqst.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_exports_match_header(lib):
    declared = _declared()
    assert set(declared) == set(_lib.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_static_strings(lib):
    assert lib.qst_status_string(0) == b"ok"
    assert b"gfx950" in lib.qst_build_info()
    for s in range(9):
        assert lib.qst_status_string(s)


def _vh(lib):
    h = ctypes.c_void_p()
    assert lib.qst_create(-1, None, ctypes.byref(h)) == 0
    return h


def _inst(n=10, R=4, B=3, atoms=0x1000, weights=0x2000, settings=0x3000, freqs=0x4000):
    return _lib.QstInstance(n, R, B, 0, atoms, weights, settings, freqs)


def test_validation_paths(lib):
    h = _vh(lib)
    try:
        one = (_lib.QstInstance * 1)(_inst())
        ok_args = dict(loss=_lib.LOSS_CE, eps=1e-8, path=_lib.PATH_AUTO)
        # valid arguments on a validation-only handle stop before any launch
        assert lib.qst_forward(h, one, 1, None, ctypes.c_void_p(0x5000), _lib.LOSS_CE, 1e-8, 0) == 4
        # shape errors
        neg = _inst()
        neg.settings_per_batch = -1
        for bad in (_inst(n=0), _inst(n=31), _inst(R=0), _inst(R=257), _inst(B=0), neg,
                    _inst(n=26, R=16), _inst(n=30, R=1)):  # the last two: one setting's vectors >= 4 GiB
            arr = (_lib.QstInstance * 1)(bad)
            assert lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, 0) == 2
        # shapes the staged passes take: two passes (n=20, R=16), three (n=21, R=16;
        # n=24, R=16; n=20, R=17; n=28, R=1) and the largest rank (n=18, R=256); they stop at the device gate
        for okshape in ((20, 16), (21, 16), (24, 16), (20, 17), (28, 1), (18, 256), (14, 256), (6, 256)):
            arr = (_lib.QstInstance * 1)(_inst(n=okshape[0], R=okshape[1]))
            assert lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, 0) == 4, okshape
            assert b"device" in lib.qst_last_error(h).lower(), (okshape, lib.qst_last_error(h))
        # a rank above 2^(14-n) below 14 qubits has no staged shape: n = 11..13 runs on chip (FP32
        # Pauli settings, dense frequencies), n = 10 not at all
        for path, shape, ok in ((_lib.PATH_BUTTERFLY_F32, (12, 40), True), (_lib.PATH_BUTTERFLY_BF16, (12, 40), False),
                                (_lib.PATH_BUTTERFLY_F32, (10, 32), False), (_lib.PATH_BUTTERFLY_BF16, (10, 32), False)):
            arr = (_lib.QstInstance * 1)(_inst(n=shape[0], R=shape[1], atoms=0x10000, freqs=0x20000))
            assert lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, path) == 4
            msg = lib.qst_last_error(h)
            assert (b"device" in msg.lower()) if ok else (b"tile-stage shapes" in msg), (path, shape, msg)
        # the plain and tile paths stop at n = 20, R = 16
        for bad in (_inst(n=21, R=4), _inst(n=12, R=32)):
            arr = (_lib.QstInstance * 1)(bad)
            assert lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, _lib.PATH_PLAIN_F32) == 4
            assert b"plain and tile" in lib.qst_last_error(h)
        # null pointers
        for bad in (_inst(atoms=0), _inst(weights=0), _inst(settings=0)):
            arr = (_lib.QstInstance * 1)(bad)
            assert lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, 0) == 1
        assert lib.qst_forward(h, one, 0, None, None, 2, 0.0, 0) == 1
        assert lib.qst_forward(None, one, 1, None, None, 2, 0.0, 0) == 1
        # loss without freqs, bad enums, bad eps
        arr = (_lib.QstInstance * 1)(_inst(freqs=0))
        assert lib.qst_forward(h, arr, 1, None, ctypes.c_void_p(0x5000), _lib.LOSS_CE, 1e-8, 0) == 1
        assert lib.qst_forward(h, one, 1, None, None, 7, 1e-8, 0) == 1
        assert lib.qst_forward(h, one, 1, None, None, 0, -1.0, 0) == 1
        assert lib.qst_forward(h, one, 1, None, None, 0, float("nan"), 0) == 1
        assert lib.qst_forward(h, one, 1, None, None, 0, 1e-8, 99) == 1
        # misaligned atoms
        arr = (_lib.QstInstance * 1)(_inst(atoms=0x1004))
        assert lib.qst_forward(h, arr, 1, None, None, 2, 0.0, 0) == 3
        # backward: needs atom_grad, exclusive grad_p / loss
        grads = (ctypes.c_void_p * 1)(0x6000)
        gp = (ctypes.c_void_p * 1)(0x7000)
        assert lib.qst_backward(h, one, 1, None, None, None, None, 0, 1e-8, 0, 0) == 1
        assert lib.qst_backward(h, one, 1, gp, grads, None, None, _lib.LOSS_CE, 1e-8, 0, 0) == 1
        assert lib.qst_backward(h, one, 1, None, grads, None, None, _lib.LOSS_NONE, 1e-8, 0, 0) == 1
        assert lib.qst_backward(h, one, 1, gp, grads, None, None, _lib.LOSS_NONE, 0.0, 0, 0) == 4
        alias = (ctypes.c_void_p * 1)(0x1000)
        assert lib.qst_backward(h, one, 1, None, alias, None, None, 0, 1e-8, 0, 0) == 1
        # FP64 path: whole state on chip only
        big = (_lib.QstInstance * 1)(_inst(n=14, R=4, atoms=0x10000))
        assert lib.qst_forward(h, big, 1, None, None, 2, 0.0, _lib.PATH_BUTTERFLY_F64) == 4
        assert b"FP64" in lib.qst_last_error(h)
        # reweight
        assert lib.qst_reweight_simplex(h, None, None, 4, 0.1, 1e-3, None, None, None) == 1
        p = ctypes.c_void_p(0x8000)
        assert lib.qst_reweight_simplex(h, p, p, 0, 0.1, 1e-3, p, p, p) == 2
        assert lib.qst_reweight_simplex(h, p, p, 2000, 0.1, 1e-3, p, p, p) == 2
        assert lib.qst_reweight_simplex(h, p, p, 8, float("inf"), 1e-3, p, p, p) == 1
        assert lib.qst_reweight_simplex(h, p, p, 8, 0.1, 1e-3, p, p, p) == 4
        # refactor
        v = ctypes.c_void_p(0x9000)
        assert lib.qst_refactor(h, one, _lib.LOSS_NONE, 1e-8, 0.5, 1e-3, 1e-3, 8, 30, v, v, v, v, v, v, v, v, 0) == 1
        assert lib.qst_refactor(h, one, _lib.LOSS_CE, 1e-8, 0.0, 1e-3, 1e-3, 8, 30, v, v, v, v, v, v, v, v, 0) == 1
        assert lib.qst_refactor(h, one, _lib.LOSS_CE, 1e-8, 0.5, 1e-3, 1e-3, 0, 30, v, v, v, v, v, v, v, v, 0) == 2
        assert lib.qst_refactor(h, one, _lib.LOSS_CE, 1e-8, 0.5, 1e-3, 1e-3, 8, 30, v, v, v, v, v, v, v, v, 0) == 4
        assert ok_args
    finally:
        assert lib.qst_destroy(h) == 0


def test_create_without_device(lib):
    # On a host without a GPU (or with a bad index) creation fails cleanly.
    h = ctypes.c_void_p()
    rc = lib.qst_create(4096, None, ctypes.byref(h))
    assert rc in (1, 5) and not h.value
    assert lib.qst_destroy(None) == 1


def test_validation_of_general_sparse_trial_and_iteration(lib):
    """Argument checks of the later entry points and instance fields (validation-only handle:
    valid arguments come back as QST_ERR_UNSUPPORTED = 4 before any launch)."""
    h = _vh(lib)
    try:
        def fwd(inst, path=0):
            arr = (_lib.QstInstance * 1)(inst)
            return lib.qst_forward(h, arr, 1, None, None, _lib.LOSS_NONE, 0.0, path)

        # general local settings: table size, alignment, path
        for k, addr, want in ((3, 0x5000, 4), (0, 0x5000, 2), (254, 0x5000, 2), (3, 0x5004, 3)):
            g = _inst()
            g.unitaries, g.n_unitaries = addr, k
            assert fwd(g) == want, (k, addr)
        g = _inst()
        g.unitaries, g.n_unitaries = 0x5000, 3
        assert fwd(g, _lib.PATH_TILE_F16) == 4 and b"general local settings" in lib.qst_last_error(h)
        # sparse frequencies: index and values needed, nnz in 0..B*D, alignment
        B, D = 3, 1 << 10
        for rowptr, index, nnz, want in ((0x6000, 0x7000, 10, 4), (0x6000, 0, 10, 1), (0x6000, 0x7000, -1, 2),
                                         (0x6000, 0x7000, B * D + 1, 2), (0x6004, 0x7000, 10, 3),
                                         (0x6000, 0x7002, 10, 3)):
            sp = _inst()
            sp.freqs_rowptr, sp.freqs_index, sp.freqs_nnz = rowptr, index, nnz
            assert fwd(sp) == want, (rowptr, index, nnz)
        # atom step: atom index, trial vector, aliasing
        one = (_lib.QstInstance * 1)(_inst())
        p = ctypes.c_void_p
        assert lib.qst_atom_trial(h, one, 1, p(0x8000), p(0x9000), p(0xA000), p(0xB000), _lib.LOSS_CE, 1e-8, 0) == 4
        assert lib.qst_atom_trial(h, one, 4, p(0x8000), p(0x9000), None, None, _lib.LOSS_NONE, 0.0, 0) == 1
        assert lib.qst_atom_trial(h, one, -1, p(0x8000), p(0x9000), None, None, _lib.LOSS_NONE, 0.0, 0) == 1
        assert lib.qst_atom_trial(h, one, 0, None, p(0x9000), None, None, _lib.LOSS_NONE, 0.0, 0) == 1
        assert lib.qst_atom_trial(h, one, 0, p(0x8000), p(0x9000), p(0x9000), None, _lib.LOSS_NONE, 0.0, 0) == 1
        assert lib.qst_atom_trial(h, one, 0, p(0x8004), p(0x9000), None, None, _lib.LOSS_NONE, 0.0, 0) == 3
        # the iteration: schedule and stopping parameters, ranks, outputs
        rank = ctypes.c_int32()

        def solve(**kw):
            prm = _lib.QstSolveParams(kw.get("max_slots", 10), kw.get("t_alpha", 5), kw.get("t_ref", 0),
                                      kw.get("n_grid", 11), kw.get("rank_max", 8), 30, 20, _lib.LOSS_CE, 1e-4,
                                      1e-3, 1e-8, 1e-3, 1e-10, 1000)
            return lib.qst_solve(h, one, ctypes.byref(prm), None, 0, p(0xC000), p(0xD000), ctypes.byref(rank),
                                 None, None, 0)

        assert solve() == 4
        assert solve(n_grid=0) == 1
        assert solve(rank_max=17) == 2
        assert solve(rank_max=2) == 2  # initial rank 4 above rank_max
        assert solve(t_ref=10) == 1  # spectral slots without start vectors
        assert solve(max_slots=-1) == 1
        # Gram-form state error
        out = ctypes.c_double()
        assert lib.qst_state_error(h, 10, p(0x1000), p(0x2000), 4, p(0x3000), p(0x4000), 2, ctypes.byref(out), 0) == 4
        assert lib.qst_state_error(h, 0, p(0x1000), p(0x2000), 4, p(0x3000), p(0x4000), 2, ctypes.byref(out), 0) == 2
        assert lib.qst_state_error(h, 10, None, p(0x2000), 4, p(0x3000), p(0x4000), 2, ctypes.byref(out), 0) == 1
        assert lib.qst_state_error(h, 10, p(0x1000), p(0x2000), 0, p(0x3000), p(0x4000), 2, ctypes.byref(out), 0) == 2
    finally:
        assert lib.qst_destroy(h) == 0
