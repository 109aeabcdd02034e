"""Tensor-level binding of the C ABI (same names as include/qst.h).

PyTorch supplies device memory and the stream; these functions only check
dtypes/shapes, pass raw pointers and allocate the outputs.  All arithmetic of
the hot path runs in ``libqst.so``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (LOSS_CE, LOSS_LS, LOSS_NONE, PATH_AUTO, PATH_BUTTERFLY_BF16, PATH_BUTTERFLY_F32,
                   PATH_BUTTERFLY_F64, PATH_PLAIN_F32, PATH_TILE_BF16, PATH_TILE_F16, QSTError, QstChoice,
                   QstInstance, QstSolveParams)

__all__ = [
    "Handle", "Instance", "qst_forward", "qst_backward", "qst_backward_static", "qst_atom_trial", "qst_reweight_simplex", "qst_refactor",
    "qst_plan", "qst_plan_choice", "qst_solve", "qst_state_error", "SolveParams",
    "LOSS_CE", "LOSS_LS", "LOSS_NONE", "PATH_AUTO", "PATH_BUTTERFLY_F32", "PATH_BUTTERFLY_F64", "PATH_PLAIN_F32",
    "PATH_TILE_F16", "PATH_TILE_BF16", "PATH_BUTTERFLY_BF16", "QSTError",
]

_C_OF_PATH = {
    PATH_AUTO: torch.complex64, PATH_BUTTERFLY_F32: torch.complex64, PATH_BUTTERFLY_F64: torch.complex128,
    PATH_PLAIN_F32: torch.complex64, PATH_TILE_F16: torch.complex64, PATH_TILE_BF16: torch.complex64,
    PATH_BUTTERFLY_BF16: torch.complex64,
}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Handle:
    """Owns a ``qst_handle`` bound to one device and stream (``device=-1``: validation only)."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        if device >= 0:
            s = stream if stream is not None else torch.cuda.current_stream(device)
            sp = ctypes.c_void_p(s.cuda_stream)
        else:
            sp = None
        _lib.check(self.lib.qst_create(device, sp, ctypes.byref(h)))
        self.h = h

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        _lib.check(self.lib.qst_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), self.h)

    def profile(self, enable: bool = True) -> None:
        _lib.check(self.lib.qst_profile_enable(self.h, int(enable)), self.h)

    STAGES = ("decode", "hi_fwd", "lo_fused", "hi_adj", "reduce", "other", "gv", "mid")

    def profile_read(self, reset: bool = True) -> dict:
        """{stage: (launches, total_ms)} since the last reset (synchronises the stream)."""
        out = {}
        for k, name in enumerate(self.STAGES):
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            _lib.check(self.lib.qst_profile_read(self.h, k, ctypes.byref(n), ctypes.byref(ms), 0), self.h)
            out[name] = (int(n.value), float(ms.value))
        if reset:
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            _lib.check(self.lib.qst_profile_read(self.h, 0, ctypes.byref(n), ctypes.byref(ms), 1), self.h)
        return out

    def close(self) -> None:
        if self.h:
            self.lib.qst_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Instance:
    """One tomography instance: atoms [R][D] complex, weights [R] float64,
    settings [B][N] uint8 (X=0, Y=1, Z=2), freqs [B][D] float32 (optional),
    probs_base [B][D] of the path's real type (optional: p = probs_base + the atoms' part),
    unitaries [K][2][2] complex128 (optional: settings codes c >= 3 apply unitaries[c - 3]),
    freqs_csr (rowptr int64 [B+1], index int32 [nnz], values float32 [nnz]) in place of freqs for
    sparse frequencies."""

    atoms: torch.Tensor
    weights: torch.Tensor
    settings: torch.Tensor
    freqs: Optional[torch.Tensor] = None
    settings_per_batch: int = 0  # 0: library default
    probs_base: Optional[torch.Tensor] = None
    unitaries: Optional[torch.Tensor] = None
    freqs_csr: Optional[tuple] = None

    @property
    def shape(self):
        B, N = self.settings.shape
        return N, self.atoms.shape[0], B

    def c_struct(self, path: int) -> QstInstance:
        N, R, B = self.shape
        want = _C_OF_PATH[path]
        if self.atoms.dtype != want:
            raise TypeError(f"atoms must be {want} for path {path}, got {self.atoms.dtype}")
        if self.weights.dtype != torch.float64 or self.settings.dtype != torch.uint8:
            raise TypeError("weights must be float64 and settings uint8")
        if self.freqs is not None and self.freqs.dtype != torch.float32:
            raise TypeError("freqs must be float32")
        for t in (self.atoms, self.weights, self.settings, self.freqs):
            if t is not None and not t.is_contiguous():
                raise ValueError("all tensors must be contiguous")
        if self.atoms.dim() != 2 or self.atoms.shape[1] != (1 << N) or self.weights.shape != (R,):
            raise ValueError("atoms must be [R][2^N] and weights [R]")
        if self.freqs is not None and tuple(self.freqs.shape) != (B, 1 << N):
            raise ValueError("freqs must be [B][2^N]")
        csr = self.freqs_csr
        if csr is not None:
            if self.freqs is not None:
                raise ValueError("give freqs or freqs_csr, not both")
            rp, ix, vals = csr
            if (rp.dtype != torch.int64 or ix.dtype != torch.int32 or vals.dtype != torch.float32
                    or rp.shape != (B + 1,) or ix.dim() != 1 or vals.shape != ix.shape
                    or not (rp.is_contiguous() and ix.is_contiguous() and vals.is_contiguous())):
                raise ValueError("freqs_csr must be (rowptr int64 [B+1], index int32 [nnz], values float32 [nnz])")
        pb = self.probs_base
        if pb is not None and (pb.dtype != _real_of(path) or not pb.is_contiguous() or tuple(pb.shape) != (B, 1 << N)):
            raise ValueError("probs_base must be contiguous [B][2^N] of the path's real type")
        u = self.unitaries
        if u is not None and (u.dtype != torch.complex128 or not u.is_contiguous() or u.dim() != 3
                              or tuple(u.shape[1:]) != (2, 2)):
            raise ValueError("unitaries must be contiguous [K][2][2] complex128")
        fptr = self.freqs.data_ptr() if self.freqs is not None else (csr[2].data_ptr() if csr is not None else None)
        return QstInstance(N, R, B, int(self.settings_per_batch), self.atoms.data_ptr(), self.weights.data_ptr(),
                           self.settings.data_ptr(), fptr,
                           None if pb is None else pb.data_ptr(),
                           None if u is None else u.data_ptr(),
                           None if csr is None else csr[0].data_ptr(), None if csr is None else csr[1].data_ptr(),
                           0 if csr is None else int(csr[1].numel()),
                           0 if u is None else int(u.shape[0]))


def _structs(insts: Sequence[Instance], path: int):
    arr = (QstInstance * len(insts))()
    for i, inst in enumerate(insts):
        arr[i] = inst.c_struct(path)
    return arr


def _real_of(path: int):
    return torch.float64 if path == PATH_BUTTERFLY_F64 else torch.float32


def qst_plan(h: Handle, insts: Sequence[Instance], path: int = PATH_AUTO, autotune: bool = False) -> None:
    arr = _structs(insts, path)
    _lib.check(h.lib.qst_plan(h.h, arr, len(insts), path, int(autotune)), h.h)


CHOICE_FIELDS = ("kind", "settings_per_batch", "tile_bits_fwd", "tile_bits_adj", "values_per_thread_log2", "w_row_bits",
                 "x_row_bits", "tuned", "best_ms", "default_ms")


def qst_plan_choice(h: Handle, inst: Instance, path: int = PATH_AUTO, set_to: Optional[dict] = None) -> dict:
    """The implementation choice for the shape of ``inst`` (a dict of ``CHOICE_FIELDS``); with
    ``set_to`` the given fields are pinned first (missing ones take the defaults)."""
    arr = _structs([inst], path)
    c = QstChoice()
    c.kind = -1
    if set_to is not None:
        for k, v in set_to.items():
            setattr(c, k, v)
        _lib.check(h.lib.qst_plan_choice(h.h, arr, path, 1, ctypes.byref(c)), h.h)
    _lib.check(h.lib.qst_plan_choice(h.h, arr, path, 0, ctypes.byref(c)), h.h)
    return {k: getattr(c, k) for k in CHOICE_FIELDS}


def qst_forward(h: Handle, insts: Sequence[Instance], want_probs: bool = True, loss: int = LOSS_NONE,
                eps: float = 1e-8, path: int = PATH_AUTO):
    """Returns ``(probs list or None, loss tensor [n] float64 or None)``."""
    arr = _structs(insts, path)
    dev = insts[0].atoms.device
    probs = None
    pp = None
    if want_probs:
        probs = [torch.empty((i.shape[2], 1 << i.shape[0]), dtype=_real_of(path), device=dev) for i in insts]
        pp = (ctypes.c_void_p * len(insts))(*[p.data_ptr() for p in probs])
    lt = torch.empty(len(insts), dtype=torch.float64, device=dev) if loss != LOSS_NONE else None
    _lib.check(h.lib.qst_forward(h.h, arr, len(insts), pp, _ptr(lt), loss, float(eps), path), h.h)
    return probs, lt


def qst_backward(h: Handle, insts: Sequence[Instance], grad_p: Optional[Sequence[torch.Tensor]] = None,
                 loss: int = LOSS_CE, eps: float = 1e-8, project_tangent: bool = False, path: int = PATH_AUTO,
                 want_loss: bool = True, out: Optional[List[torch.Tensor]] = None, _entry: str = "qst_backward"):
    """Fused forward + adjoint.  Returns ``(loss [n] float64 or None, atom_grads, weight_grads)``."""
    arr = _structs(insts, path)
    n = len(insts)
    dev = insts[0].atoms.device
    ag = out if out is not None else [torch.empty_like(i.atoms) for i in insts]
    wg = [torch.empty(i.shape[1], dtype=torch.float64, device=dev) for i in insts]
    agp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ag])
    wgp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in wg])
    gpp = None
    if grad_p is not None:
        for g, i in zip(grad_p, insts):
            if g.dtype != _real_of(path) or not g.is_contiguous() or tuple(g.shape) != (i.shape[2], 1 << i.shape[0]):
                raise ValueError("grad_p must be contiguous [B][D] of the path's real type")
        gpp = (ctypes.c_void_p * n)(*[g.data_ptr() for g in grad_p])
        loss = LOSS_NONE
        want_loss = False
    lt = torch.empty(n, dtype=torch.float64, device=dev) if want_loss else None
    _lib.check(getattr(h.lib, _entry)(h.h, arr, n, gpp, agp, wgp, _ptr(lt), loss, float(eps), int(project_tangent),
                                      path), h.h)
    return lt, ag, wg


def qst_backward_static(h: Handle, insts: Sequence[Instance], grad_p: Optional[Sequence[torch.Tensor]] = None,
                        loss: int = LOSS_CE, eps: float = 1e-8, project_tangent: bool = False, path: int = PATH_AUTO,
                        want_loss: bool = True, out: Optional[List[torch.Tensor]] = None):
    """``qst_backward`` through the no-allocation entry point (the library's scratch is a fixed
    64 MiB device array per GPU; calls that need more raise QST_ERR_SHAPE).  The outputs are
    allocated here unless ``out`` is given; the library itself allocates nothing."""
    return qst_backward(h, insts, grad_p, loss, eps, project_tangent, path, want_loss, out,
                        _entry="qst_backward_static")


def qst_atom_trial(h: Handle, inst: Instance, r: int, psi_trial: torch.Tensor, probs_t: Optional[torch.Tensor],
                   want_probs: bool = True, loss: int = LOSS_NONE, eps: float = 1e-8, path: int = PATH_AUTO):
    """Response of the atom step: ``p~ = p_t + alpha_r (a(psi_trial) - a(psi_r))`` and the loss
    at ``p~``.  Returns ``(probs [B][D] or None, loss [1] float64 or None)``."""
    arr = _structs([inst], path)
    N, R, B = inst.shape
    dev = inst.atoms.device
    if psi_trial.dtype != inst.atoms.dtype or not psi_trial.is_contiguous() or psi_trial.numel() != (1 << N):
        raise ValueError("psi_trial must be a contiguous [D] vector of the atoms' dtype")
    if probs_t is not None and (probs_t.dtype != _real_of(path) or not probs_t.is_contiguous()
                                or tuple(probs_t.shape) != (B, 1 << N)):
        raise ValueError("probs_t must be contiguous [B][D] of the path's real type")
    out = torch.empty((B, 1 << N), dtype=_real_of(path), device=dev) if want_probs else None
    lt = torch.empty(1, dtype=torch.float64, device=dev) if loss != LOSS_NONE else None
    _lib.check(h.lib.qst_atom_trial(h.h, arr, int(r), _ptr(psi_trial), _ptr(probs_t), _ptr(out), _ptr(lt), loss,
                                    float(eps), path), h.h)
    return out, lt


def qst_reweight_simplex(h: Handle, alpha: torch.Tensor, hvec: torch.Tensor, eta: float, tau: float):
    """Coefficient step + pruning on the device.  Returns ``(alpha_out [R], keep_idx [R], R_out [1])``."""
    R = alpha.numel()
    out = torch.empty(R, dtype=torch.float64, device=alpha.device)
    keep = torch.empty(R, dtype=torch.int32, device=alpha.device)
    rout = torch.empty(1, dtype=torch.int32, device=alpha.device)
    _lib.check(h.lib.qst_reweight_simplex(h.h, _ptr(alpha), _ptr(hvec), R, float(eta), float(tau), _ptr(out),
                                          _ptr(keep), _ptr(rout)), h.h)
    return out, keep, rout


def qst_refactor(h: Handle, inst: Instance, loss: int, eps: float, eta_rho: float, mu: float, tau: float, L_max: int,
                 n_lanczos: int, v0: torch.Tensor, path: int = PATH_AUTO):
    """Spectral refactorisation (host-orchestrated Lanczos).  Returns a dict of device tensors."""
    arr = _structs([inst], path)
    dev = inst.atoms.device
    D = inst.atoms.shape[1]
    if v0.dtype != torch.complex128 or v0.numel() != D:
        raise ValueError("v0 must be complex128 [D]")
    atoms_out = torch.empty((L_max, D), dtype=inst.atoms.dtype, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    w_out, rv, rr, qs = (torch.empty(L_max, **f64) for _ in range(4))
    r_out = torch.empty(1, dtype=torch.int32, device=dev)
    s_star = torch.empty(1, dtype=torch.int32, device=dev)
    _lib.check(h.lib.qst_refactor(h.h, arr, loss, float(eps), float(eta_rho), float(mu), float(tau), int(L_max),
                                  int(n_lanczos), _ptr(v0), _ptr(atoms_out), _ptr(w_out), _ptr(r_out), _ptr(s_star),
                                  _ptr(rv), _ptr(rr), _ptr(qs), path), h.h)
    return dict(atoms=atoms_out, weights=w_out, R=r_out, s_star=s_star, ritz_vals=rv, ritz_resid=rr, q_scores=qs)


@dataclass
class SolveParams:
    """Parameters of the rank-adaptive iteration; defaults of the paper's Table sim-parameters."""

    max_slots: int = 1000
    t_alpha: int = 5
    t_ref: int = 50
    n_grid: int = 11
    rank_max: int = 8
    n_lanczos: int = 30
    stop_window: int = 20
    loss_kind: int = LOSS_CE
    stop_delta: float = 1e-4
    mu: float = 1e-3
    eps: float = 1e-8
    tau: float = 1e-3
    tau_acc: float = 1e-10
    oracle_budget: int = 100_000

    def c_struct(self) -> QstSolveParams:
        return QstSolveParams(self.max_slots, self.t_alpha, self.t_ref, self.n_grid, self.rank_max, self.n_lanczos,
                              self.stop_window, self.loss_kind, self.stop_delta, self.mu, self.eps, self.tau,
                              self.tau_acc, self.oracle_budget)


def qst_solve(h: Handle, inst: Instance, params: SolveParams, v0s: Optional[torch.Tensor] = None,
              path: int = PATH_AUTO) -> dict:
    """Rank-adaptive iteration from the state in ``inst``.  ``v0s`` [n_v0][D] complex128 holds the Lanczos
    start vectors.  Returns a dict: atoms [R][D], weights [R], rank, history [slots][6] (numpy), slots,
    oracle_calls, stopped ('slots', 'delta' or 'budget')."""
    import numpy as np

    arr = _structs([inst], path)
    N, R, B = inst.shape
    dev = inst.atoms.device
    if v0s is not None and (v0s.dtype != torch.complex128 or not v0s.is_contiguous() or v0s.dim() != 2
                            or v0s.shape[1] != (1 << N)):
        raise ValueError("v0s must be contiguous [n_v0][D] complex128")
    cap = params.rank_max
    atoms = torch.zeros((cap, 1 << N), dtype=inst.atoms.dtype, device=dev)
    w = torch.zeros(cap, dtype=torch.float64, device=dev)
    rank = ctypes.c_int32(0)
    hist = np.zeros((max(params.max_slots, 1), 6), dtype=np.float64)
    info = np.zeros(3, dtype=np.int64)
    prm = params.c_struct()
    n_v0 = 0 if v0s is None else int(v0s.shape[0])
    _lib.check(h.lib.qst_solve(h.h, arr, ctypes.byref(prm), _ptr(v0s), n_v0, _ptr(atoms), _ptr(w),
                               ctypes.byref(rank), hist.ctypes.data_as(ctypes.c_void_p),
                               info.ctypes.data_as(ctypes.c_void_p), path), h.h)
    Rf = int(rank.value)
    slots = int(info[0])
    return dict(atoms=atoms[:Rf], weights=w[:Rf], rank=Rf, history=hist[:slots], slots=slots,
                oracle_calls=int(info[1]), stopped=("slots", "delta", "budget")[int(info[2])])


def qst_state_error(h: Handle, atoms_a: torch.Tensor, w_a: torch.Tensor, atoms_b: torch.Tensor, w_b: torch.Tensor,
                    path: int = PATH_AUTO) -> float:
    """``||rho_a - rho_b||_F / ||rho_b||_F`` of two atomic states (Gram form, on the device)."""
    D = atoms_a.shape[1]
    n = D.bit_length() - 1
    for t in (atoms_a, w_a, atoms_b, w_b):
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
    if atoms_a.dtype != _C_OF_PATH[path] or atoms_b.dtype != _C_OF_PATH[path] or atoms_b.shape[1] != D:
        raise ValueError("atoms must be [R][D] of the path's complex type")
    out = ctypes.c_double(0.0)
    _lib.check(h.lib.qst_state_error(h.h, n, _ptr(atoms_a), _ptr(w_a), atoms_a.shape[0], _ptr(atoms_b), _ptr(w_b),
                                     atoms_b.shape[0], ctypes.byref(out), path), h.h)
    return float(out.value)
