"""Benchmark of the hot path: fused forward map + adjoint on one MI355X.

Workload (default): n = 20 qubits (D = 2^20), R = 16 atoms, B = 2000 random
Pauli settings, 10^6 shots per setting, complex64 atoms, cross-entropy loss.
One step = descriptor decode, the fused forward+adjoint pass (probabilities,
loss, likelihood-ratio sensitivities, weight gradient, atom gradient with the
tangent projection) and the FP64 coefficient step with pruning, with all
inputs resident in HBM.  Metric: forward+adjoint atom-setting amplitudes per
second (B * R * D per step).

Also reported: the roofline of the dominant kernel (algorithmic bytes per
launch over its event-timed duration), a CPU baseline of the FP64 oracle on a
bounded sample of the same workload, the refactorisation time and the speedup
over the plain one-pass-per-qubit reference path.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBPS = 8000.0
WORKLOADS = {
    "n20_r16_b2000": dict(n=20, R=16, B=2000, shots=1_000_000, R_true=4),
    "n14_r8_b1000": dict(n=14, R=8, B=1000, shots=100_000, R_true=4),
    "n10_r4_b200": dict(n=10, R=4, B=200, shots=10_000, R_true=4),
}
KERNEL_SOURCES = ["paper_2607_19577_amd/csrc/qst_stages.hpp", "paper_2607_19577_amd/csrc/qst_device.hpp",
                  "paper_2607_19577_amd/csrc/qst_kernels.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- CPU baseline leg (oracle)
# Everything here runs the FP64 oracle on the host: the timed baseline and the references that
# the GPU results' errors are taken against.  Nothing else in this file imports the oracle.
_CPU = {}


def _cpu_init():
    from threadpoolctl import threadpool_limits

    threadpool_limits(1)


def oracle_reference(atoms, w, s, f):
    """The oracle's CE loss, atom gradient and weight gradient of a small sample instance, the
    reference of the error checks (FP64, on the host)."""
    from oracle import born

    Lr, _, gar, gwr = born.forward_backward(np.asarray(atoms).astype(np.complex128), w, s,
                                            np.asarray(f).astype(np.float64), born.LOSS_CE, 1e-8)
    return Lr, gar, gwr


def _cpu_probs(task):
    from oracle import born

    b, r = task
    return born.probs_axis(_CPU["atoms"][r:r + 1], _CPU["w"][r:r + 1], _CPU["s"], rows=[b])[0]


def _cpu_grads(task):
    from oracle import born

    b, r = task
    ga, gw = born.gradients_axis(_CPU["atoms"][r:r + 1], _CPU["w"][r:r + 1], _CPU["s"], _CPU["g"][[b]], rows=[b])
    return ga[0], float(gw[0])


def host_info() -> dict:
    """CPU model and core counts of the host the oracle runs on, read at run time."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count() or 1, "usable_cpus": usable}


def cpu_baseline(atoms, w, s, B, shots, n_sample: int, seed: int):
    """The FP64 oracle (per-axis tier) on an instance made of the first n_sample settings, all
    atoms: probabilities, loss and sensitivities, then the adjoint, split into (setting, atom)
    calls over a fork pool.  Returns the timing record and the oracle's outputs (frequencies,
    loss, weight and atom gradients) for the error report of the GPU path on the same sample."""
    from oracle import born

    R, D = atoms.shape
    f = synth.porter_thomas_freqs(synth.make_rng(seed), n_sample, D, synth.dirichlet_weights(
        synth.make_rng(seed + 1), 4), shots)
    _CPU.update(atoms=atoms.astype(np.complex128), w=w, s=s[:n_sample])
    tasks = [(b, r) for b in range(n_sample) for r in range(R)]
    host = host_info()
    # the pool covers the usable CPUs, at most 16 processes (the CPU share of one GPU of the
    # host the benchmark runs on)
    cores = max(1, min(16, host["usable_cpus"], len(tasks)))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_cpu_init) as pool:
        parts = pool.map(_cpu_probs, tasks)
        p = np.zeros((n_sample, D))
        for (b, _), q in zip(tasks, parts):
            p[b] += q
        loss, g = born.loss_and_sensitivity(p, f, n_sample, born.LOSS_CE, 1e-8)
        _CPU["g"] = g
    ga = np.zeros((R, D), dtype=np.complex128)
    gw = np.zeros(R)
    with ctx.Pool(cores, initializer=_cpu_init) as pool:
        for (_, r), (a, x) in zip(tasks, pool.imap(_cpu_grads, tasks)):
            ga[r] += a
            gw[r] += x
    dt = time.perf_counter() - t0
    amps = n_sample * R * D
    rec = dict(value=amps / dt, unit="amplitudes/s", cores=cores, kind="oracle", **host,
               sample=f"{n_sample} of {B} settings x {R} atoms x D={D} (an instance of those settings): "
                      f"FP64 per-axis oracle probabilities, CE loss and sensitivities, adjoint; {dt:.1f} s "
                      f"wall on {cores} processes")
    return rec, dict(freqs=f, loss=float(loss), weight_grad=gw, atom_grad=ga)


def _relerr(got, ref) -> float:
    """Norm-wise relative error ||got - ref|| / ||ref||."""
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


# ---------------------------------------------------------------- traffic file
def read_traffic(kernel_kind: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_kind}_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"<!--\s*traffic\s*(\{.*?\})\s*-->", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return float(d["bytes_per_launch"])


def tile_extra(api, h, inst) -> dict:
    """One backward of each MFMA tile path (FP16 and BF16 operands) on the step's instance after a
    warm-up call of each (for profiling the tile passes)."""
    import torch

    grad = torch.empty_like(inst.atoms)
    out = {}
    for name, pth in (("tile_f16", api.PATH_TILE_F16), ("tile_bf16", api.PATH_TILE_BF16)):
        api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=pth, out=[grad])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=pth, out=[grad])
        torch.cuda.synchronize()
        out[f"{name}_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def step_inputs(seed: int, n: int, R: int, B: int, R_true: int):
    """Host inputs of the timed step: model atoms and weights, settings, truth weights."""
    rng = synth.make_rng(seed)
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    w_true = synth.dirichlet_weights(rng, R_true)
    return atoms, w, s, w_true


def step_instance(api, dev, seed: int, n: int, R: int, B: int, shots: int, R_true: int, host=None):
    """The timed step's instance on the device (frequencies drawn on the device)."""
    import torch

    atoms, w, s, w_true = host if host is not None else step_inputs(seed, n, R, B, R_true)
    freqs = synth.porter_thomas_freqs_torch(seed + 3, B, 1 << n, w_true, shots, dev)
    return api.Instance(torch.from_numpy(atoms).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(s).to(dev),
                        freqs)


def refactor_extra(api, h, inst, seed: int) -> dict:
    """The spectral refactor (Lanczos k = 30, L = 8) on the step's instance, with its G v
    products grouped by the settings' high-bit codes (the default) and through the staged
    path (QST_GV_GROUPED=0): wall time of one call after a warm-up call, the mean G v product
    from the library's event brackets, and the agreement of the two runs' Ritz values."""
    import torch

    n = int(inst.settings.shape[1])
    D = 1 << n
    B = int(inst.settings.shape[0])
    v0 = torch.from_numpy(synth.haar_atoms(synth.make_rng(seed), 1, D)[0]).to(inst.atoms.device)
    runs = {}
    old = os.environ.get("QST_GV_GROUPED")
    try:
        for name, flag in (("grouped", "1"), ("staged", "0")):
            os.environ["QST_GV_GROUPED"] = flag
            api.qst_refactor(h, inst, api.LOSS_CE, 1e-8, 0.5, 1e-3, 1e-3, 8, 30, v0)
            torch.cuda.synchronize()
            h.profile(True)
            h.profile_read(reset=True)
            t0 = time.perf_counter()
            res = api.qst_refactor(h, inst, api.LOSS_CE, 1e-8, 0.5, 1e-3, 1e-3, 8, 30, v0)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            prof = h.profile_read(reset=True)
            h.profile(False)
            runs[name] = (wall, prof["gv"], res["ritz_vals"].cpu().numpy(), int(res["R"][0]))
    finally:
        if old is None:
            os.environ.pop("QST_GV_GROUPED", None)
        else:
            os.environ["QST_GV_GROUPED"] = old
    n_hi = max(0, n - 14)
    groups = len({bytes(r) for r in inst.settings[:, :n_hi].cpu().numpy()}) if n_hi > 0 else B
    wall, (cnt, tot), rv, rout = runs["grouped"]
    wall_s, (cnt_s, tot_s), rv_s, _ = runs["staged"]
    gv_ms = tot / max(cnt, 1)
    # grouped G v bytes: X and W of each group written and read once (stage A, low stage,
    # stage C), the sensitivities of every setting read once, v read and G v written
    gv_bytes = 4.0 * groups * D * 8 + B * D * 4 + 2.0 * D * 8
    lead = np.abs(rv[:2] - rv_s[:2]) / np.abs(rv_s[:2])
    return {
        "refactor_ms": round(wall, 1),
        "refactor_R_out": rout,
        "gv_products": cnt,
        "gv_ms": round(gv_ms, 2),
        "gv_groups": groups,
        "gv_model_bytes": gv_bytes,
        "gv_model_GBps": round(gv_bytes / (gv_ms * 1e-3) / 1e9, 1),
        "refactor_ms_staged_gv": round(wall_s, 1),
        "gv_ms_staged": round(tot_s / max(cnt_s, 1), 2),
        "ritz_rel_diff_grouped_vs_staged": float(lead.max()),
    }


def solve_extra(api, h, dev, seed: int, slots: int = 100):
    """The rank-adaptive iteration (Algorithm 1) on the n=14, R_max=8, B=1000 workload: truth of
    rank 4, frequencies Poisson(1e5 p)/1e5 from the library's own forward of the truth, start
    R_0 = R_max with alpha_0 = 1/R_max, coefficient slots every 5 and spectral slots every 10.
    Wall time of the bounded run, slots, final rank, objective and error e_rho against the truth."""
    import torch

    wl = WORKLOADS["n14_r8_b1000"]
    n, Rmax, B, shots = wl["n"], wl["R"], wl["B"], wl["shots"]
    D = 1 << n
    rng = synth.make_rng(seed)
    s = torch.from_numpy(synth.random_settings(rng, B, n)).to(dev)
    truth = torch.from_numpy(synth.haar_atoms(rng, wl["R_true"], D, dtype=np.complex64)).to(dev)
    wt = torch.from_numpy(synth.dirichlet_weights(rng, wl["R_true"])).to(dev)
    p_true, _ = api.qst_forward(h, [api.Instance(truth, wt, s)], want_probs=True)
    f = synth.poisson_freqs_torch(seed + 1, p_true[0], shots)
    del p_true
    atoms0 = torch.from_numpy(synth.haar_atoms(rng, Rmax, D, dtype=np.complex64)).to(dev)
    w0 = torch.full((Rmax,), 1.0 / Rmax, dtype=torch.float64, device=dev)
    v0s = torch.from_numpy(synth.haar_atoms(rng, 4, D, dtype=np.complex128)).to(dev)
    inst = api.Instance(atoms0, w0, s, f)
    prm = api.SolveParams(max_slots=slots, t_alpha=5, t_ref=10, rank_max=Rmax, n_lanczos=30)
    e0 = api.qst_state_error(h, atoms0, w0, truth, wt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = api.qst_solve(h, inst, prm, v0s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e1 = api.qst_state_error(h, res["atoms"].contiguous(), res["weights"].contiguous(), truth, wt)
    hist = res["history"]
    out = {"workload": "n=14, R_max=8, B=1000, 1e5 shots, truth rank 4; t_alpha=5, t_ref=10, grid 2^-j (11)",
           "slots": res["slots"], "stopped": res["stopped"], "wall_s": round(dt, 2),
           "ms_per_slot": round(dt * 1e3 / max(res["slots"], 1), 2), "accepted": int(hist[:, 4].sum()),
           "oracle_calls": res["oracle_calls"], "rank_final": res["rank"],
           "J_first_slot": round(float(hist[0, 2]), 6), "J_final": round(float(hist[-1, 2]), 6),
           "e_rho_initial": round(e0, 4), "e_rho_final": round(e1, 4)}
    return out


VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak


def config_extra(api, h, dev, seed: int, name: str = "n14_r8_b1000", steps: int = 20, warmup: int = 3,
                 reference=None):
    """One of the smaller configurations on one GPU: n=14, R=8, B=1000 (1e5 shots), where one
    (setting, atom) vector of 2^14 amplitudes fits a work-group and the whole rotation runs on
    chip (pass F with the atoms looped, pass A over slices of settings), or n=10, R=4, B=200
    (1e4 shots), whose four atoms fit one work-group together (fused slices).  The step is the
    headline's (decode, fused forward + adjoint with CE loss, weight gradient and tangent
    projection, FP64 coefficient step), event-timed, with the passes' times, the modelled HBM
    bytes, a roofline against the FP32 vector peak (these paths are bound by vector work and LDS
    transposes, not HBM) and, with `reference` (the CPU baseline leg's oracle), errors on a
    sample of settings."""
    import torch

    wl = WORKLOADS[name]
    n, R, B, shots = wl["n"], wl["R"], wl["B"], wl["shots"]
    D = 1 << n
    rng = synth.make_rng(seed)
    atoms = synth.haar_atoms(rng, R, D, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    freqs = synth.porter_thomas_freqs_torch(seed + 1, B, D, synth.dirichlet_weights(rng, wl["R_true"]), shots, dev)
    inst = api.Instance(torch.from_numpy(atoms).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(s).to(dev),
                        freqs)
    grad = torch.empty_like(inst.atoms)

    def step():
        _, _, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, project_tangent=True, out=[grad])
        api.qst_reweight_simplex(h, inst.weights, wg[0], -0.5, 1e-3)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    h.profile(True)
    h.profile_read(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    stages = h.profile_read(reset=True)
    h.profile(False)
    step_ms = float(np.median(ms))
    amps = B * R * D
    # the method's flops per (setting, atom) amplitude, forward + adjoint: two rotations of
    # 2 flop per element and qubit (a third of the qubits are Z, free), and 12 for |phi|^2, the
    # atom sum, the weight-gradient term, the scaling by alpha g and the sum over settings
    fpa = 4 * n + 12
    tflops = fpa * amps / (step_ms * 1e-3) / 1e12
    onchip = R * D > 16384
    if onchip:
        # frequencies read, 2^-k dL/dp written and read back (its re-reads by the other atom tiles
        # of a slice come from L2), the slice partials written and summed, atoms and gradient
        slices = max(1, min(256 // R, B // 16))
        hbm = 3 * B * D * 4 + 2 * slices * R * D * 8 + 3 * R * D * 8
        passes = {"forward_atoms_looped": round(stages["hi_fwd"][1] / steps, 4),
                  "adjoint_slices": round(stages["lo_fused"][1] / steps, 4),
                  "sums_reductions_tangent": round(stages["reduce"][1] / steps, 4)}
    else:
        # frequencies read, the slice partials written and summed, atoms and gradient
        slices = max(1, B // 4)
        hbm = B * D * 4 + 2 * slices * R * D * 8 + 3 * R * D * 8
        passes = {"fused_slices": round(stages["lo_fused"][1] / steps, 4),
                  "sums_reductions_tangent": round(stages["reduce"][1] / steps, 4)}
    out = {"workload": f"n={n}, R={R}, B={B}, {shots} shots/setting, complex64, cross-entropy",
           "kernels": "on chip, atoms looped" if onchip else "fused slices",
           "ms_per_step": round(step_ms, 4), "amplitudes_per_s": amps / (step_ms * 1e-3),
           "pass_ms_per_step": passes,
           "model_hbm_bytes_per_step": hbm, "model_GBps": round(hbm / (step_ms * 1e-3) / 1e9, 1),
           "roofline": {"bound": "alu", "achieved": round(tflops, 2), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / VALU_PEAK_TFLOPS, 4),
                        "flops": f"{fpa} per (setting, atom) amplitude, the method's forward + adjoint"}}
    if reference is not None:
        sample = [0, B // 3, (2 * B) // 3, B - 1]
        sub_s = s[sample]
        sub_f = synth.porter_thomas_freqs(synth.make_rng(seed + 2), len(sample), D,
                                          synth.dirichlet_weights(synth.make_rng(seed + 3), 4), shots)
        sub = api.Instance(inst.atoms, inst.weights, torch.from_numpy(sub_s).to(dev), torch.from_numpy(sub_f).to(dev))
        lt_s, ag_s, wg_s = api.qst_backward(h, [sub], loss=api.LOSS_CE, eps=1e-8)
        torch.cuda.synchronize()
        Lr, gar, gwr = reference(atoms, w, sub_s, sub_f)
        errs = {"loss": _relerr(float(lt_s[0]), Lr), "weight_grad": _relerr(wg_s[0].cpu().numpy(), gwr),
                "atom_grad": _relerr(ag_s[0].cpu().numpy(), gar)}
        out["errors_vs_oracle"] = {"settings": len(sample), **{k: float(f"{v:.3e}") for k, v in errs.items()},
                                   "tol": 1e-5, "pass": all(v <= 1e-5 for v in errs.values())}
    return out


def n22_extra(api, h, dev, seed: int, n: int = 22, R: int = 16, B: int = 500, shots: int = 1_000_000,
              steps: int = 3, warmup: int = 1) -> dict:
    """A state above twenty qubits: n=22, R=16, B=500 (as many setting-atom amplitudes per step as
    the headline's n=20, B=2000).  Ten low bits would leave twelve above them, more than one
    2^14-amplitude tile takes with at most 2^10 rows; with Pauli settings and dense data the low
    stage takes twelve bits with its atoms looped in one work-group (two sweeps over X), so two
    tile passes remain (otherwise a middle tile pass runs in place on X and W).  The step is the
    headline's, event-timed, with the stages' times and the modelled HBM bytes of the schedule
    that ran."""
    import torch

    D = 1 << n
    inst = step_instance(api, dev, seed, n, R, B, shots, 4)
    grad = torch.empty_like(inst.atoms)

    def step():
        _, _, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, project_tangent=True, out=[grad],
                                    path=api.PATH_BUTTERFLY_F32)
        api.qst_reweight_simplex(h, inst.weights, wg[0], -0.5, 1e-3)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    h.profile(True)
    h.profile_read(reset=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    stages = h.profile_read(reset=True)
    h.profile(False)
    step_ms = float(np.median(ms))
    amps = B * R * D
    ch, cb = 8, 8
    batches = stages["lo_fused"][0] // steps
    S = -(-B // batches)
    mid = stages["mid"][0] > 0
    # per (setting, atom) amplitude: X written by stage A and W read by stage C (8 + 8); the low
    # stage reads X twice and writes W (two sweeps: 24), or reads X and writes W once while the
    # middle pass reads and writes both once more (16 + 32); frequencies once per setting; atoms
    # read by both tile stages and the gradient read and written once per batch
    per_amp = (8 + 8 + 16 + 32) if mid else (8 + 8 + 24)
    hbm = per_amp * B * R * D + B * D * 4 + batches * 3 * R * D * cb
    kinds = ("hi_fwd", "mid", "lo_fused", "hi_adj")
    out = {"workload": f"n={n}, R={R}, B={B}, {shots} shots/setting, complex64, cross-entropy",
           "schedule": ("three passes (top tile stage, middle tile pass, low stage)" if mid else
                        "two tile passes around a two-sweep low stage of n - 10 bits"),
           "settings_per_batch": S,
           "ms_per_step": round(step_ms, 3), "amplitudes_per_s": amps / (step_ms * 1e-3),
           "stage_ms_per_step": {k: round(stages[k][1] / steps, 3) for k in kinds + ("reduce",)},
           "model_hbm_bytes_per_step": hbm, "model_GBps": round(hbm / (step_ms * 1e-3) / 1e9, 1)}
    del grad, inst
    torch.cuda.empty_cache()
    return out


def uneven_batch_extra(api, h, dev, seed: int, reps: int = 5):
    """64 independent instances, n in 6..12, R in 1..8, B in 50..500 (fused CE backward with the
    tangent projection), planned with the autotuner: one call (one launch of each pass per class
    of equal n), the same call replayed from a graph, and 64 one-instance calls.  Median wall
    time of `reps` runs each."""
    import torch

    rng = synth.make_rng(seed)
    insts = []
    amps = 0
    for k, sh in enumerate(synth.uneven_batch_shapes(rng, 64)):
        n, R, B = sh["n"], sh["R"], sh["B"]
        r = synth.make_rng(seed + 1000 + k)
        atoms = torch.from_numpy(synth.haar_atoms(r, R, 1 << n, dtype=np.complex64)).to(dev)
        w = torch.from_numpy(synth.dirichlet_weights(r, R)).to(dev)
        st = torch.from_numpy(synth.random_settings(r, B, n)).to(dev)
        f = synth.porter_thomas_freqs_torch(seed + 2000 + k, B, 1 << n, synth.dirichlet_weights(r, min(R, 4)),
                                            10_000, dev)
        insts.append(api.Instance(atoms, w, st, f))
        amps += B * R * (1 << n)
    # the autotuner times the call's routing (which instances run atoms-looped on chip or as fused
    # slices) and keeps the fastest for calls with these shapes
    api.qst_plan(h, insts, autotune=True)

    def timed(fn):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts[1:])) * 1e3

    one = lambda: api.qst_backward(h, insts, loss=api.LOSS_CE, eps=1e-8, project_tangent=True)  # noqa: E731
    sep = lambda: [api.qst_backward(h, [i], loss=api.LOSS_CE, eps=1e-8, project_tangent=True)  # noqa: E731
                   for i in insts]
    batched_ms = timed(one)
    separate_ms = timed(sep)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        h.set_stream(side)
        one()
    h.set_stream(torch.cuda.current_stream())
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.set_stream(torch.cuda.current_stream())
        one()
    h.set_stream(torch.cuda.current_stream())
    graph_ms = timed(g.replay)
    return {"instances": 64, "amplitudes": amps, "batched_call_ms": round(batched_ms, 3),
            "separate_calls_ms": round(separate_ms, 3), "graph_replay_ms": round(graph_ms, 3),
            "graph_amplitudes_per_s": amps / (graph_ms * 1e-3),
            "speedup_graph_vs_separate": round(separate_ms / graph_ms, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="n20_r16_b2000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip refactor / plain-path timings")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--path", default="butterfly_f32", choices=["butterfly_f32", "butterfly_bf16"],
                    help="path of the timed step: FP32 butterflies (default, the 1e-5 path) or the same with "
                         "BF16 intermediates (1e-2 variant)")
    ap.add_argument("--batch", type=int, default=0, help="settings per batch (0: library default or --autotune)")
    ap.add_argument("--copy-calibration", action="store_true", help="run only a 1 GiB device copy (counter scale)")
    ap.add_argument("--only", choices=["uneven64", "solve", "onchip", "cfg_n10", "refactor", "tile",
                                         "n22"], default=None,
                    help="run only one extra (for profiling) and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    n, R, B, shots = wl["n"], wl["R"], wl["B"], wl["shots"]
    D = 1 << n
    seed = 20260101

    if args.only:
        import torch

        from paper_2607_19577_amd import api

        dev = torch.device("cuda:0")
        h = api.Handle(0)
        if args.only == "uneven64":
            res = uneven_batch_extra(api, h, dev, seed + 21)
        elif args.only == "onchip":
            res = config_extra(api, h, dev, seed + 41, reference=oracle_reference)
        elif args.only == "cfg_n10":
            res = config_extra(api, h, dev, seed + 51, name="n10_r4_b200", reference=oracle_reference)
        elif args.only == "n22":
            res = n22_extra(api, h, dev, seed + 61)
        elif args.only == "tile":
            inst = step_instance(api, dev, seed, n, R, B, shots, wl["R_true"])
            res = tile_extra(api, h, inst)
        elif args.only == "refactor":
            inst = step_instance(api, dev, seed, n, R, B, shots, wl["R_true"])
            res = refactor_extra(api, h, inst, seed + 11)
        else:
            res = solve_extra(api, h, dev, seed + 31)
        print(json.dumps({args.only: res}), flush=True)
        h.close()
        return

    if args.copy_calibration:
        import torch

        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return

    atoms, w, s, w_true = step_inputs(seed, n, R, B, wl["R_true"])

    cpu = cpu_ref = None
    if not args.no_cpu_baseline:
        n_sample = 16 if n >= 18 else min(B, 64 if n <= 12 else 8)
        cpu, cpu_ref = cpu_baseline(atoms, w, s, B, shots, n_sample, seed + 7)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} amplitudes/s ({cpu['sample']})", file=sys.stderr, flush=True)

    if args.batch > 0:
        # read once by the library when it is loaded
        os.environ["QST_SETTINGS_PER_BATCH"] = str(args.batch)

    import torch

    from paper_2607_19577_amd import api

    dev = torch.device("cuda:0")
    inst = step_instance(api, dev, seed, n, R, B, shots, wl["R_true"], (atoms, w, s, w_true))
    freqs = inst.freqs
    grad = torch.empty_like(inst.atoms)
    h = api.Handle(0)
    if args.autotune:
        api.qst_plan(h, [inst], autotune=True)
    print(f"[bench] inputs resident: atoms {inst.atoms.numel() * 8 / 2**20:.0f} MiB, freqs "
          f"{freqs.numel() * 4 / 2**30:.2f} GiB", file=sys.stderr, flush=True)

    step_path = api.PATH_BUTTERFLY_BF16 if args.path == "butterfly_bf16" else api.PATH_BUTTERFLY_F32

    def step():
        lt, ag, wg = api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, project_tangent=True, out=[grad],
                                      path=step_path)
        # coefficient step: beta = proj(alpha + eta (A^T c)) with A^T c = -dL/dalpha
        api.qst_reweight_simplex(h, inst.weights, wg[0], -0.5, 1e-3)
        return lt

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.profile(True)
    h.profile_read(reset=True)
    torch.cuda.synchronize()
    # events on the stream the library launches on (torch's current stream) bracket each step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        lt = step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    stages = h.profile_read(reset=True)
    h.profile(False)
    ms_per_step = elapsed * 1e3 / args.steps
    amps = B * R * D
    value = amps * args.steps / elapsed
    print(f"[bench] {ms_per_step:.2f} ms/step, loss {float(lt[0]):.6f}, stages {stages}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    from paper_2607_19577_amd._lib import load  # noqa: F401

    S = None
    lo_launches = stages["lo_fused"][0]
    if lo_launches:
        S = B * args.steps / lo_launches  # settings per batch (uniform batches)
    cb = 8  # bytes per complex64 (atoms, gradient)
    ch = 4 if args.path == "butterfly_bf16" else 8  # bytes per complex of the intermediates X and W
    per_launch_bytes = {
        "hi_fwd": (R * D * cb + S * R * D * ch) if S else None,
        "lo_fused": (S * R * D * ch + S * D * 4 + S * R * D * ch) if S else None,
        "hi_adj": (S * R * D * ch + 2 * R * D * cb) if S else None,
    }
    dom = max(("hi_fwd", "lo_fused", "hi_adj"), key=lambda k: stages[k][1])
    nl, tot_ms = stages[dom]
    avg_ms = tot_ms / max(nl, 1)
    achieved = per_launch_bytes[dom] / (avg_ms * 1e-3) / 1e9 if per_launch_bytes[dom] else None
    names = {"hi_fwd": "k_stage_hi_fwd", "lo_fused": "k_stage_lo_fused", "hi_adj": "k_stage_hi_adj"}
    traffic = read_traffic(names[dom], args.workload) if args.path == "butterfly_f32" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
                "traffic": traffic, "kernel": names[dom], "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": per_launch_bytes[dom]}
    model_bytes_step = sum((per_launch_bytes[k] or 0) * stages[k][0] for k in per_launch_bytes) / args.steps
    # every stage against the same peak: algorithmic bytes per launch / average launch time
    stage_bw = {}
    for k, b in per_launch_bytes.items():
        nk, tk = stages[k]
        if b and nk and tk > 0:
            gbps = b / (tk / nk * 1e-3) / 1e9
            stage_bw[names[k]] = {"GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4)}

    extras = {}
    if cpu_ref is not None:
        # errors of the timed path against the oracle on the CPU sample (same atoms, weights and
        # settings; the sample's own frequencies)
        ns = cpu_ref["freqs"].shape[0]
        sub = api.Instance(inst.atoms, inst.weights, inst.settings[:ns].contiguous(),
                           torch.from_numpy(cpu_ref["freqs"]).to(dev))
        def path_errors(pth):
            lt_s, ag_s, wg_s = api.qst_backward(h, [sub], loss=api.LOSS_CE, eps=1e-8, path=pth)
            torch.cuda.synchronize()
            return {"loss": _relerr(float(lt_s[0]), cpu_ref["loss"]),
                    "weight_grad": _relerr(wg_s[0].cpu().numpy(), cpu_ref["weight_grad"]),
                    "atom_grad": _relerr(ag_s[0].cpu().numpy(), cpu_ref["atom_grad"])}

        tol = 1e-5 if args.path == "butterfly_f32" else 1e-2
        errs = path_errors(step_path)
        extras["errors_vs_oracle"] = {"settings": ns, "norm": "||x - x_oracle|| / ||x_oracle||",
                                      **{k: float(f"{v:.3e}") for k, v in errs.items()}, "tol": tol,
                                      "pass": all(v <= tol for v in errs.values())}
        if not args.no_extras:
            # the other paths on the same sample, beside their timings below
            other = {}
            for name, pth, ptol in (("plain_f32", api.PATH_PLAIN_F32, 1e-5), ("tile_f16", api.PATH_TILE_F16, 1e-2),
                                    ("tile_bf16", api.PATH_TILE_BF16, 1e-2),
                                    ("butterfly_bf16", api.PATH_BUTTERFLY_BF16, 1e-2)):
                e = path_errors(pth)
                other[name] = {**{k: float(f"{v:.3e}") for k, v in e.items()}, "tol": ptol,
                               "pass": all(v <= ptol for v in e.values())}
            extras["errors_vs_oracle_other_paths"] = other
        del sub, cpu_ref
    if not args.no_extras:
        # plain one-pass-per-qubit reference kernel on the same workload (one call)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=api.PATH_PLAIN_F32, out=[grad])
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3
        extras["plain_path_ms"] = round(plain_ms, 1)
        t0 = time.perf_counter()
        api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, out=[grad])
        torch.cuda.synchronize()
        fused_ms = (time.perf_counter() - t0) * 1e3
        extras["speedup_vs_plain"] = round(plain_ms / fused_ms, 2)
        # MFMA tile paths (one pass per 4-qubit group, FP16 / BF16 operands) and the staged path with
        # BF16 intermediates (tolerance 1e-2 variants)
        for name, pth in (("tile_f16", api.PATH_TILE_F16), ("tile_bf16", api.PATH_TILE_BF16),
                          ("butterfly_bf16", api.PATH_BUTTERFLY_BF16)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.qst_backward(h, [inst], loss=api.LOSS_CE, eps=1e-8, path=pth, out=[grad])
            torch.cuda.synchronize()
            tms = (time.perf_counter() - t0) * 1e3
            extras[f"{name}_path_ms"] = round(tms, 1)
            extras[f"{name}_speedup_vs_plain"] = round(plain_ms / tms, 2)
            if name.startswith("tile"):
                # matrix-core work of the call: 16x16 complex tiles over every (setting, atom)
                # amplitude, ceil(n/4) groups per direction, 128 flop per amplitude and group
                # (twice that executed with split BF16 operands), against the dense peak
                groups = -(-n // 4)
                flop = 2 * groups * B * R * D * 128 * (2 if name == "tile_bf16" else 1)
                tf = flop / (tms * 1e-3) / 1e12
                extras[f"{name}_mfma"] = {"achieved": round(tf, 1), "peak": 2500.0, "unit": "TFLOP/s",
                                          "frac": round(tf / 2500.0, 4)}
        # general local settings: three Haar 2x2 unitaries besides the Pauli bases (codes 0..5),
        # one fused backward on the same atoms and frequencies
        grng = synth.make_rng(seed + 17)
        table = torch.from_numpy(synth.haar_unitaries_2x2(grng, 3)).to(dev)
        gset = torch.from_numpy(synth.random_general_settings(grng, B, n, 3)).to(dev)
        ginst = api.Instance(inst.atoms, inst.weights, gset, freqs, unitaries=table)
        api.qst_backward(h, [ginst], loss=api.LOSS_CE, eps=1e-8, out=[grad])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.qst_backward(h, [ginst], loss=api.LOSS_CE, eps=1e-8, out=[grad])
        torch.cuda.synchronize()
        extras["general_settings_backward_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        # atom step (eq. pi-update): response of one replaced atom on top of p_t, with the loss,
        # against the full forward (probabilities and loss of all R atoms)
        def med3(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return sorted(ts)[1]

        p_t, _ = api.qst_forward(h, [inst], want_probs=True, loss=api.LOSS_CE, eps=1e-8)
        trial = torch.from_numpy(synth.haar_atoms(synth.make_rng(seed + 13), 1, D, dtype=np.complex64)[0]).to(dev)
        fwd_ms = med3(lambda: api.qst_forward(h, [inst], want_probs=True, loss=api.LOSS_CE, eps=1e-8))
        trial_ms = med3(lambda: api.qst_atom_trial(h, inst, R // 2, trial, p_t[0], loss=api.LOSS_CE, eps=1e-8))
        del p_t
        # the unfused autograd route: probabilities through the forward map, the loss in torch,
        # the caller's dL/dp through the adjoint (generic-sensitivity mode)
        from paper_2607_19577_amd.autograd import born_map

        a_req = inst.atoms.detach().clone().requires_grad_(True)
        w_req = inst.weights.detach().clone().requires_grad_(True)

        def autograd_route():
            p = born_map(a_req, w_req, inst.settings, h)
            loss = -((freqs / B) * torch.log(p / B + 1e-8)).sum()
            loss.backward()
            a_req.grad = None
            w_req.grad = None

        extras["autograd_route_ms"] = round(med3(autograd_route), 1)
        del a_req, w_req
        extras["forward_probs_loss_ms"] = round(fwd_ms, 1)
        extras["atom_trial_ms"] = round(trial_ms, 1)
        extras["atom_trial_speedup_vs_forward"] = round(fwd_ms / trial_ms, 2)
        extras.update(refactor_extra(api, h, inst, seed + 11))

    if not args.no_extras:
        ref = None if args.no_cpu_baseline else oracle_reference
        extras["n14_r8_b1000_onchip"] = config_extra(api, h, dev, seed + 41, reference=ref)
        extras["n10_r4_b200_fused_slices"] = config_extra(api, h, dev, seed + 51, name="n10_r4_b200", reference=ref)
        extras["uneven64"] = uneven_batch_extra(api, h, dev, seed + 21)
        extras["solve"] = solve_extra(api, h, dev, seed + 31)
        extras["n22_r16_b500"] = n22_extra(api, h, dev, seed + 61)

    out = {
        "metric": "fwd+adjoint atom-setting amplitudes/s",
        "value": value,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.path == "butterfly_f32" else "f32 (bf16 intermediates)",
        "data": "synthetic",
        "config": {"workload": f"n={n} qubits, R={R} atoms, B={B} random Pauli settings, {shots} shots/setting, "
                               "complex64 atoms, cross-entropy", "n": n, "R": R, "B": B, "D": D,
                   "settings_per_batch": S},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_ms_events": {"median": round(float(np.median(step_ms)), 3),
                           "iqr": round(float(np.percentile(step_ms, 75) - np.percentile(step_ms, 25)), 3),
                           "min": round(float(step_ms.min()), 3), "max": round(float(step_ms.max()), 3)},
        "stage_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in stages.items()},
        "stage_bandwidth": stage_bw,
        "model_hbm_bytes_per_step": model_bytes_step,
        "model_GBps_whole_step": round(model_bytes_step / (ms_per_step * 1e-3) / 1e9, 1),
        "kernel_source_hash": kernel_source_hash(),
        **extras,
    }
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
