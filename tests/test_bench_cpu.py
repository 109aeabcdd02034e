"""Host-side pieces of bench.py: the one-GPU guard, the committed traffic summaries (taken on
the current kernel sources), and the CPU baseline's oracle outputs, which the bench compares
with the timed path."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import synth
from oracle import born

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("kernel", ["k_stage_hi_fwd", "k_stage_lo_fused", "k_stage_hi_adj"])
def test_traffic_summaries_match_the_kernel_sources(kernel):
    """The HBM traffic in the bench line comes from profiles/ only if they were taken on these
    sources; each stage's measured bytes are its algorithmic bytes: X and W once each way, the
    frequencies once per setting, the atoms and the gradient once per batch."""
    t = bench.read_traffic(kernel, "n20_r16_b2000")
    assert t is not None, "profiles/ were taken on other kernel sources"
    n, R, B = 20, 16, 2000
    D, S = 1 << n, B / 16.0  # 16 batches (the default of 128 settings, the last of 80)
    alg = {"k_stage_hi_fwd": R * D * 8 + S * R * D * 8,
           "k_stage_lo_fused": 2 * S * R * D * 8 + S * D * 4,
           "k_stage_hi_adj": S * R * D * 8 + 2 * R * D * 8}[kernel]
    assert abs(t / alg - 1.0) < 0.01


def test_cpu_baseline_returns_the_oracle_outputs():
    rng = synth.make_rng(31)
    n, R, B = 6, 3, 40
    atoms = synth.haar_atoms(rng, R, 1 << n, dtype=np.complex64)
    w = synth.dirichlet_weights(rng, R)
    s = synth.random_settings(rng, B, n)
    rec, ref = bench.cpu_baseline(atoms, w, s, B, 1000, 5, 77)
    assert rec["kind"] == "oracle" and rec["value"] > 0 and rec["cores"] >= 1
    a = atoms.astype(np.complex128)
    p = born.probs_axis(a, w, s[:5])
    L, g = born.loss_and_sensitivity(p, ref["freqs"], 5, born.LOSS_CE, 1e-8)
    ga, gw = born.gradients_axis(a, w, s[:5], g)
    assert abs(L - ref["loss"]) <= 1e-12 * abs(L)
    assert bench._relerr(ref["weight_grad"], gw) < 1e-12
    assert bench._relerr(ref["atom_grad"], ga) < 1e-12
