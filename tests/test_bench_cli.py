"""The bench's contract on the CPU: one GPU only, and the algorithmic FLOP
counts behind its roofline figure."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth.configs import BASE  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_flop_counts_match_the_encoder_closed_form():
    """A 512-token record through the base encoder: each layer's GEMMs cost
    twice their weight count per token (4h^2 + 2hf weights), attention
    4 L h per token, the classifier 2 h C; 188.8 MFLOP per position."""
    h, f, C, L = BASE.hidden, BASE.ffn, BASE.n_labels, 512
    cu = np.array([0, L])
    per_layer_token = 2 * (4 * h * h + 2 * h * f) + 4 * L * h
    want = BASE.n_layers * per_layer_token * L + 2 * h * C * L
    assert bench.path_flops(BASE, cu) == want
    assert abs(want / L / 1e6 - 188.8) < 0.05
    # attention is quadratic per record and additive over records
    cu3 = np.array([0, 10, 10, 40])
    assert bench.attention_flops(cu3, BASE) == 4 * h * (10 ** 2 + 0 + 30 ** 2)
    g = bench.gemm_flops_per_token(BASE)
    assert g["qkv"] == 3 * g["oproj"] and g["ffn1"] == g["ffn2"] == 2 * h * f


def test_modern_attention_flops_count_the_window_pairs():
    """The ModernBERT-style FLOP accounting: attention counts every key a
    query sees (all of its record on global layers, those at most 64 positions
    away on local ones), checked against a brute-force pair count."""
    import numpy as np
    import bench
    from synth.configs import MODERN_BASE
    cu = np.array([0, 3, 100, 700, 829])
    f = bench.modern_flops(MODERN_BASE, cu)
    L = np.diff(cu)
    band = sum(sum(1 for i in range(n) for j in range(n) if abs(i - j) <= 64) for n in L)
    full = sum(int(n) * int(n) for n in L)
    n_glob = len(range(0, MODERN_BASE.n_layers, MODERN_BASE.global_every))
    assert f["attn"] == 4 * MODERN_BASE.hidden * (n_glob * full + (MODERN_BASE.n_layers - n_glob) * band)
    assert f["ffn1"] == MODERN_BASE.n_layers * 2 * 768 * 2 * 1152 * 829
