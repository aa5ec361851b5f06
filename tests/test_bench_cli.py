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


def test_traffic_is_read_for_the_tile_order_the_run_chose():
    """The FFN1 counter file holds one entry per tile order; the bench takes
    the entry of the order its own run chose, and none for an order the
    counters were not taken on (or for a GEMM source that changed since)."""
    path = os.path.join(ROOT, "profiles", "base_bf16_ffn1_counters.json")
    with open(path) as f:
        c = json.load(f)
    entries = c["entries"]
    assert len({e["tile"] for e in entries}) == len(entries) >= 2
    for e in entries:
        got, src = bench.counter_traffic("base_bf16", "ffn1", e["tile"])
        if got is None:  # the kernel source changed after the counters were taken
            assert "changed" in src
            return
        assert got == e["bytes_per_launch"] and e["tile"] in src
    got, src = bench.counter_traffic("base_bf16", "ffn1", "bf16_no_such_tile")
    assert got is None and "this run chose bf16_no_such_tile" in src
