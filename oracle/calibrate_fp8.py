"""Static FP8 activation scales from a calibration pass of the FP64 oracle.

Test infrastructure: this script calls only the oracle and the seeded input
generator.  For each layer it runs the pure FP64 encoder over calibration
records and takes the largest magnitude of the four GEMM inputs (the layer
input x, the attention output, the post-LN1 hidden state, the GELU output);
each scale is the smallest power of two s with amax / s <= 448, the E4M3
maximum.  Static scales keep a record's result independent of the other
records in its batch (a per-batch amax would not).

    python -m oracle.calibrate_fp8 large_fp8
writes tests/golden/fp8_scales_<workload>.json.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import encoder  # noqa: E402

CAL_SEED = 99
CAL_RECORDS = 64


def calibrate(cfg, W, lengths, n_records: int = CAL_RECORDS, seed: int = CAL_SEED):
    rb = synth.generate_records(n_records, lengths, cfg.n_types, cfg.vocab, seed)
    taps: dict = {}
    encoder.hidden_states(W, cfg, rb.ids, rb.cu_seqlens, encoder.Precision("pure"), taps=taps)
    out = []
    for l in range(cfg.n_layers):
        t = taps[l]
        amax = [float(np.abs(t["x_in"]).max()), float(np.abs(t["attn"]).max()), float(np.abs(t["x_mid"]).max()),
                float(np.abs(t["ffn1"]).max())]
        out.append([encoder.power_of_two_scale(a) for a in amax])
    return out, rb.n_tokens


def main(name: str) -> str:
    wl = synth.workload(name)
    W = synth.make_weights(wl.model, wl.weight_seed, wl.o_target)
    t0 = time.time()
    scales, ntok = calibrate(wl.model, W, wl.lengths)
    path = os.path.join(ROOT, "tests", "golden", f"fp8_scales_{name}.json")
    with open(path, "w") as f:
        json.dump({"source": "written by oracle/calibrate_fp8.py: pure FP64 oracle over "
                             f"{CAL_RECORDS} generator records (seed {CAL_SEED}) of workload {name}, "
                             f"{ntok} tokens; per layer [qkv_in, attn_out, ffn1_in, ffn2_in] power-of-two scales",
                   "workload": name, "scales": scales}, f, indent=1)
    print(f"wrote {path} in {time.time() - t0:.1f} s")
    return path


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "large_fp8")
