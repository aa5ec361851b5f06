"""How far apart can two correct reduced-precision evaluations of the encoder be?

Test infrastructure: calls only the oracle and the seeded generator.  The
bf16 reading rounds every stored activation; rounding is discontinuous, so a
relative perturbation far below bf16 resolution (1e-7, the order of FP32
accumulation error) flips some roundings, and over many layers these flips
spread into logit differences of the size of bf16 noise itself.  This script
measures that spread on the oracle alone:

* the bf16 oracle against itself with a 1e-7 relative perturbation before each
  rounding (what any FP32-accumulating GPU implementation amounts to);
* the bf16 oracle against the pure float64 oracle.

The largest spread sets the label-agreement margin that a reduced-precision
path can be held to: two evaluations that differ by at most d per logit can
disagree on the argmax only where the top-2 margin is below 2d.

    python -m oracle.sensitivity base_bf16   -> tests/golden/sensitivity_base_bf16.json
    python -m oracle.sensitivity base2_windowed_bf16   (the windowed BF16 test's case)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import encoder  # noqa: E402
from oracle.numerics import round_bf16  # noqa: E402

LENGTHS = [512, 37, 200, 16, 129, 300]
EPS = 1e-7


class _Perturbed(encoder.Precision):
    """The reduced-precision reading with every value that the GPU forms in
    FP32 and then rounds to bf16 (stored activations, attention
    probabilities) perturbed by a relative ``eps`` first.  FP8 GEMM inputs
    are quantised from values already rounded to bf16, exactly on both
    sides, so they are not perturbed again."""

    def __init__(self, mode, eps, seed, act_scales=None):
        super().__init__(mode, act_scales or [])
        self.rng = np.random.default_rng(seed)
        self.eps = eps

    def _jitter(self, x):
        x = np.asarray(x, dtype=np.float64)
        return x * (1.0 + self.eps * self.rng.standard_normal(x.shape))

    def store(self, x):
        return round_bf16(self._jitter(x))

    def probs(self, p):
        return round_bf16(self._jitter(p))


def perturbed_precision(mode: str, seed: int, act_scales=None, eps: float = EPS) -> encoder.Precision:
    """The perturbed reading as a Precision (its own random stream)."""
    return _Perturbed(mode, eps, seed, act_scales)


def ambiguous_tokens(labels, zq, tokens, runs) -> list:
    """The tokens among ``tokens`` where another reduced-precision evaluation
    may legitimately give ``labels``: for some perturbed run (logits, labels,
    margins of the oracle perturbed by 1e-7 before each bf16 rounding, on the
    same tokens) the run gives that label there, or the run's margin there is
    below the run's own largest logit deviation from the rounding oracle zq."""
    out = []
    for t in tokens:
        for zn, ln, mn in runs:
            if ln[t] == labels[t] or mn[t] < np.abs(zn - zq).max():
                out.append(int(t))
                break
    return out


def perturbed_forward(W, cfg, ids, cu_seqlens, mode: str, seed: int, act_scales=None, eps: float = EPS,
                      window: int = 0, stride: int = 0):
    """Logits, labels and margins of the perturbed reading (one seed)."""
    from oracle import pipeline as opipe
    return opipe.ner(W, cfg, ids, cu_seqlens, _Perturbed(mode, eps, seed, act_scales), window, stride)


def measure(name: str) -> dict:
    wl = synth.workload(name)
    cfg = wl.model
    W = synth.make_weights(cfg, wl.weight_seed, wl.o_target)
    rb = synth.generate_records(len(LENGTHS), np.array(LENGTHS), cfg.n_types, cfg.vocab, 17)
    mode = wl.precision
    scales = None
    if mode == "fp8":
        with open(os.path.join(ROOT, "tests", "golden", f"fp8_scales_{name}.json")) as f:
            scales = json.load(f)["scales"]
    zq, lq, mq = encoder.forward(W, cfg, rb.ids, rb.cu_seqlens, encoder.Precision(mode, scales or []))
    zp, lp, mp = encoder.forward(W, cfg, rb.ids, rb.cu_seqlens)
    zn, ln, mn = encoder.forward(W, cfg, rb.ids, rb.cu_seqlens, _Perturbed(mode, EPS, 1, scales))
    dn, dp = np.abs(zn - zq), np.abs(zq - zp)
    return {
        "source": "written by oracle/sensitivity.py (oracle only)",
        "workload": name, "layers": cfg.n_layers, "hidden": cfg.hidden, "tokens": int(rb.n_tokens),
        "perturbation": EPS,
        "perturbed_vs_rounding_oracle": {"max": float(dn.max()), "rms": float(np.sqrt((dn ** 2).mean()))},
        "rounding_oracle_vs_pure": {"max": float(dp.max()), "rms": float(np.sqrt((dp ** 2).mean()))},
        "confident_label_flips_at_1e-2": int(((ln != lq) & (mq > 1e-2)).sum()),
        "tokens_with_margin_above_1e-2": int((mq > 1e-2).sum()),
    }


# Base widths with two layers, windowed as the dataset-scale stream is (512
# tokens every 448), on records longer than one window: the case of the
# windowed BF16 parity test, with its weights and records.
WINDOWED = {"lengths": [1300, 513, 900, 200], "records_seed": 13, "weight_seed": 2, "window": 512, "stride": 448}


def measure_windowed_base2() -> dict:
    from oracle import pipeline as opipe
    from synth.configs import ModelConfig
    cfg = ModelConfig(n_layers=2, hidden=768, n_heads=12, ffn=3072, vocab=30522, n_labels=17)
    W = synth.make_weights(cfg, WINDOWED["weight_seed"])
    rb = synth.generate_records(len(WINDOWED["lengths"]), np.array(WINDOWED["lengths"]), cfg.n_types, cfg.vocab,
                                WINDOWED["records_seed"])
    win, st = WINDOWED["window"], WINDOWED["stride"]
    zq, lq, mq = opipe.ner(W, cfg, rb.ids, rb.cu_seqlens, encoder.Precision("bf16"), win, st)
    zp, lp, mp = opipe.ner(W, cfg, rb.ids, rb.cu_seqlens, None, win, st)
    zn, ln, mn = opipe.ner(W, cfg, rb.ids, rb.cu_seqlens, _Perturbed("bf16", EPS, 1), win, st)
    dn, dp = np.abs(zn - zq), np.abs(zq - zp)
    return {
        "source": "written by oracle/sensitivity.py (oracle only)",
        "workload": "base2_windowed_bf16", "layers": cfg.n_layers, "hidden": cfg.hidden, "tokens": int(rb.n_tokens),
        "case": WINDOWED, "perturbation": EPS,
        "perturbed_vs_rounding_oracle": {"max": float(dn.max()), "rms": float(np.sqrt((dn ** 2).mean()))},
        "rounding_oracle_vs_pure": {"max": float(dp.max()), "rms": float(np.sqrt((dp ** 2).mean()))},
        "confident_label_flips_at_1e-2": int(((ln != lq) & (mq > 1e-2)).sum()),
        "tokens_with_margin_above_1e-2": int((mq > 1e-2).sum()),
    }


if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else "base_bf16"
    out = measure_windowed_base2() if name == "base2_windowed_bf16" else measure(name)
    path = os.path.join(ROOT, "tests", "golden", f"sensitivity_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
