"""Synthetic encoder weights: N(0, 0.02) draws in a fixed tensor order.

The paper's NER models are pretrained checkpoints (Sec. II, stage 2) that are
not available here; the encoder is exercised with seeded random weights.  All
matrices, embeddings and biases are N(0, 0.02); LayerNorm gains are
1 + N(0, 0.02) and LayerNorm shifts N(0, 0.02), so every bias path carries a
non-trivial value.  Matrices are stored in "x @ W" orientation ([in, out]).

The flat FP32 blob handed to the GPU library lists the tensors in exactly the
order of :func:`tensor_specs`.

Classifier head.  With a random head roughly 1/C of tokens argmax to O, which
would turn almost every token into an entity.  For the larger workloads a
constant is added to the O logit's bias so that about ``o_target`` of tokens
predict O.  The constant is chosen from the distribution the head sees: the
final LayerNorm output has unit variance per channel, so each logit is close
to N(0, h * 0.02^2) and the bias solves
``P(Z_0 + delta > max(Z_1..Z_{C-1})) = o_target`` for i.i.d. normal Z.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize, stats

from .configs import ModelConfig, ModernConfig

STD = 0.02


def modern_tensor_specs(cfg: ModernConfig) -> list[tuple[str, tuple[int, ...]]]:
    """ModernBERT-style encoder (no biases but the classifier's; LayerNorms
    without shifts; layer 0 has no attention LayerNorm).  wi holds the MLP's
    input half in columns [0, I) and its gate half in [I, 2I)."""
    h, I, C = cfg.hidden, cfg.intermediate, cfg.n_labels
    specs = [("tok_emb", (cfg.vocab, h)), ("emb_ln_g", (h,))]
    for l in range(cfg.n_layers):
        if l > 0:
            specs.append((f"l{l}.attn_ln_g", (h,)))
        specs += [(f"l{l}.wqkv", (h, 3 * h)), (f"l{l}.wo", (h, h)), (f"l{l}.mlp_ln_g", (h,)),
                  (f"l{l}.wi", (h, 2 * I)), (f"l{l}.wo2", (I, h))]
    specs += [("final_ln_g", (h,)), ("head_w", (h, h)), ("head_ln_g", (h,)), ("wc", (h, C)), ("bc", (C,))]
    return specs


def tensor_specs(cfg) -> list[tuple[str, tuple[int, ...]]]:
    if isinstance(cfg, ModernConfig):
        return modern_tensor_specs(cfg)
    h, f, C = cfg.hidden, cfg.ffn, cfg.n_labels
    specs = [("tok_emb", (cfg.vocab, h)), ("pos_emb", (cfg.max_pos, h)),
             ("emb_ln_g", (h,)), ("emb_ln_b", (h,))]
    for l in range(cfg.n_layers):
        specs += [(f"l{l}.wqkv", (h, 3 * h)), (f"l{l}.bqkv", (3 * h,)),
                  (f"l{l}.wo", (h, h)), (f"l{l}.bo", (h,)),
                  (f"l{l}.ln1_g", (h,)), (f"l{l}.ln1_b", (h,)),
                  (f"l{l}.w1", (h, f)), (f"l{l}.b1", (f,)),
                  (f"l{l}.w2", (f, h)), (f"l{l}.b2", (h,)),
                  (f"l{l}.ln2_g", (h,)), (f"l{l}.ln2_b", (h,))]
    specs += [("wc", (h, C)), ("bc", (C,))]
    return specs


def o_bias_for(cfg, o_target: float) -> float:
    """Bias on the O logit giving P(argmax = O) = o_target for i.i.d. N(0, s^2) logits."""
    s = math.sqrt(cfg.hidden) * STD
    k = cfg.n_labels - 1

    def p_win(delta):
        f = lambda z: stats.norm.pdf(z) * stats.norm.cdf(z + delta / s) ** k
        return integrate.quad(f, -12, 12)[0]

    return float(optimize.brentq(lambda d: p_win(d) - o_target, -10 * s, 20 * s))


def make_weights(cfg, seed: int = 0, o_target: float | None = None) -> dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    out: dict[str, np.ndarray] = {}
    for name, shape in tensor_specs(cfg):
        w = (rng.standard_normal(shape, dtype=np.float32) * np.float32(STD)).astype(np.float32)
        if name.endswith("_g"):
            w = (w + np.float32(1.0)).astype(np.float32)
        out[name] = w
    if o_target is not None:
        out["bc"] = out["bc"].copy()
        out["bc"][0] += np.float32(o_bias_for(cfg, o_target))
    return out


def weights_blob(cfg, weights: dict[str, np.ndarray]) -> np.ndarray:
    """The weights as one contiguous FP32 array in :func:`tensor_specs` order."""
    parts = []
    for name, shape in tensor_specs(cfg):
        w = weights[name]
        assert w.shape == shape and w.dtype == np.float32, (name, w.shape, shape)
        parts.append(w.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def make_key(seed: int = 0) -> bytes:
    """The 32-byte HMAC key (operator-defined in the paper, Sec. II stage 3)."""
    return np.random.default_rng(seed).bytes(32)
