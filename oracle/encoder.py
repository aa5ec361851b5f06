"""FP64 token-classification encoder (test infrastructure only).

What it computes.  The paper's stage 2 (Sec. II) labels every token with an
entity class using a pretrained transformer NER model run on the GPU.  No
architecture is given; this oracle follows the encoder shapes the build is
measured on: a post-LayerNorm BERT-style encoder with learned absolute
positions, an embedding LayerNorm, exact-erf GELU, no token-type embedding and
a linear token-classification head.  In order:

    x      = LN_e(E[id] + P[pos])                  pos counts from 0 per record
    per layer:
      qkv  = x Wqkv + bqkv                         columns [Q | K | V], head j
                                                   owns columns j*d .. (j+1)*d
      A_j  = softmax(Q_j K_j^T / sqrt(d)) V_j      keys of the same record only
      x    = LN1(x + A Wo + bo)
      x    = LN2(x + GELU(x W1 + b1) W2 + b2)
    z      = x Wc + bc
    label  = argmax z (lowest index on ties), margin = z(1) - z(2)

    LN(y)  = g * (y - mean) / sqrt(var + eps) + b  (population variance)
    GELU(u)= u/2 * (1 + erf(u / sqrt 2))

Everything is float64 ("pure").  A second reading, "bf16", rounds to
bfloat16 at exactly the points where the GPU's BF16 path stores a value:
both operands of every GEMM, the stored hidden state after each LayerNorm
(which is also the residual input of the next sublayer), the residual sum
x + sublayer(x) that each LayerNorm reads, Q/K/V, the attention
probabilities before they multiply V (taken against the power of two at or
above the row maximum, see attention()), the attention
output, and the GELU output.  Dot products, LayerNorm statistics, the softmax
max/sum and the classifier stay float64 (FP32 on the GPU).  "fp8" additionally rounds the inputs of the
QKV, output-projection, FFN1 and FFN2 GEMMs to FP8-E4M3 with static
power-of-two per-tensor scales.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf

from .numerics import round_bf16, round_e4m3


def layer_norm(y: np.ndarray, g: np.ndarray, b: np.ndarray, eps: float) -> np.ndarray:
    mu = y.mean(axis=-1, keepdims=True)
    var = ((y - mu) ** 2).mean(axis=-1, keepdims=True)
    return g * (y - mu) / np.sqrt(var + eps) + b


def gelu(u: np.ndarray) -> np.ndarray:
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def softmax_rows(s: np.ndarray) -> np.ndarray:
    p = np.exp(s - s.max(axis=-1, keepdims=True))
    return p / p.sum(axis=-1, keepdims=True)


def attention(q: np.ndarray, k: np.ndarray, v: np.ndarray, round_p=None) -> np.ndarray:
    """Full bidirectional attention of one record.  q, k, v: [L, H, d] -> [L, H, d].

    Without ``round_p``: softmax(q k^T / sqrt(d)) v, with the row maximum
    subtracted before the exponential.  With ``round_p`` (the reduced-
    precision reading) the unnormalised probabilities are taken against the
    power of two at or above the row maximum, p = 2^(s log2(e) - c) with
    c = ceil(max(s) log2(e)), rounded by ``round_p`` before they multiply v,
    and the result is divided by the sum of the unrounded p.  Softmax does not
    depend on the reference; the reference only fixes where p is rounded, and
    any power of two at or above the maximum gives the same rounded values up
    to that power of two.
    """
    d = q.shape[-1]
    qh, kh, vh = (np.ascontiguousarray(t.transpose(1, 0, 2)) for t in (q, k, v))   # [H, L, d]
    s = qh @ kh.transpose(0, 2, 1) / math.sqrt(d)                                   # [H, Lq, Lk]
    if round_p is None:
        p = np.exp(s - s.max(axis=-1, keepdims=True))
        pv = p
    else:
        c = np.ceil(s.max(axis=-1, keepdims=True) / math.log(2.0))
        p = np.exp2(s / math.log(2.0) - c)
        pv = round_p(p)
    l = p.sum(axis=-1, keepdims=True)
    o = (pv @ vh) / l
    return o.transpose(1, 0, 2)


def positions(cu_seqlens: np.ndarray) -> np.ndarray:
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    return np.concatenate([np.arange(cu[i + 1] - cu[i]) for i in range(len(cu) - 1)] or [np.zeros(0, np.int64)])


def power_of_two_scale(amax: float) -> float:
    """Smallest power of two s with amax / s <= 448 (the E4M3 maximum)."""
    if amax <= 0.0:
        return 1.0
    s = float(2.0 ** math.ceil(math.log2(amax / 448.0)))
    # log2 of a rounded quotient can land one binade off near amax = 448 * 2**k
    while amax / s > 448.0:
        s *= 2.0
    while amax / (s / 2.0) <= 448.0:
        s /= 2.0
    return s


@dataclass
class Precision:
    """Where values are rounded.  ``mode`` is "pure", "bf16" or "fp8".

    For "fp8", ``act_scales[l]`` holds the static scales of the four GEMM
    inputs of layer l, in the order (qkv, o, ffn1, ffn2).
    """
    mode: str = "pure"
    act_scales: list = field(default_factory=list)

    def store(self, x):
        return x if self.mode == "pure" else round_bf16(x)

    def gemm_in(self, x, layer: int, which: int):
        if self.mode == "pure":
            return x
        if self.mode == "bf16":
            return round_bf16(x)
        s = self.act_scales[layer][which]
        return s * round_e4m3(x / s)

    def gemm_w(self, w):
        if self.mode == "pure":
            return w
        if self.mode == "bf16":
            return round_bf16(w)
        s = power_of_two_scale(float(np.abs(w).max()))
        return s * round_e4m3(w / s)

    def probs(self, p):
        return p if self.mode == "pure" else round_bf16(p)


def _w(W, name):
    return np.asarray(W[name], dtype=np.float64)


def embed(W, cfg, ids: np.ndarray, cu_seqlens: np.ndarray) -> np.ndarray:
    pos = positions(cu_seqlens)
    y = _w(W, "tok_emb")[np.asarray(ids, np.int64)] + _w(W, "pos_emb")[pos]
    return layer_norm(y, _w(W, "emb_ln_g"), _w(W, "emb_ln_b"), cfg.ln_eps)


def encoder_layer(W, cfg, l: int, x: np.ndarray, cu_seqlens: np.ndarray, prec: Precision,
                  taps: dict | None = None) -> np.ndarray:
    h, H = cfg.hidden, cfg.n_heads
    d = h // H
    p = f"l{l}."
    x_in = x
    qkv = prec.gemm_in(x, l, 0) @ prec.gemm_w(_w(W, p + "wqkv")) + _w(W, p + "bqkv")
    qkv = prec.store(qkv)
    A = np.empty((x.shape[0], h))
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    rp = None if prec.mode == "pure" else prec.probs
    for s in range(len(cu) - 1):
        a, b = int(cu[s]), int(cu[s + 1])
        if b == a:
            continue
        L = b - a
        A[a:b] = attention(qkv[a:b, :h].reshape(L, H, d), qkv[a:b, h:2 * h].reshape(L, H, d),
                           qkv[a:b, 2 * h:].reshape(L, H, d), rp).reshape(L, h)
    A = prec.store(A)
    y = prec.store(x + prec.gemm_in(A, l, 1) @ prec.gemm_w(_w(W, p + "wo")) + _w(W, p + "bo"))
    x = prec.store(layer_norm(y, _w(W, p + "ln1_g"), _w(W, p + "ln1_b"), cfg.ln_eps))
    x_mid = x
    g = prec.store(gelu(prec.gemm_in(x, l, 2) @ prec.gemm_w(_w(W, p + "w1")) + _w(W, p + "b1")))
    y = prec.store(x + prec.gemm_in(g, l, 3) @ prec.gemm_w(_w(W, p + "w2")) + _w(W, p + "b2"))
    x = prec.store(layer_norm(y, _w(W, p + "ln2_g"), _w(W, p + "ln2_b"), cfg.ln_eps))
    if taps is not None:
        taps[l] = dict(qkv=qkv, attn=A, ffn1=g, x_in=x_in, x_mid=x_mid)
    return x


def hidden_states(W, cfg, ids, cu_seqlens, prec: Precision | None = None, n_layers: int | None = None,
                  taps: dict | None = None) -> np.ndarray:
    """Hidden state after ``n_layers`` layers (0: after the embedding LayerNorm)."""
    prec = prec or Precision()
    x = prec.store(embed(W, cfg, ids, cu_seqlens))
    nl = cfg.n_layers if n_layers is None else n_layers
    for l in range(nl):
        x = encoder_layer(W, cfg, l, x, cu_seqlens, prec, taps)
    return x


def classify_logits(W, x: np.ndarray) -> np.ndarray:
    return x @ _w(W, "wc") + _w(W, "bc")


def argmax_margin(z: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Label = first index of the maximum; margin = top-1 minus top-2 logit."""
    labels = np.argmax(z, axis=-1)
    srt = np.sort(z, axis=-1)
    margin = srt[:, -1] - srt[:, -2] if z.shape[-1] > 1 else np.full(z.shape[0], np.inf)
    return labels.astype(np.uint8), margin


def forward(W, cfg, ids, cu_seqlens, prec: Precision | None = None):
    """Logits [T, C], labels u8 [T] and top-2 margins [T] for a packed batch."""
    x = hidden_states(W, cfg, ids, cu_seqlens, prec)
    z = classify_logits(W, x)
    labels, margin = argmax_margin(z)
    return z, labels, margin
