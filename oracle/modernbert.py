"""FP64 ModernBERT-style token-classification encoder (test infrastructure only).

The paper names SecureModernBERT-NER as one of the two NER models of stage 2
(Sec. II) and uses it for the accuracy evaluation (Sec. IV-B, App. D); it
gives no architecture.  This oracle follows the published ModernBERT design:

    x      = LN_e(E[id])                              LayerNorms have no shift
    per layer l (pre-LayerNorm, no biases):
      h    = x for l = 0, else LN_a(x)
      q,k,v= h Wqkv, split per head; q and k rotated (RoPE) by their position
             within the record, base 160000 on global layers, 10000 on local
      A_j  = softmax(q_j k_j^T / sqrt(d)) v_j       over the record's keys; on a
             local layer only keys at most w = local_window/2 positions away
      x    = x + A Wo
      [u|g]= LN_m(x) Wi;  x = x + (GELU(u) * g) Wo2
    x      = LN_f(x)
    z      = LN_h(GELU(x Wd)) Wc + bc                 dense + GELU + LN head
    label  = argmax z (lowest index on ties), margin = z(1) - z(2)

Global layers are l = 0, global_every, 2*global_every, ...; the rest are
local.  RoPE rotates the pairs (i, i + d/2) of a head by the angle
pos * base^(-2i/d).  GELU is the exact erf form.

Everything is float64 ("pure").  The "bf16" reading rounds where the GPU's
BF16 path stores a value: both operands of every GEMM, q/k (after the
rotation) and v, the attention probabilities (against the power of two at or
above the row maximum, as in oracle.encoder.attention), the attention output,
the gated MLP output, the LayerNorm outputs and the head's GELU output.  The
residual stream x stays unrounded (FP32 on the GPU).
"""
from __future__ import annotations

import math

import numpy as np

from .encoder import Precision, argmax_margin, gelu, layer_norm, positions


def _w(W, name):
    return np.asarray(W[name], dtype=np.float64)


def rope_angles(pos: np.ndarray, d: int, theta: float) -> np.ndarray:
    """[L, d/2] rotation angles pos * theta^(-2i/d), i = 0 .. d/2 - 1."""
    inv = theta ** (-np.arange(0, d, 2, dtype=np.float64) / d)
    return np.asarray(pos, dtype=np.float64)[:, None] * inv[None, :]


def rope(x: np.ndarray, pos: np.ndarray, theta: float) -> np.ndarray:
    """Rotate [L, H, d] by position: (x_i, x_{i+d/2}) -> (x_i c - x_{i+d/2} s, x_{i+d/2} c + x_i s)."""
    d = x.shape[-1]
    half = d // 2
    ang = rope_angles(pos, d, theta)[:, None, :]
    c, s = np.cos(ang), np.sin(ang)
    x1, x2 = x[..., :half], x[..., half:]
    return np.concatenate([x1 * c - x2 * s, x2 * c + x1 * s], axis=-1)


def attention(q, k, v, window: int | None, round_p=None) -> np.ndarray:
    """Bidirectional attention of one record, [L, H, d] -> [L, H, d]; with
    ``window`` only keys j with |i - j| <= window are seen by query i.  The
    rounding reading of the probabilities is that of oracle.encoder.attention."""
    L, H, d = q.shape
    qh, kh, vh = (np.ascontiguousarray(t.transpose(1, 0, 2)) for t in (q, k, v))
    s = qh @ kh.transpose(0, 2, 1) / math.sqrt(d)
    if window is not None:
        i = np.arange(L)
        s = np.where(np.abs(i[:, None] - i[None, :]) <= window, s, -np.inf)
    if round_p is None:
        p = np.exp(s - s.max(axis=-1, keepdims=True))
        pv = p
    else:
        c = np.ceil(s.max(axis=-1, keepdims=True) / math.log(2.0))
        p = np.exp2(s / math.log(2.0) - c)
        pv = round_p(p)
    l = p.sum(axis=-1, keepdims=True)
    return ((pv @ vh) / l).transpose(1, 0, 2)


def layer(W, cfg, l: int, x: np.ndarray, cu_seqlens, pos: np.ndarray, prec: Precision) -> np.ndarray:
    h, H = cfg.hidden, cfg.n_heads
    d = h // H
    p = f"l{l}."
    zero = np.zeros(h)
    hn = x if l == 0 else prec.store(layer_norm(x, _w(W, p + "attn_ln_g"), zero, cfg.ln_eps))
    qkv = prec.gemm_in(hn, l, 0) @ prec.gemm_w(_w(W, p + "wqkv"))
    glob = cfg.is_global(l)
    theta = cfg.theta_global if glob else cfg.theta_local
    window = None if glob else cfg.local_window // 2
    T = x.shape[0]
    q = prec.store(rope(qkv[:, :h].reshape(T, H, d), pos, theta))
    k = prec.store(rope(qkv[:, h:2 * h].reshape(T, H, d), pos, theta))
    v = prec.store(qkv[:, 2 * h:].reshape(T, H, d))
    A = np.empty((T, h))
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    rp = None if prec.mode == "pure" else prec.probs
    for r in range(len(cu) - 1):
        a, b = int(cu[r]), int(cu[r + 1])
        if b > a:
            A[a:b] = attention(q[a:b], k[a:b], v[a:b], window, rp).reshape(b - a, h)
    A = prec.store(A)
    x = x + prec.gemm_in(A, l, 1) @ prec.gemm_w(_w(W, p + "wo"))
    m = prec.store(layer_norm(x, _w(W, p + "mlp_ln_g"), zero, cfg.ln_eps))
    ug = prec.gemm_in(m, l, 2) @ prec.gemm_w(_w(W, p + "wi"))
    I = cfg.intermediate
    y = prec.store(gelu(ug[:, :I]) * ug[:, I:])
    return x + prec.gemm_in(y, l, 3) @ prec.gemm_w(_w(W, p + "wo2"))


def hidden_states(W, cfg, ids, cu_seqlens, prec: Precision | None = None, n_layers: int | None = None):
    """Residual stream after ``n_layers`` layers (0: after the embedding LayerNorm)."""
    prec = prec or Precision()
    pos = positions(cu_seqlens)
    x = layer_norm(_w(W, "tok_emb")[np.asarray(ids, np.int64)], _w(W, "emb_ln_g"), np.zeros(cfg.hidden),
                   cfg.ln_eps)
    for l in range(cfg.n_layers if n_layers is None else n_layers):
        x = layer(W, cfg, l, x, cu_seqlens, pos, prec)
    return x


def head_logits(W, cfg, x: np.ndarray, prec: Precision) -> np.ndarray:
    zero = np.zeros(cfg.hidden)
    xf = prec.store(layer_norm(x, _w(W, "final_ln_g"), zero, cfg.ln_eps))
    t = prec.store(gelu(prec.gemm_in(xf, 0, 0) @ prec.gemm_w(_w(W, "head_w"))))
    u = prec.store(layer_norm(t, _w(W, "head_ln_g"), zero, cfg.ln_eps))
    return u @ _w(W, "wc") + _w(W, "bc")


def forward(W, cfg, ids, cu_seqlens, prec: Precision | None = None):
    """Logits [T, C], labels u8 [T] and top-2 margins [T] for a packed batch."""
    prec = prec or Precision()
    z = head_logits(W, cfg, hidden_states(W, cfg, ids, cu_seqlens, prec), prec)
    labels, margin = argmax_margin(z)
    return z, labels, margin
