"""Pins of the ModernBERT-style oracle (oracle/modernbert.py), CPU only.

The library special case: the whole oracle in float64 against the transformers
ModernBertForTokenClassification model (eager attention, float64, weights
copied) on records longer than the local window, so that global and local
layers, rotary positions, the gated MLP and the head are all exercised.  The
library forms its rotary angles in float32, the oracle in float64; below 400
positions the logits agree to about 1e-9 relative, and the bar is 1e-7 (a
window one key wider moves them by about 1e-3, another rotary base by 2e-4).
Further pins: the rotation
against its closed form (an orthogonal map, identity at position 0, scores
depending on the position difference only), the sliding window against a
brute-force triple loop, and the packed batch against each record alone."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import modernbert as mb
from oracle.encoder import Precision
from synth.configs import MODERN_TINY, ModernConfig


def _hf_model(cfg: ModernConfig, W):
    torch = pytest.importorskip("torch")
    tr = pytest.importorskip("transformers")
    conf = tr.ModernBertConfig(vocab_size=cfg.vocab, hidden_size=cfg.hidden, intermediate_size=cfg.intermediate,
                               num_hidden_layers=cfg.n_layers, num_attention_heads=cfg.n_heads,
                               max_position_embeddings=cfg.max_pos, norm_eps=cfg.ln_eps, norm_bias=False,
                               attention_bias=False, mlp_bias=False, classifier_bias=False,
                               classifier_activation="gelu", hidden_activation="gelu",
                               local_attention=cfg.local_window, global_attn_every_n_layers=cfg.global_every,
                               global_rope_theta=cfg.theta_global, local_rope_theta=cfg.theta_local,
                               num_labels=cfg.n_labels, pad_token_id=0, bos_token_id=1, eos_token_id=2,
                               cls_token_id=1, sep_token_id=2, attn_implementation="eager")
    m = tr.ModernBertForTokenClassification(conf).double().eval()
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    with torch.no_grad():
        m.model.embeddings.tok_embeddings.weight.copy_(t(W["tok_emb"]))
        m.model.embeddings.norm.weight.copy_(t(W["emb_ln_g"]))
        for l, lay in enumerate(m.model.layers):
            p = f"l{l}."
            if l > 0:
                lay.attn_norm.weight.copy_(t(W[p + "attn_ln_g"]))
            lay.attn.Wqkv.weight.copy_(t(W[p + "wqkv"]).T)
            lay.attn.Wo.weight.copy_(t(W[p + "wo"]).T)
            lay.mlp_norm.weight.copy_(t(W[p + "mlp_ln_g"]))
            lay.mlp.Wi.weight.copy_(t(W[p + "wi"]).T)
            lay.mlp.Wo.weight.copy_(t(W[p + "wo2"]).T)
        m.model.final_norm.weight.copy_(t(W["final_ln_g"]))
        m.head.dense.weight.copy_(t(W["head_w"]).T)
        m.head.norm.weight.copy_(t(W["head_ln_g"]))
        m.classifier.weight.copy_(t(W["wc"]).T)
        m.classifier.bias.copy_(t(W["bc"]))
    return m


def test_oracle_matches_transformers_modernbert_float64():
    """P5 for the ModernBERT-style encoder: records of 300, 129 and 64 tokens
    (beyond, at and inside the 128-token local window)."""
    torch = pytest.importorskip("torch")
    cfg = MODERN_TINY
    W = synth.make_weights(cfg, 3)
    hf = _hf_model(cfg, W)
    rb = synth.generate_records(3, np.array([300, 129, 64]), cfg.n_types, cfg.vocab, 5)
    z, _, _ = mb.forward(W, cfg, rb.ids, rb.cu_seqlens)
    for r in range(rb.n_records):
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        with torch.no_grad():
            want = hf(input_ids=torch.from_numpy(rb.ids[a:b].astype(np.int64))[None]).logits[0].numpy()
        rel = np.abs(z[a:b] - want).max() / np.abs(want).max()
        assert rel < 1e-7, (r, rel)


def test_rope_is_a_position_rotation():
    rng = np.random.default_rng(0)
    L, H, d = 50, 2, 64
    x = rng.normal(size=(L, H, d))
    pos = np.arange(L)
    y = mb.rope(x, pos, 10000.0)
    # orthogonal (norms kept), identity at position 0
    np.testing.assert_allclose(np.linalg.norm(y, axis=-1), np.linalg.norm(x, axis=-1), rtol=1e-13)
    np.testing.assert_array_equal(y[0], x[0])
    # pair i rotates by pos * theta^(-2i/d): check one pair by hand
    i, t = 5, 17
    ang = t * 10000.0 ** (-2 * i / d)
    c, s = math.cos(ang), math.sin(ang)
    np.testing.assert_allclose([y[t, 0, i], y[t, 0, i + d // 2]],
                               [x[t, 0, i] * c - x[t, 0, i + d // 2] * s, x[t, 0, i + d // 2] * c + x[t, 0, i] * s],
                               rtol=1e-13)
    # the score of a rotated pair depends only on the position difference
    q, k = rng.normal(size=(1, 1, d)), rng.normal(size=(1, 1, d))
    s1 = (mb.rope(q, np.array([7]), 160000.0) * mb.rope(k, np.array([3]), 160000.0)).sum()
    s2 = (mb.rope(q, np.array([104]), 160000.0) * mb.rope(k, np.array([100]), 160000.0)).sum()
    assert abs(s1 - s2) < 1e-12


def test_sliding_window_attention_brute_force():
    rng = np.random.default_rng(1)
    L, H, d, w = 23, 2, 8, 4
    q, k, v = (rng.normal(size=(L, H, d)) for _ in range(3))
    got = mb.attention(q, k, v, w)
    want = np.zeros_like(got)
    for i in range(L):
        for hd in range(H):
            js = [j for j in range(L) if abs(i - j) <= w]
            s = np.array([q[i, hd] @ k[j, hd] / math.sqrt(d) for j in js])
            p = np.exp(s - s.max())
            p /= p.sum()
            want[i, hd] = sum(pj * v[j, hd] for pj, j in zip(p, js))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)
    # a window wider than the record is full attention
    np.testing.assert_allclose(mb.attention(q, k, v, L), mb.attention(q, k, v, None), rtol=1e-13)


def test_packed_batch_equals_records_alone_and_bf16_reading_is_close():
    cfg = MODERN_TINY
    W = synth.make_weights(cfg, 4, 0.92)
    rb = synth.generate_records(4, np.array([200, 17, 140, 1]), cfg.n_types, cfg.vocab, 8)
    z, _, _ = mb.forward(W, cfg, rb.ids, rb.cu_seqlens)
    for r in range(rb.n_records):
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        z1, _, _ = mb.forward(W, cfg, rb.ids[a:b], np.array([0, b - a]))
        np.testing.assert_allclose(z1, z[a:b], rtol=1e-12, atol=1e-12)
    zq, _, _ = mb.forward(W, cfg, rb.ids, rb.cu_seqlens, Precision("bf16"))
    err = np.abs(zq - z).max() / np.abs(z).max()
    assert 1e-5 < err < 5e-2, err
