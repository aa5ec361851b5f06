"""Pins for the FP64 encoder oracle (CPU only).

Each check compares the oracle with something other than itself: closed forms
of LayerNorm and softmax, a brute-force attention loop, torch's own
TransformerEncoderLayer in float64 (the textbook post-LN encoder layer), erf
from the math module, and torch's bfloat16 / float8_e4m3fn casts.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import encoder
from oracle.numerics import round_bf16, round_e4m3
from synth.configs import ModelConfig, TINY


def test_layernorm_constant_row_gives_shift():
    g = np.linspace(0.5, 1.5, 16)
    b = np.linspace(-1, 1, 16)
    y = np.full((3, 16), 7.25)
    np.testing.assert_allclose(encoder.layer_norm(y, g, b, 1e-5), np.broadcast_to(b, (3, 16)), atol=1e-12)


def test_layernorm_plus_minus_row_closed_form():
    a, eps = 0.3, 1e-5
    g = np.linspace(0.5, 1.5, 8)
    b = np.linspace(-1, 1, 8)
    y = np.array([[a, -a] * 4])
    # mean 0, population variance a^2
    want = g * y / math.sqrt(a * a + eps) + b
    np.testing.assert_allclose(encoder.layer_norm(y, g, b, eps), want, rtol=1e-13)


def test_layernorm_uses_population_variance():
    y = np.array([[1.0, 2.0, 3.0, 4.0]])
    out = encoder.layer_norm(y, np.ones(4), np.zeros(4), 0.0)
    np.testing.assert_allclose(out, (y - 2.5) / math.sqrt(1.25), rtol=1e-13)


def test_softmax_rows_sum_to_one():
    rng = np.random.default_rng(1)
    s = rng.normal(0, 5, (7, 33))
    p = encoder.softmax_rows(s)
    assert np.all(np.abs(p.sum(-1) - 1) < 1e-12)
    assert np.all(p > 0)


def test_attention_with_constant_values_returns_them():
    rng = np.random.default_rng(2)
    q, k = rng.normal(size=(2, 11, 3, 8))
    v = np.ones((11, 3, 8))
    np.testing.assert_allclose(encoder.attention(q, k, v), v, rtol=1e-13)


def test_attention_length_one_returns_v():
    rng = np.random.default_rng(3)
    q, k, v = rng.normal(size=(3, 1, 4, 16))
    np.testing.assert_allclose(encoder.attention(q, k, v), v, rtol=1e-13)


@pytest.mark.parametrize("L", [1, 2, 5, 8])
def test_attention_matches_triple_loop(L):
    rng = np.random.default_rng(L)
    H, d = 2, 4
    q, k, v = rng.normal(size=(3, L, H, d))
    want = np.zeros((L, H, d))
    for h in range(H):
        for i in range(L):
            s = [sum(q[i, h, c] * k[j, h, c] for c in range(d)) / math.sqrt(d) for j in range(L)]
            m = max(s)
            e = [math.exp(x - m) for x in s]
            tot = sum(e)
            for c in range(d):
                want[i, h, c] = sum(e[j] * v[j, h, c] for j in range(L)) / tot
    np.testing.assert_allclose(encoder.attention(q, k, v), want, rtol=1e-12, atol=1e-14)


def test_gelu_against_math_erf():
    xs = np.linspace(-6, 6, 97)
    want = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    np.testing.assert_allclose(encoder.gelu(xs), want, rtol=1e-14, atol=1e-300)
    assert encoder.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(encoder.gelu(np.array([30.0])), [30.0], rtol=1e-15)
    assert abs(encoder.gelu(np.array([-30.0]))[0]) < 1e-100


def _torch_layer(W, cfg, l):
    h = cfg.hidden
    layer = torch.nn.TransformerEncoderLayer(
        d_model=h, nhead=cfg.n_heads, dim_feedforward=cfg.ffn, dropout=0.0, activation="gelu",
        layer_norm_eps=cfg.ln_eps, batch_first=True, norm_first=False).double().eval()
    p = f"l{l}."
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    with torch.no_grad():
        layer.self_attn.in_proj_weight.copy_(t(W[p + "wqkv"]).T)
        layer.self_attn.in_proj_bias.copy_(t(W[p + "bqkv"]))
        layer.self_attn.out_proj.weight.copy_(t(W[p + "wo"]).T)
        layer.self_attn.out_proj.bias.copy_(t(W[p + "bo"]))
        layer.linear1.weight.copy_(t(W[p + "w1"]).T)
        layer.linear1.bias.copy_(t(W[p + "b1"]))
        layer.linear2.weight.copy_(t(W[p + "w2"]).T)
        layer.linear2.bias.copy_(t(W[p + "b2"]))
        layer.norm1.weight.copy_(t(W[p + "ln1_g"]))
        layer.norm1.bias.copy_(t(W[p + "ln1_b"]))
        layer.norm2.weight.copy_(t(W[p + "ln2_g"]))
        layer.norm2.bias.copy_(t(W[p + "ln2_b"]))
    return layer


SMALL = ModelConfig(n_layers=2, hidden=64, n_heads=4, ffn=128, vocab=500, n_labels=9, max_pos=64)


def test_whole_encoder_matches_torch_float64_per_record():
    """Embedding + post-LN layers + head vs torch modules in float64, one record at a time."""
    W = synth.make_weights(SMALL, seed=5)
    rng = np.random.default_rng(5)
    lens = [1, 7, 33, 64]
    ids = rng.integers(4, SMALL.vocab, sum(lens)).astype(np.int32)
    cu = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    z, labels, margin = encoder.forward(W, SMALL, ids, cu)
    layers = [_torch_layer(W, SMALL, l) for l in range(SMALL.n_layers)]
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    for r in range(len(lens)):
        a, b = cu[r], cu[r + 1]
        with torch.no_grad():
            x = torch.nn.functional.embedding(torch.from_numpy(ids[a:b].astype(np.int64)), t(W["tok_emb"]))
            x = x + t(W["pos_emb"])[: b - a]
            x = torch.nn.functional.layer_norm(x, (SMALL.hidden,), t(W["emb_ln_g"]), t(W["emb_ln_b"]), SMALL.ln_eps)
            x = x[None]
            for layer in layers:
                x = layer(x)
            zt = torch.nn.functional.linear(x[0], t(W["wc"]).T, t(W["bc"])).numpy()
        np.testing.assert_allclose(z[a:b], zt, rtol=1e-10, atol=1e-12)
        np.testing.assert_array_equal(labels[a:b], np.argmax(zt, -1))


def test_packed_batch_equals_records_one_by_one():
    W = synth.make_weights(SMALL, seed=6)
    rng = np.random.default_rng(6)
    lens = [5, 1, 17, 40, 2]
    ids = rng.integers(4, SMALL.vocab, sum(lens)).astype(np.int32)
    cu = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    zp, _, _ = encoder.forward(W, SMALL, ids, cu)
    for r in range(len(lens)):
        a, b = cu[r], cu[r + 1]
        zr, _, _ = encoder.forward(W, SMALL, ids[a:b], np.array([0, b - a]))
        # BLAS may block a packed product differently: equal up to float64 rounding
        np.testing.assert_allclose(zp[a:b], zr, rtol=1e-12, atol=1e-14)


def test_argmax_ties_take_lowest_index_and_margin():
    z = np.array([[0.5, 2.0, 2.0, -1.0], [3.0, 1.0, 2.5, 0.0], [1.0, 1.0, 1.0, 1.0]])
    lab, m = encoder.argmax_margin(z)
    np.testing.assert_array_equal(lab, [1, 0, 0])
    np.testing.assert_allclose(m, [0.0, 0.5, 0.0])


def test_round_bf16_matches_torch_cast():
    rng = np.random.default_rng(7)
    x32 = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 5000), rng.normal(0, 300, 5000),
                          [0.0, 1.0, -2.5, 1.00390625, 1.01171875, 65504.0]]).astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x32.astype(np.float64)), want)


def test_round_e4m3_matches_torch_cast_in_range():
    rng = np.random.default_rng(8)
    x32 = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(0, 0.01, 5000),
                          rng.normal(0, 1, 5000), [0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 0.001953125 * 1.5]])
    x32 = x32.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_e4m3(x32.astype(np.float64)), want)
    assert round_e4m3(np.array([1000.0, -1e6]))[0] == 448.0


def test_bf16_reading_is_close_to_pure_and_idempotent_storage():
    W = synth.make_weights(TINY, seed=0)
    rb = synth.generate_records(6, ("uniform", 16, 64), 4, TINY.vocab, 3)
    zp, _, _ = encoder.forward(W, TINY, rb.ids, rb.cu_seqlens)
    zq, _, _ = encoder.forward(W, TINY, rb.ids, rb.cu_seqlens, encoder.Precision("bf16"))
    err = np.abs(zq - zp).max()
    assert 1e-5 < err < 5e-2, err
    x = round_bf16(np.random.default_rng(0).normal(size=1000))
    np.testing.assert_array_equal(round_bf16(x), x)


def test_positions_restart_per_record():
    np.testing.assert_array_equal(encoder.positions(np.array([0, 3, 3, 5])), [0, 1, 2, 0, 1])


def test_rounded_probabilities_reference_is_a_power_of_two():
    """The reduced-precision reading rounds p = 2^(s log2 e - c) with c the
    smallest integer at or above max(s) log2 e.  Pins: (1) with no rounding it
    is softmax itself (the reference cancels); (2) any larger integer
    reference rounds to the same values times the power of two (so a
    single pass whose reference grows reaches the same rounded p); (3) a
    non-integer reference would not (the rounding point really moves);
    (4) the largest rounded p lies in [1/2, 1]."""
    rng = np.random.default_rng(5)
    L, H, d = 37, 3, 16
    q, k, v = (rng.normal(size=(L, H, d)) for _ in range(3))
    ident = encoder.attention(q, k, v, round_p=lambda p: p)
    np.testing.assert_allclose(ident, encoder.attention(q, k, v), rtol=1e-12, atol=1e-14)
    s = rng.normal(scale=3.0, size=(200, 64))
    x = s / np.log(2.0)
    c = np.ceil(x.max(axis=-1, keepdims=True))
    p0 = round_bf16(np.exp2(x - c))
    assert (p0.max(axis=-1) >= 0.5).all() and (p0.max(axis=-1) <= 1.0).all()
    for shift in (1, 7, 40):
        np.testing.assert_array_equal(round_bf16(np.exp2(x - (c + shift))) * 2.0 ** shift, p0)
    moved = round_bf16(np.exp2(x - (c + 0.37))) * 2.0 ** 0.37
    assert (np.abs(moved - p0) > 0).mean() > 0.3
