"""The ModernBERT-style encoder on the GPU against its FP64 oracle
(oracle/modernbert.py): FP32 layer by layer and logits, BF16 against the
rounding oracle with the label gate, alone vs packed, the whole NER +
pseudonymize path, and the ModernBERT-base shapes on sampled records."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import modernbert as mb, pipeline as opipe, sensitivity
from oracle.encoder import Precision
from synth.configs import MODERN_BASE, MODERN_TINY
from tests.gpu_common import FP32_LOGIT_RTOL, confident_labels_agree, logit_rel_err, oracle_ner, \
    reduced_label_gate, say

pytestmark = pytest.mark.gpu

# records around the local window (128 wide: 64 keys each side) and the
# attention tile and work-item bounds
LENS = [300, 129, 64, 1, 65, 200, 513, 17, 128, 257]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _model(cfg, precision, seed, o_target=0.92):
    from paper_2606_15650_amd import api
    W = synth.make_weights(cfg, seed, o_target)
    return W, api.ModernModel(cfg, synth.weights_blob(cfg, W), precision)


def _ner(m, rb):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    lab, z, mg = Pipeline(m).ner(DeviceBatch(rb), logits=True)
    torch.cuda.synchronize()
    T = rb.n_tokens
    return lab[:T].cpu().numpy(), z[:T].cpu().numpy(), mg[:T].cpu().numpy()


def _perturbed(W, cfg, rb, seed):
    return oracle_ner(W, cfg, rb.ids, rb.cu_seqlens, lambda g: sensitivity.perturbed_precision("bf16", 1000 * seed + g),
                      forward=mb.forward)


def test_fp32_residual_stream_layer_by_layer(torch_dev):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch
    W, m = _model(MODERN_TINY, "fp32", 3)
    rb = synth.generate_records(len(LENS), np.array(LENS), MODERN_TINY.n_types, MODERN_TINY.vocab, 5)
    db = DeviceBatch(rb)
    ws = torch.empty(m.workspace_size(db.T, db.B), dtype=torch.uint8, device="cuda")
    out = torch.empty((db.T, MODERN_TINY.hidden), dtype=torch.float32, device="cuda")
    for nl in range(MODERN_TINY.n_layers + 1):
        m.hidden(db.ids, db.cu, db.B, db.T, nl, out, ws, ws.numel())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = mb.hidden_states(W, MODERN_TINY, rb.ids, rb.cu_seqlens, n_layers=nl)
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"[modern fp32] after {nl} layers: max rel err {err:.2e}")
        assert err < 1e-5, nl
    m.close()


def test_fp32_logits_and_labels(torch_dev):
    W, m = _model(MODERN_TINY, "fp32", 3)
    rb = synth.generate_records(len(LENS), np.array(LENS), MODERN_TINY.n_types, MODERN_TINY.vocab, 5)
    lab, z, mg = _ner(m, rb)
    zr, lr, mr = mb.forward(W, MODERN_TINY, rb.ids, rb.cu_seqlens)
    rel = logit_rel_err(z, zr)
    say(f"[modern fp32] T={rb.n_tokens}: max rel logit err {rel.max():.2e}, O-rate {(lr == 0).mean():.3f}")
    assert rel.max() <= FP32_LOGIT_RTOL
    bad, n = confident_labels_agree(lab, lr, mr)
    assert len(bad) == 0 and n > 0
    m.close()


def test_bf16_against_the_rounding_oracle_alone_and_packed(torch_dev):
    """BF16 against the oracle that rounds where the GPU stores; the logit
    bar is twice the oracle's own spread when every value it rounds moves by
    1e-7 first (3 seeds); labels as the 1e-2 gate; each record alone gives
    the bits it gives in the batch."""
    W, m = _model(MODERN_TINY, "bf16", 4)
    rb = synth.generate_records(len(LENS), np.array(LENS), MODERN_TINY.n_types, MODERN_TINY.vocab, 6)
    lab, z, mg = _ner(m, rb)
    zq, lq, mq = mb.forward(W, MODERN_TINY, rb.ids, rb.cu_seqlens, Precision("bf16"))
    runs = {sd: _perturbed(W, MODERN_TINY, rb, sd) for sd in (1, 2, 3)}
    spread = max(np.abs(r[0] - zq).max() for r in runs.values())
    err = np.abs(z - zq).max()
    zp, _, _ = mb.forward(W, MODERN_TINY, rb.ids, rb.cu_seqlens)
    say(f"[modern bf16] max |z - z_bf16oracle| {err:.3e} (perturbed spread {spread:.3e}); "
        f"vs pure {np.abs(z - zp).max():.3e}")
    assert err < max(2 * spread, 1e-3)
    reduced_label_gate(lab, zq, lq, mq, lambda sd: runs[sd], batch=rb, n_types=MODERN_TINY.n_types)
    for r in (0, 1, 3, 6):
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        l1, z1, _ = _ner(m, rb.subset([r]))
        np.testing.assert_array_equal(z1, z[a:b], err_msg=f"record of {LENS[r]} tokens")
    m.close()


def test_attention_configurations_agree_with_windows(torch_dev):
    """The windowed attention of every attention tile configuration gives the
    same bits (the local layers skip tiles outside an item's band)."""
    W, m = _model(MODERN_TINY, "bf16", 7)
    rb = synth.generate_records(len(LENS), np.array(LENS), MODERN_TINY.n_types, MODERN_TINY.vocab, 9)
    ref = None
    for ci in range(len(m.attn_configs())):
        m.set_tiles([-1] * 5, ci)
        lab, z, mg = _ner(m, rb)
        if ref is None:
            ref = z
        np.testing.assert_array_equal(z, ref, err_msg=m.attn_configs()[ci])
    m.close()


def test_full_path_on_gpu_labels_matches_oracle_tail(torch_dev):
    import torch
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list, spans_to_numpy
    W, m = _model(MODERN_TINY, "bf16", 4)
    rb = synth.generate_records(40, ("uniform", 16, 300), MODERN_TINY.n_types, MODERN_TINY.vocab, 11)
    key = synth.make_key(0)
    cache = api.PseudonymCache(key, 10, rb.type_names, 1 << 14)
    pl = Pipeline(m, cache)
    labels, spans, cu_spans, out, cu_out = pl.step(DeviceBatch(rb))
    torch.cuda.synchronize()
    lab = labels[:rb.n_tokens].cpu().numpy()
    res = opipe.run(W, MODERN_TINY, rb, key, 10, labels_override=lab)
    say(f"[modern path] {int(cu_spans[-1])} spans over {rb.n_records} records")
    assert outputs_to_list(out, cu_out) == res.outputs
    np.testing.assert_array_equal(spans_to_numpy(spans, int(cu_spans.cpu()[-1])), res.spans)
    cache.close()
    m.close()


def test_modernbert_base_sampled_records(torch_dev):
    """ModernBERT-base shapes (22 layers, h768, GeGLU 1152, vocab 50368): a
    packed batch of records around the window and tile bounds against the
    rounding oracle, with the logit bar twice the perturbed oracle's spread."""
    W, m = _model(MODERN_BASE, "bf16", 0)
    lens = [512, 37, 200, 129, 300, 65, 1, 450]
    rb = synth.generate_records(len(lens), np.array(lens), MODERN_BASE.n_types, MODERN_BASE.vocab, 21)
    say(f"[modern base] lengths {lens}: GPU, then the oracle")
    lab, z, mg = _ner(m, rb)
    zq, lq, mq = oracle_ner(W, MODERN_BASE, rb.ids, rb.cu_seqlens, lambda g: Precision("bf16"), forward=mb.forward)
    runs = {sd: _perturbed(W, MODERN_BASE, rb, sd) for sd in (1, 2, 3)}
    spread = max(np.abs(r[0] - zq).max() for r in runs.values())
    err = np.abs(z - zq).max()
    say(f"  max |z - z_bf16oracle| {err:.3e} (perturbed spread {spread:.3e}), O-rate {(lq == 0).mean():.3f}")
    assert err < 2 * spread
    reduced_label_gate(lab, zq, lq, mq, lambda sd: runs[sd], batch=rb, n_types=MODERN_BASE.n_types)
    m.close()
