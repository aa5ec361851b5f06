"""GPU path vs the FP64 oracle through the C ABI (needs an MI355X).

Bars: FP32 logits within 1e-4 relative per token of the pure oracle; labels
equal wherever the reference margin exceeds 1e-2 (pure oracle for FP32, the
bf16-rounding oracle for BF16); spans, pseudonyms and substituted bytes
bit-exact for integer work.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import encoder, pipeline as opipe, pseudonym as ops, spans as ospans
from synth.configs import TINY, BASE, LARGE, ModelConfig
from oracle import sensitivity
from tests.gpu_common import (MARGIN, FP32_LOGIT_RTOL, LOGIT_BOUND, confident_labels_agree, confident_records,
                              logit_rel_err, make_cache, make_model, oracle_ner, reduced_label_gate, say)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


@pytest.fixture(scope="module")
def tiny_batch():
    return synth.generate_records(64, ("uniform", 16, 128), 4, TINY.vocab, 0)


@pytest.fixture(scope="module")
def tiny_fp32(torch_dev):
    W, m = make_model(TINY, "fp32", 0)
    return W, m


def _run_ner(m, rb, logits=True, window=0, stride=0):
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    db = DeviceBatch(rb)
    pl = Pipeline(m)
    lab, z, mg = pl.ner(db, logits=logits, margin=True, window=window, stride=stride)
    import torch
    torch.cuda.synchronize()
    T = rb.n_tokens
    return lab[:T].cpu().numpy(), (z[:T].cpu().numpy() if z is not None else None), mg[:T].cpu().numpy()


def test_tiny_fp32_hidden_states_layer_by_layer(tiny_fp32, tiny_batch):
    W, m = tiny_fp32
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    db = DeviceBatch(tiny_batch)
    pl = Pipeline(m)
    for nl in range(TINY.n_layers + 1):
        say(f"[tiny fp32] hidden after {nl} layers, T={tiny_batch.n_tokens}")
        h = pl.hidden(db, nl)[: tiny_batch.n_tokens].cpu().numpy()
        ref = encoder.hidden_states(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens, n_layers=nl)
        err = np.abs(h - ref).max()
        assert err < 2e-5 * max(1.0, np.abs(ref).max()), (nl, err)


def test_tiny_fp32_logits_and_labels(tiny_fp32, tiny_batch):
    W, m = tiny_fp32
    say("[tiny fp32] ner_forward logits")
    lab, z, mg = _run_ner(m, tiny_batch)
    zr, lr, mr = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens)
    rel = logit_rel_err(z, zr)
    say(f"  max rel logit err {rel.max():.3e}")
    assert rel.max() <= FP32_LOGIT_RTOL
    bad, n = confident_labels_agree(lab, lr, mr)
    assert len(bad) == 0 and n > 0.8 * len(lr)
    np.testing.assert_allclose(mg, mr, atol=2e-5)


def test_tiny_bf16_matches_rounding_oracle(torch_dev, tiny_batch):
    W, m = make_model(TINY, "bf16", 0)
    say("[tiny bf16] ner_forward vs bf16-rounding oracle")
    lab, z, mg = _run_ner(m, tiny_batch)
    zq, lq, mq = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens, encoder.Precision("bf16"))
    zp, lp, mp = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens)
    err_q = np.abs(z - zq).max()
    err_p = np.abs(z - zp).max()
    say(f"  max |z - z_bf16oracle| {err_q:.3e}   max |z - z_pure| {err_p:.3e}")
    bad, n = confident_labels_agree(lab, lq, mq)
    assert len(bad) == 0, (len(bad), n)
    assert err_q < 5e-3


def test_batch_invariance_alone_vs_packed(tiny_fp32, tiny_batch):
    _, m = tiny_fp32
    say("[tiny fp32] records alone vs packed")
    lab, z, _ = _run_ner(m, tiny_batch)
    for r in [0, 7, 33, 63]:
        sub = tiny_batch.subset([r])
        l1, z1, _ = _run_ner(m, sub)
        a, b = tiny_batch.cu_seqlens[r], tiny_batch.cu_seqlens[r + 1]
        np.testing.assert_array_equal(z1, z[a:b])
        np.testing.assert_array_equal(l1, lab[a:b])


def test_edge_lengths_one_token_and_max_pos(torch_dev):
    cfg = ModelConfig(n_layers=2, hidden=128, n_heads=2, ffn=256, vocab=500, n_labels=9, max_pos=512)
    W, m = make_model(cfg, "fp32", 3)
    for lens in ([1], [512], [1, 512, 2, 129, 128, 127, 64, 65], [300, 1, 1, 1]):
        say(f"[edge fp32] lengths {lens}")
        rb = synth.generate_records(len(lens), np.array(lens), 4, cfg.vocab, 5)
        lab, z, mg = _run_ner(m, rb)
        zr, lr, mr = encoder.forward(W, cfg, rb.ids, rb.cu_seqlens)
        assert logit_rel_err(z, zr).max() <= FP32_LOGIT_RTOL


def test_bf16_attention_length_classes_and_block_counts(torch_dev):
    """BF16 attention streams each record's keys in 64-key tiles (128 in one
    configuration) with a reference that grows every 64 keys, in work items
    of 32*W query rows.  Lengths at and around every tile and item bound, with
    partial and whole last tiles of 1 to 16 32-key blocks, agree with the
    bf16-rounding oracle, and each record alone gives the bits it gives inside
    the packed batch."""
    cfg = ModelConfig(n_layers=2, hidden=128, n_heads=2, ffn=256, vocab=500, n_labels=9, max_pos=512)
    W, m = make_model(cfg, "bf16", 4)
    lens = [1, 31, 32, 33, 64, 96, 127, 128, 129, 160, 255, 256, 257, 320, 383, 384, 385, 448, 511, 512]
    say(f"[edge bf16] lengths {lens}")
    rb = synth.generate_records(len(lens), np.array(lens), 4, cfg.vocab, 6)
    lab, z, mg = _run_ner(m, rb)
    zq, lq, mq = encoder.forward(W, cfg, rb.ids, rb.cu_seqlens, encoder.Precision("bf16"))
    err = np.abs(z - zq).max()
    say(f"  max |z - z_bf16oracle| {err:.3e}")
    assert err < 5e-3
    bad, n = confident_labels_agree(lab, lq, mq)
    assert len(bad) == 0, (len(bad), n)
    for r in (0, 3, 8, 11, 16, 19):
        sub = rb.subset([r])
        l1, z1, _ = _run_ner(m, sub)
        a, b = rb.cu_seqlens[r], rb.cu_seqlens[r + 1]
        np.testing.assert_array_equal(z1, z[a:b], err_msg=f"record of {lens[r]} tokens")
        np.testing.assert_array_equal(l1, lab[a:b])


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_attention_configurations_are_bit_identical(torch_dev, precision):
    """Every attention tile configuration (query rows per item, keys per LDS
    tile, ring stages) gives the same bits on records that span every tile
    and item bound, so the attention autotuner never changes a result; the
    autotuner's pick is one of them."""
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    cfg = ModelConfig(n_layers=2, hidden=256, n_heads=4, ffn=512, vocab=700, n_labels=9, max_pos=512)
    W = synth.make_weights(cfg, 9)
    scales = None
    if precision == "fp8":
        from oracle import calibrate_fp8
        sc, _ = calibrate_fp8.calibrate(cfg, W, ("uniform", 16, 512), n_records=8)
        scales = np.asarray(sc, np.float32).reshape(-1)
    m = api.Model(cfg, synth.weights_blob(cfg, W), precision, act_scales=scales)
    lens = [1, 63, 64, 65, 127, 128, 129, 191, 255, 256, 257, 300, 383, 384, 385, 449, 511, 512]
    rb = synth.generate_records(len(lens), np.array(lens), 4, cfg.vocab, 19)
    names = m.attn_configs()
    say(f"[attn configs] {precision}: {names}")
    ref = None
    for ci in range(len(names)):
        m.set_attn_config(ci)
        lab, z, mg = _run_ner(m, rb)
        if ref is None:
            ref = (lab, z)
        else:
            np.testing.assert_array_equal(z, ref[1], err_msg=names[ci])
            np.testing.assert_array_equal(lab, ref[0], err_msg=names[ci])
    pl = Pipeline(m)
    chosen, times = pl.autotune_attention(DeviceBatch(rb))
    say(f"  autotune picked {names[chosen]}; times {np.round(times, 4).tolist()}")
    assert 0 <= chosen < len(names) and m.attn_config() == chosen
    lab, z, mg = _run_ner(m, rb)
    np.testing.assert_array_equal(z, ref[1])
    m.close()


def test_empty_batch_is_a_no_op(tiny_fp32):
    import torch
    from paper_2606_15650_amd import api
    _, m = tiny_fp32
    say("[empty] ner_forward with T=0")
    cu = torch.zeros(1, dtype=torch.int32, device="cuda")
    api.ner_forward(m, None, cu, 0, 0, None)
    torch.cuda.synchronize()


def test_out_of_range_token_id_is_flagged_not_faulting(tiny_fp32, tiny_batch):
    import torch
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline
    _, m = tiny_fp32
    say("[errors] token id >= vocab")
    api.device_errors(0, clear=True)
    rb = tiny_batch.subset([0, 1])
    rb.ids = rb.ids.copy()
    rb.ids[3] = TINY.vocab + 100
    db = DeviceBatch(rb)
    Pipeline(m).ner(db)
    torch.cuda.synchronize()
    assert api.device_errors(0, clear=True) & api.ERR_TOKEN_ID


def test_windowed_ner_matches_oracle(tiny_fp32):
    W, m = tiny_fp32
    rb = synth.generate_records(5, np.array([40, 200, 130, 64, 65]), 4, TINY.vocab, 9)
    for win, st in ((64, 48), (128, 96)):
        say(f"[tiny fp32] windowed ner window={win} stride={st}")
        lab, z, mg = _run_ner(m, rb, window=win, stride=st)
        zr, lr, mr = opipe.ner(W, TINY, rb.ids, rb.cu_seqlens, window=win, stride=st)
        assert logit_rel_err(z, zr).max() <= FP32_LOGIT_RTOL
        bad, _ = confident_labels_agree(lab, lr, mr)
        assert len(bad) == 0


def test_bf16_windowed_at_the_stream_window(torch_dev):
    """The dataset-scale configuration's windows (512 tokens every 448) on
    records longer than one window (1300, 513, 900 tokens) and one shorter,
    base widths with two layers, against the rounding oracle.  The logit bar
    is twice the spread the oracle itself shows on this very case when its
    inputs to every bf16 rounding move by 1e-7 (the size of FP32 summation
    differences; tests/golden/sensitivity_base2_windowed_bf16.json, written
    by oracle/sensitivity.py): at base widths that spread exceeds the tiny
    models' 5e-3.  Labels must agree wherever the oracle's margin exceeds
    1e-2 (and so above the 2d a deviation of d could flip)."""
    with open(os.path.join(GOLDEN, "sensitivity_base2_windowed_bf16.json")) as f:
        probe = json.load(f)
    case = probe["case"]
    cfg = ModelConfig(n_layers=2, hidden=768, n_heads=12, ffn=3072, vocab=30522, n_labels=17)
    W, m = make_model(cfg, "bf16", case["weight_seed"])
    rb = synth.generate_records(len(case["lengths"]), np.array(case["lengths"]), cfg.n_types, cfg.vocab,
                                case["records_seed"])
    win, st = case["window"], case["stride"]
    say(f"[base-width bf16] windowed ner window={win} stride={st}")
    lab, z, mg = _run_ner(m, rb, window=win, stride=st)
    zq, lq, mq = opipe.ner(W, cfg, rb.ids, rb.cu_seqlens, encoder.Precision("bf16"), window=win, stride=st)
    d = 2.0 * probe["perturbed_vs_rounding_oracle"]["max"]
    err = np.abs(z - zq).max()
    say(f"  max |z - z_bf16oracle| {err:.3e} (bar {d:.3e})")
    bad, n = confident_labels_agree(lab, lq, mq)
    assert len(bad) == 0, (len(bad), n)
    assert err <= d


def _decode_gpu(rb, labels, n_types, span_cap=None):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, spans_to_numpy
    from paper_2606_15650_amd import api
    db = DeviceBatch(rb)
    cap = rb.n_tokens if span_cap is None else span_cap
    lab = torch.from_numpy(np.ascontiguousarray(labels, np.uint8)).cuda()
    spans = torch.empty((max(cap, 1), 3), dtype=torch.int64, device="cuda")
    cu_spans = torch.empty(rb.n_records + 1, dtype=torch.int32, device="cuda")
    ws = torch.empty(api.decode_workspace_size(rb.n_tokens, rb.n_records), dtype=torch.uint8, device="cuda")
    api.decode_spans(lab, db.tok_off, db.cu, rb.n_records, rb.n_tokens, n_types, spans, cap, cu_spans, ws, ws.numel())
    torch.cuda.synchronize()
    cs = cu_spans.cpu().numpy()
    return spans_to_numpy(spans, min(int(cs[-1]), cap)), cs


@pytest.mark.parametrize("kind", ["gold", "random", "all_entity"])
def test_decode_spans_bit_exact(torch_dev, kind):
    rb = synth.generate_records(200, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 21)
    rng = np.random.default_rng(4)
    if kind == "gold":
        lab = rb.gold_labels
    elif kind == "random":
        lab = rng.integers(0, 17, rb.n_tokens).astype(np.uint8)
    else:
        lab = rng.integers(1, 17, rb.n_tokens).astype(np.uint8)
    say(f"[decode] {kind} labels, T={rb.n_tokens}")
    got, cs = _decode_gpu(rb, lab, 8)
    want = ospans.bio_decode(lab, rb.tok_off, rb.cu_seqlens, 8)
    np.testing.assert_array_equal(got, want)
    assert cs[-1] == len(want)
    if kind == "gold":
        np.testing.assert_array_equal(got, rb.gold_spans)


def test_decode_span_capacity_reports_total(torch_dev):
    rb = synth.generate_records(20, ("uniform", 16, 64), 4, 8192, 2)
    lab = np.ones(rb.n_tokens, np.uint8)  # every token a B- label
    say("[decode] span_cap smaller than the span count")
    got, cs = _decode_gpu(rb, lab, 4, span_cap=10)
    assert cs[-1] == rb.n_tokens and len(got) == 10


def _pseudo_gpu(rb, spans, cache, B=None):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list
    from paper_2606_15650_amd import api
    db = DeviceBatch(rb)
    n = len(spans)
    cap = max(n, 1)
    raw = np.zeros((cap, 3), np.int64)
    if n:
        raw[:n, 0] = (spans[:, 0] & 0xFFFFFFFF) | (spans[:, 1] << 32)
        raw[:n, 1] = spans[:, 2]
        raw[:n, 2] = spans[:, 3]
    d_sp = torch.from_numpy(raw).cuda()
    counts = np.bincount(spans[:, 0], minlength=rb.n_records) if n else np.zeros(rb.n_records, np.int64)
    cu_spans = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)).cuda()
    pl = Pipeline.__new__(Pipeline)
    pl.cache, pl.device, pl._ws = cache, torch.device("cuda:0"), {}
    out, cu_out = pl.pseudonymize(db, d_sp, cu_spans, cap)
    torch.cuda.synchronize()
    return outputs_to_list(out, cu_out)


@pytest.mark.parametrize("slug", [0, 10, 64])
def test_pseudonymize_bit_exact_on_gold_spans(torch_dev, slug):
    rb = synth.generate_records(300, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 31)
    cache = make_cache(rb.type_names, slug=slug)
    key = synth.make_key(0)
    say(f"[pseudonymize] gold spans, slug={slug}, spans={len(rb.gold_spans)}")
    got = _pseudo_gpu(rb, rb.gold_spans, cache)
    want = ops.pseudonymize_batch(rb.text, rb.cu_bytes, rb.gold_spans, rb.n_records, rb.type_names, key, slug)
    assert got == want
    # second call: served from the table, same bytes (cache on/off invariance)
    got2 = _pseudo_gpu(rb, rb.gold_spans, cache)
    assert got2 == want
    st = cache.stats()
    if slug:
        assert st["hits"] > 0 and st["entries"] > 0
    cache.set_enabled(False)
    assert _pseudo_gpu(rb, rb.gold_spans, cache) == want


def test_hmac_block_edges(torch_dev):
    """Entity lengths around the SHA-256 padding and block edges, and past the table limit."""
    lens = [0, 1, 2, 31, 32, 55, 56, 57, 63, 64, 65, 96, 97, 119, 120, 128, 200, 300]
    rng = np.random.default_rng(0)
    parts, spans, pos = [], [], 0
    for L in lens:
        e = bytes(rng.integers(33, 127, L).astype(np.uint8))
        parts.append(b"x " + e + b" ")
        spans.append((0, 1, pos + 2, pos + 2 + L))
        pos += L + 3
    text = b"".join(parts)
    rb = synth.records.RecordBatch(text, np.array([0, len(text)]), np.zeros(1, np.int32), np.zeros((1, 2), np.int32),
                                   np.array([0, 1], np.int32), np.zeros(1, np.uint8), np.zeros((0, 4)), ["HASH"])
    sp = np.array(spans, np.int64)
    key = b"\x0b" * 20
    for slug in (64, 7):
        from paper_2606_15650_amd import api
        cache = api.PseudonymCache(key, slug, ["HASH"], 4096)
        say(f"[hmac] {len(lens)} entity lengths, slug={slug}")
        got = _pseudo_gpu(rb, sp, cache)
        want = ops.pseudonymize_batch(text, [0, len(text)], sp, 1, ["HASH"], key, slug)
        assert got == want


def test_long_key_is_hashed_first(torch_dev):
    from paper_2606_15650_amd import api
    key = bytes(range(200))
    text = b"host 10.1.2.3 and web01.corp"
    rb = synth.records.RecordBatch(text, np.array([0, len(text)]), np.zeros(1, np.int32), np.zeros((1, 2), np.int32),
                                   np.array([0, 1], np.int32), np.zeros(1, np.uint8), np.zeros((0, 4)),
                                   ["IP_ADDRESS", "HOSTNAME"])
    sp = np.array([[0, 1, 5, 13], [0, 2, 18, 28]], np.int64)
    cache = api.PseudonymCache(key, 12, ["IP_ADDRESS", "HOSTNAME"], 1024)
    say("[hmac] 200-byte key")
    got = _pseudo_gpu(rb, sp, cache)
    want = ops.pseudonymize_batch(text, [0, len(text)], sp, 1, ["IP_ADDRESS", "HOSTNAME"], key, 12)
    assert got == want


def test_bad_spans_are_skipped_and_flagged(torch_dev):
    from paper_2606_15650_amd import api
    text = b"aaaa bbbb cccc"
    rb = synth.records.RecordBatch(text, np.array([0, len(text)]), np.zeros(1, np.int32), np.zeros((1, 2), np.int32),
                                   np.array([0, 1], np.int32), np.zeros(1, np.uint8), np.zeros((0, 4)), ["T"])
    # second span overlaps the first, third runs past the record: both skipped
    sp = np.array([[0, 1, 0, 4], [0, 1, 2, 6], [0, 1, 10, 99]], np.int64)
    cache = api.PseudonymCache(b"k", 4, ["T"], 1024)
    api.device_errors(0, clear=True)
    say("[pseudonymize] malformed spans")
    got = _pseudo_gpu(rb, sp, cache)
    want = ops.pseudonymize_batch(text, [0, len(text)], sp[:1], 1, ["T"], b"k", 4)
    assert got == want
    assert api.device_errors(0, clear=True) & api.ERR_SPAN


def test_full_path_tiny_fp32_matches_oracle(tiny_fp32, tiny_batch):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list, spans_to_numpy
    W, m = tiny_fp32
    cache = make_cache(tiny_batch.type_names)
    key = synth.make_key(0)
    say("[tiny fp32] whole path: ner -> spans -> pseudonyms")
    db = DeviceBatch(tiny_batch)
    pl = Pipeline(m, cache)
    labels, spans, cu_spans, out, cu_out = pl.step(db)
    torch.cuda.synchronize()
    outs = outputs_to_list(out, cu_out)
    res = opipe.run(W, TINY, tiny_batch, key, 10)
    conf = confident_records(res.margin, tiny_batch.cu_seqlens)
    assert len(conf) > 0
    for r in conf:
        assert outs[r] == res.outputs[r]
    # the integer tail is exact given the GPU's own labels
    lab = labels[: tiny_batch.n_tokens].cpu().numpy()
    res_g = opipe.run(W, TINY, tiny_batch, key, 10, labels_override=lab)
    assert outs == res_g.outputs
    cs = cu_spans.cpu().numpy()
    np.testing.assert_array_equal(spans_to_numpy(spans, int(cs[-1])), res_g.spans)


def test_base_bf16_small_batch_vs_rounding_oracle(torch_dev):
    """12-layer h768 encoder, a few records (incl. 512 tokens), BF16 vs the bf16 oracle."""
    rb = synth.generate_records(6, np.array([512, 37, 200, 16, 129, 300]), 8, BASE.vocab, 17)
    W, m = make_model(BASE, "bf16", 0, o_target=0.92)
    say(f"[base bf16] T={rb.n_tokens}")
    lab, z, mg = _run_ner(m, rb)
    zq, lq, mq = oracle_ner(W, BASE, rb.ids, rb.cu_seqlens, lambda g: encoder.Precision("bf16"))
    zp, lp, mp = oracle_ner(W, BASE, rb.ids, rb.cu_seqlens)
    dev_q, dev_p = np.abs(z - zq).max(), np.abs(z - zp).max()
    bound = LOGIT_BOUND[("bf16", BASE.n_layers)]
    say(f"  max |z-zq| {dev_q:.3e}  max |z-zpure| {dev_p:.3e}  O-rate {(lab == 0).mean():.3f}")
    assert dev_q < bound and dev_p < bound
    reduced_label_gate(lab, zq, lq, mq, lambda sd: _perturbed(W, BASE, rb, "bf16", sd), batch=rb,
                       n_types=BASE.n_types)
    m.close()


def _perturbed(W, cfg, rb, mode, seed, scales=None):
    """The perturbed oracle on a batch (each thread group draws its own stream)."""
    return oracle_ner(W, cfg, rb.ids, rb.cu_seqlens,
                      lambda g: sensitivity.perturbed_precision(mode, 1000 * seed + g, scales))


def _class_sample(L: np.ndarray, per_class: int, seed: int) -> list[int]:
    """Records drawn evenly from the four attention length classes
    (<= 128, <= 256, <= 384, <= 512 tokens), plus the first and last."""
    rng = np.random.default_rng(seed)
    out = {0, len(L) - 1}
    for lo, hi in ((1, 128), (129, 256), (257, 384), (385, 512)):
        idx = np.nonzero((L >= lo) & (L <= hi))[0]
        out.update(rng.choice(idx, min(per_class, len(idx)), replace=False).tolist())
    return sorted(out)


@pytest.mark.timeout(900)
def test_base_bf16_full_batch_sampled_records(torch_dev):
    """The bench's workload and launch configuration (4096 records, autotuned tiles):
    66 records, 16 from each attention length class plus the first and the
    last, are checked against the oracle, alone and inside the batch."""
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list, spans_to_numpy
    wl = synth.workload("base_bf16")
    rb = synth.generate_records(wl.n_records, wl.lengths, BASE.n_types, BASE.vocab, wl.seed)
    W, m = make_model(BASE, "bf16", wl.weight_seed, o_target=wl.o_target)
    cache = make_cache(rb.type_names, capacity=1 << 20)
    pl = Pipeline(m, cache)
    say(f"[base bf16 full] T={rb.n_tokens} B={rb.n_records}: autotune + one step")
    pl.autotune(rb.n_tokens, rb.n_records)
    db = DeviceBatch(rb)
    z_lab, z_full, _ = pl.ner(db, logits=True)
    labels, spans, cu_spans, out, cu_out = pl.step(db)
    torch.cuda.synchronize()
    lab = labels[: rb.n_tokens].cpu().numpy()
    np.testing.assert_array_equal(lab, z_lab[: rb.n_tokens].cpu().numpy())
    outs = outputs_to_list(out, cu_out)
    cs = cu_spans.cpu().numpy()
    sp = spans_to_numpy(spans, int(cs[-1]))
    z_full = z_full[: rb.n_tokens].cpu().numpy()
    sample = _class_sample(np.diff(rb.cu_seqlens), 16, 7)
    sub = rb.subset(sample)
    say(f"  {len(sample)} records, {sub.n_tokens} tokens, lengths {np.diff(sub.cu_seqlens).tolist()}: oracle")
    zq, lq, mq = oracle_ner(W, BASE, sub.ids, sub.cu_seqlens, lambda g: encoder.Precision("bf16"))
    rows = np.concatenate([np.arange(rb.cu_seqlens[r], rb.cu_seqlens[r + 1]) for r in sample])
    dev = np.abs(z_full[rows] - zq).max()
    say(f"  max |z - z_bf16oracle| {dev:.3e} (bound {LOGIT_BOUND[('bf16', BASE.n_layers)]})")
    assert dev < LOGIT_BOUND[("bf16", BASE.n_layers)]
    reduced_label_gate(lab[rows], zq, lq, mq, lambda sd: _perturbed(W, BASE, sub, "bf16", sd), batch=sub,
                       n_types=BASE.n_types)
    key = synth.make_key(0)
    res = opipe.run(W, BASE, sub, key, 10, labels_override=lab[rows])
    for i, r in enumerate(sample):
        # integer tail of this record: exact given the GPU labels
        assert outs[r] == res.outputs[i]
        mine = sp[sp[:, 0] == r].copy()
        mine[:, 0] = i
        np.testing.assert_array_equal(mine, res.spans[res.spans[:, 0] == i])
        # the same record alone gives the same bits as inside the batch
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        l1, z1, _ = _run_ner(m, rb.subset([r]))
        np.testing.assert_array_equal(z1, z_full[a:b], err_msg=f"record {r} ({b - a} tokens)")
    m.close()


def test_base_fp32_small_batch_vs_pure_oracle(torch_dev):
    rb = synth.generate_records(4, np.array([512, 100, 17, 250]), 8, BASE.vocab, 18)
    W, m = make_model(BASE, "fp32", 0, o_target=0.92)
    say(f"[base fp32] T={rb.n_tokens}")
    lab, z, mg = _run_ner(m, rb)
    zr, lr, mr = encoder.forward(W, BASE, rb.ids, rb.cu_seqlens)
    rel = logit_rel_err(z, zr)
    say(f"  max rel logit err {rel.max():.3e}")
    assert rel.max() <= FP32_LOGIT_RTOL
    bad, _ = confident_labels_agree(lab, lr, mr)
    assert len(bad) == 0
    m.close()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_tile_configurations_are_bit_identical(torch_dev, tiny_batch, precision):
    """Every GEMM tile shape (register-staged or LDS-ring kernel) gives the same
    bits (fixed K order): tuning never changes results."""
    scales = None
    if precision == "fp8":
        scales = np.asarray(_fp8_scales("tiny_fp8"), np.float32).reshape(-1)
    W, m = make_model(TINY, precision, 0, act_scales=scales)
    names = m.tile_configs()
    say(f"[tiles] {len(names)} {precision} tile configurations")
    ref = None
    h, f = TINY.hidden, TINY.ffn
    from paper_2606_15650_amd import api
    for ci in range(len(names)):
        tiles = []
        for (N, K) in ((3 * h, h), (h, h), (f, h), (h, f)):
            # use ci where it fits the shape, else the default
            tiles.append(ci if _fits(names[ci], N, K) else -1)
        m.set_tiles(tiles)
        lab, z, _ = _run_ner(m, tiny_batch)
        if ref is None:
            ref = z
        else:
            np.testing.assert_array_equal(z, ref, err_msg=names[ci])
    # the tile order (groups of row blocks) changes no result either
    m.set_tiles([-1] * 4)
    for groups in ([2, 3, 4, 8], [16, 16, 16, 16]):
        m.set_tile_groups(groups)
        lab, z, _ = _run_ner(m, tiny_batch)
        np.testing.assert_array_equal(z, ref, err_msg=str(groups))
        assert m.get_tiles()[1] == groups
    with pytest.raises(RuntimeError):
        m.set_tile_groups([-1, 1, 1, 1])


def _fits(name, N, K):
    # names: <type>_<BM>x<BN>x<BK>_w<WGM>x<WGN>[_s<stages>]
    bm, bn, bk = [int(x) for x in name.split("_")[1].split("x")]
    return N % bn == 0 and K % bk == 0


def _fp8_scales(name):
    import json, os
    from tests.conftest import GOLDEN
    with open(os.path.join(GOLDEN, f"fp8_scales_{name}.json")) as fh:
        return json.load(fh)["scales"]


def test_tiny_fp8_matches_rounding_oracle(torch_dev, tiny_batch):
    sc = _fp8_scales("tiny_fp8")
    W, m = make_model(TINY, "fp8", 0, act_scales=np.asarray(sc, np.float32).reshape(-1))
    say("[tiny fp8] ner_forward vs fp8-rounding oracle")
    lab, z, mg = _run_ner(m, tiny_batch)
    prec = encoder.Precision("fp8", act_scales=sc)
    zq, lq, mq = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens, prec)
    zp, lp, mp = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens)
    err_q = np.abs(z - zq).max()
    say(f"  max |z - z_fp8oracle| {err_q:.3e}   max |z - z_pure| {np.abs(z - zp).max():.3e}  "
        f"label agreement vs pure {(lab == lp).mean():.4f}")
    bad, n = confident_labels_agree(lab, lq, mq)
    assert len(bad) == 0, (len(bad), n)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_classifier_ties_and_margins(torch_dev, tiny_batch, precision):
    """Argmax ties go to the lowest class index with margin 0; margins follow
    the oracle's top-1 minus top-2 (the head is FP32 on every path)."""
    from paper_2606_15650_amd import api
    W = synth.make_weights(TINY, 0)
    W["wc"] = W["wc"].copy()
    W["bc"] = W["bc"].copy()
    # classes 3 and 5: identical head rows and a bias that puts them on top
    W["wc"][:, 5] = W["wc"][:, 3]
    W["bc"][3] = W["bc"][5] = 8.0
    m = api.Model(TINY, synth.weights_blob(TINY, W), precision)
    lab, z, mg = _run_ner(m, tiny_batch)
    say(f"[classifier {precision}] tie: labels {np.unique(lab)}, max margin {mg.max():.3e}")
    assert (lab == 3).all()
    assert (mg == 0).all()
    assert np.array_equal(z[:, 3], z[:, 5])
    m.close()
    # no tie: class 3 alone on top; margins against the oracle's
    W["bc"][5] = 0.0
    m = api.Model(TINY, synth.weights_blob(TINY, W), precision)
    lab, z, mg = _run_ner(m, tiny_batch)
    prec = None if precision == "fp32" else encoder.Precision(precision)
    zr, lr, mr = encoder.forward(W, TINY, tiny_batch.ids, tiny_batch.cu_seqlens, prec)
    assert (lab == 3).all() and (lr == 3).all()
    err = np.abs(mg - mr).max()
    say(f"[classifier {precision}] max |margin - oracle| {err:.3e}")
    assert err <= (1e-4 if precision == "fp32" else 5e-3) * max(1.0, np.abs(zr).max())
    m.close()


FP8_CLASS_LENGTHS = [1, 128, 129, 256, 257, 384, 385, 512]


@pytest.mark.timeout(900)
def test_large_fp8_records_at_every_attention_class_bound(torch_dev):
    """24-layer h1024 encoder with FP8-E4M3 GEMM inputs (the large FP8 workload's
    model and scales): records of 1, 128, 129, 256, 257, 384, 385 and 512
    tokens put the fp8-output attention kernel through all four length
    classes; packed with 8 records of the workload's length distribution and
    autotuned tiles, every record is checked against the FP8-rounding oracle,
    and each alone gives the bits it gives in the batch."""
    wl = synth.workload("large_fp8")
    scales = np.asarray(_fp8_scales("large_fp8"), np.float32).reshape(-1)
    W, m = make_model(LARGE, "fp8", wl.weight_seed, o_target=wl.o_target, act_scales=scales)
    filler = synth.generate_records(8, wl.lengths, LARGE.n_types, LARGE.vocab, wl.seed)
    lens = FP8_CLASS_LENGTHS + np.diff(filler.cu_seqlens).tolist()
    rb = synth.generate_records(len(lens), np.array(lens), LARGE.n_types, LARGE.vocab, wl.seed + 1)
    from paper_2606_15650_amd.pipeline import Pipeline
    Pipeline(m).autotune(rb.n_tokens, rb.n_records)
    say(f"[large fp8] lengths {lens}: GPU, then the oracle")
    lab, z, mg = _run_ner(m, rb)
    bound = LOGIT_BOUND[("fp8", LARGE.n_layers)]
    sc = _fp8_scales("large_fp8")
    zq, lq, mq = oracle_ner(W, LARGE, rb.ids, rb.cu_seqlens, lambda g: encoder.Precision("fp8", act_scales=sc))
    for r, n in enumerate(lens):
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        say(f"  record {r} ({n} tokens): max |z - z_oracle| {np.abs(z[a:b] - zq[a:b]).max():.3e}")
    assert np.abs(z - zq).max() < bound
    reduced_label_gate(lab, zq, lq, mq, lambda sd: _perturbed(W, LARGE, rb, "fp8", sd, sc), batch=rb,
                       n_types=LARGE.n_types)
    for r in range(len(FP8_CLASS_LENGTHS)):
        a, b = int(rb.cu_seqlens[r]), int(rb.cu_seqlens[r + 1])
        l1, z1, _ = _run_ner(m, rb.subset([r]))
        np.testing.assert_array_equal(z1, z[a:b], err_msg=f"record of {lens[r]} tokens")
    m.close()


def test_fp8_attention_length_classes_two_layers(torch_dev):
    """FP8 GEMM inputs at base-like widths reduced to two layers: lengths at and
    around every attention class bound (the fp8-output attention kernel of
    each class) against the FP8-rounding oracle, with static scales from an
    oracle calibration pass of this model, alone and in the batch."""
    from oracle import calibrate_fp8
    cfg = ModelConfig(n_layers=2, hidden=256, n_heads=4, ffn=1024, vocab=3000, n_labels=9, max_pos=512)
    W = synth.make_weights(cfg, 11)
    sc, _ = calibrate_fp8.calibrate(cfg, W, ("uniform", 16, 512), n_records=16)
    from paper_2606_15650_amd import api
    m = api.Model(cfg, synth.weights_blob(cfg, W), "fp8", act_scales=np.asarray(sc, np.float32).reshape(-1))
    lens = [1, 31, 33, 127, 128, 129, 200, 255, 256, 257, 300, 383, 384, 385, 450, 511, 512]
    rb = synth.generate_records(len(lens), np.array(lens), 4, cfg.vocab, 12)
    say(f"[fp8 classes] lengths {lens}")
    lab, z, mg = _run_ner(m, rb)
    zq, lq, mq = oracle_ner(W, cfg, rb.ids, rb.cu_seqlens, lambda g: encoder.Precision("fp8", act_scales=sc))
    err = np.abs(z - zq).max()
    # the bar: twice the oracle's own spread on this case when perturbed by
    # 1e-7 before each bf16 rounding (about 5e-3 here: wider and longer
    # records than the tiny model's)
    runs = {sd: _perturbed(W, cfg, rb, "fp8", sd, sc) for sd in (1, 2, 3)}
    spread = max(np.abs(r[0] - zq).max() for r in runs.values())
    say(f"  max |z - z_fp8oracle| {err:.3e}; perturbed oracle spread {spread:.3e}")
    assert err < 2 * spread
    reduced_label_gate(lab, zq, lq, mq, lambda sd: runs[sd], batch=rb, n_types=4)
    for r in range(len(lens)):
        a, b = rb.cu_seqlens[r], rb.cu_seqlens[r + 1]
        l1, z1, _ = _run_ner(m, rb.subset([r]))
        np.testing.assert_array_equal(z1, z[a:b], err_msg=f"record of {lens[r]} tokens")
    m.close()


def test_record_permutation_and_repeated_runs_are_bit_identical(tiny_fp32, tiny_batch):
    """The batch in another record order gives each record the same logits,
    and running the same batch again gives the same bits."""
    _, m = tiny_fp32
    perm = np.random.default_rng(21).permutation(tiny_batch.n_records)
    lab0, z0, _ = _run_ner(m, tiny_batch)
    lab1, z1, _ = _run_ner(m, tiny_batch)
    assert np.array_equal(z0, z1) and np.array_equal(lab0, lab1)
    pb = tiny_batch.subset(perm.tolist())
    _, zp, _ = _run_ner(m, pb)
    cu, cp = tiny_batch.cu_seqlens, pb.cu_seqlens
    for new, old in enumerate(perm):
        np.testing.assert_array_equal(zp[cp[new]:cp[new + 1]], z0[cu[old]:cu[old + 1]])


@pytest.mark.parametrize("case", ["decreasing", "too_long", "total"])
def test_malformed_cu_seqlens_are_flagged_not_faulting(tiny_fp32, case):
    """Boundaries that are not non-decreasing, a record longer than max_pos
    (no windowing) or a last boundary short of T set the sequence-length
    bit; the kernels clamp and skip, nothing faults, and the next call is
    unaffected."""
    import torch
    from paper_2606_15650_amd import api
    _, m = tiny_fp32
    T = 700
    cu = {"decreasing": [0, 300, 200, 700], "too_long": [0, 50, 50 + TINY.max_pos + 10, 700],
          "total": [0, 100, 300, 650]}[case]
    ids = torch.from_numpy(np.random.default_rng(3).integers(0, TINY.vocab, T, dtype=np.int32)).cuda()
    cu_d = torch.tensor(cu, dtype=torch.int32, device="cuda")
    lab = torch.empty(T, dtype=torch.uint8, device="cuda")
    ws_b = m.workspace_size(T, 3)
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    api.device_errors(0, clear=True)
    say(f"[errors] cu_seqlens {cu}")
    api.ner_forward(m, ids, cu_d, 3, T, lab, None, None, ws, ws_b)
    torch.cuda.synchronize()
    assert api.device_errors(0, clear=True) & api.ERR_SEQLENS
    # the library is still usable
    rb = synth.generate_records(4, ("uniform", 16, 64), TINY.n_types, TINY.vocab, 2)
    _run_ner(m, rb)
    assert api.device_errors(0, clear=True) == 0
