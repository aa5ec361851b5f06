"""Pins for the composed oracle pipeline and the seeded generator (CPU only)."""
import numpy as np

import synth
from oracle import encoder, pipeline, spans
from synth.configs import TINY


def test_windowed_path_equals_plain_path_for_short_records():
    W = synth.make_weights(TINY, 1)
    rb = synth.generate_records(6, ("uniform", 16, 60), 4, TINY.vocab, 2)
    z0, l0, _ = pipeline.ner(W, TINY, rb.ids, rb.cu_seqlens)
    z1, l1, _ = pipeline.ner(W, TINY, rb.ids, rb.cu_seqlens, window=64, stride=48)
    np.testing.assert_array_equal(z0, z1)
    np.testing.assert_array_equal(l0, l1)


def test_windowed_labels_come_from_owner_window():
    W = synth.make_weights(TINY, 1)
    rb = synth.generate_records(2, ("uniform", 150, 170), 4, TINY.vocab, 3)
    win, st = 64, 48
    z, _, _ = pipeline.ner(W, TINY, rb.ids, rb.cu_seqlens, window=win, stride=st)
    for r in range(2):
        a = int(rb.cu_seqlens[r]); n = int(rb.cu_seqlens[r + 1]) - a
        starts = spans.window_starts(n, win, st)
        own = spans.owner_window(n, win, st)
        for k, s in enumerate(starts):
            m = min(win, n - s)
            zk, _, _ = encoder.forward(W, TINY, rb.ids[a + s:a + s + m], np.array([0, m]))
            for i in np.nonzero(own == k)[0]:
                np.testing.assert_allclose(z[a + i], zk[i - s], rtol=1e-12, atol=1e-14)


def test_pipeline_outputs_replace_exactly_the_decoded_spans():
    W = synth.make_weights(TINY, 0)
    rb = synth.generate_records(8, ("uniform", 16, 128), 4, TINY.vocab, 0)
    key = synth.make_key(0)
    res = pipeline.run(W, TINY, rb, key, 10)
    assert len(res.outputs) == rb.n_records
    for r in range(rb.n_records):
        sp = res.spans[res.spans[:, 0] == r]
        txt = rb.record_text(r)
        if len(sp) == 0:
            assert res.outputs[r] == txt
        # text before the first span is untouched
        if len(sp):
            assert res.outputs[r][: sp[0, 2]] == txt[: sp[0, 2]]


def test_gold_labels_through_pipeline_replace_all_gold_entities():
    W = synth.make_weights(TINY, 0)
    rb = synth.generate_records(10, ("uniform", 30, 120), 4, TINY.vocab, 5)
    key = synth.make_key(0)
    res = pipeline.run(W, TINY, rb, key, 10, labels_override=rb.gold_labels)
    for r, t, b, e in rb.gold_spans.tolist():
        assert rb.record_text(r)[b:e] not in res.outputs[r] or rb.record_text(r).count(rb.record_text(r)[b:e]) > 1


def test_generator_is_seeded_and_shaped():
    a = synth.generate_records(32, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 11)
    b = synth.generate_records(32, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 11)
    assert a.text == b.text and np.array_equal(a.ids, b.ids)
    lens = np.diff(a.cu_seqlens)
    assert lens.min() >= 16 and lens.max() <= 512
    assert a.ids.min() >= 4 and a.ids.max() < 30522
    # token offsets re-slice to the token text and never cross whitespace
    for r in range(a.n_records):
        txt = a.record_text(r)
        t0, t1 = a.cu_seqlens[r], a.cu_seqlens[r + 1]
        for (tb, te) in a.tok_off[t0:t1][:40]:
            piece = txt[tb:te]
            assert 0 < len(piece) <= 8 and not any(c in b" \n\t" for c in piece)
        assert a.tok_off[t1 - 1, 1] == len(txt)


def test_generator_entity_density_near_eight_percent():
    rb = synth.generate_records(400, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 0)
    d = (rb.gold_labels > 0).mean()
    assert 0.05 < d < 0.12, d


def test_tokenizer_ids_are_fnv1a():
    ids, off = synth.tokenize(b"Host: 10.0.0.1 abcdefghijk", 1000)
    pieces = [b"Host", b":", b"10", b".", b"0", b".", b"0", b".", b"1", b"abcdefgh", b"ijk"]
    assert [bytes(b"Host: 10.0.0.1 abcdefghijk"[a:b]) for a, b in off] == pieces
    assert ids.tolist() == [4 + synth.fnv1a32(p) % 996 for p in pieces]
    # FNV-1a-32 reference values: empty string -> offset basis; "a" -> 0xe40c292c
    assert synth.fnv1a32(b"") == 0x811C9DC5 and synth.fnv1a32(b"a") == 0xE40C292C
