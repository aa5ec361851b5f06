"""Pins for span decoding, windows and pseudonyms in the oracle (CPU only)."""
import json
import os
import re

import numpy as np
import pytest

import synth
from oracle import pseudonym, spans
from tests.conftest import GOLDEN


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


BIO = _load("bio_cases.json")


@pytest.mark.parametrize("case", BIO["cases"], ids=[c["name"] for c in BIO["cases"]])
def test_bio_hand_made_cases(case):
    n = len(case["labels"])
    off = np.array([[3 * i, 3 * i + 2] for i in range(n)], dtype=np.int64).reshape(-1, 2)
    got = spans.bio_decode_record(np.array(case["labels"], dtype=np.int64), off, BIO["n_types"])
    want = [(t, 3 * a, 3 * b + 2) for (t, a, b) in case["spans"]]
    assert got == want


def test_bio_rejects_out_of_range_label():
    with pytest.raises(ValueError):
        spans.bio_decode_record(np.array([5]), np.array([[0, 1]]), 2)


@pytest.mark.parametrize("n_types,seed", [(4, 0), (8, 1)])
def test_gold_labels_round_trip_to_gold_spans(n_types, seed):
    rb = synth.generate_records(48, ("uniform", 16, 300), n_types, 8192, seed)
    got = spans.bio_decode(rb.gold_labels, rb.tok_off, rb.cu_seqlens, n_types)
    np.testing.assert_array_equal(got, rb.gold_spans)
    # and the gold spans are exactly the generator's entity strings
    for r, t, b, e in got[:50].tolist():
        txt = rb.record_text(r)[b:e]
        assert len(txt) > 0 and not txt.startswith(b" ") and not txt.endswith(b" ")


@pytest.mark.parametrize("n,count", [(1, 1), (512, 1), (513, 2), (960, 2), (961, 3), (1000, 3), (2000, 5)])
def test_window_count(n, count):
    st = spans.window_starts(n, 512, 448)
    assert len(st) == count
    assert st[-1] < n and st[-1] + 512 >= n
    assert all(b - a == 448 for a, b in zip(st, st[1:]))


def test_owner_window_splits_overlap_in_half():
    n = 1000
    st = spans.window_starts(n, 512, 448)
    own = spans.owner_window(n, 512, 448)
    # every token lies inside its owner window
    for i in range(n):
        k = own[i]
        assert st[k] <= i < st[k] + 512
    # overlap [448, 512): first 32 tokens to window 0, last 32 to window 1
    assert (own[448:480] == 0).all() and (own[480:512] == 1).all()
    assert (own[896:928] == 1).all() and (own[928:] == 2).all()
    assert np.all(np.diff(own) >= 0)


def test_short_record_window_table_is_identity():
    cu = np.array([0, 10, 522, 522 + 1000])
    w = spans.windows(cu, 512, 448)
    assert w.tolist() == [[0, 0, 10], [1, 0, 512], [2, 0, 512], [2, 448, 512], [2, 896, 104]]


HM = _load("hmac_sha256_rfc4231.json")


@pytest.mark.parametrize("v", HM["vectors"], ids=[v["case"] for v in HM["vectors"]])
def test_hmac_rfc4231_vectors(v):
    assert pseudonym.hmac_hex(bytes.fromhex(v["key_hex"]), bytes.fromhex(v["data_hex"])) == v["hmac_sha256"]


FMT = _load("pseudonym_format.json")


def test_pseudonym_shape_of_paper_example():
    key = synth.make_key(0)
    p = pseudonym.pseudonym(FMT["type"], key, FMT["entity"].encode(), FMT["slug_len"]).decode()
    assert re.match(FMT["regex"], p)
    assert re.match(FMT["regex"], FMT["example_output"])
    assert len(p) == len(FMT["example_output"])


@pytest.mark.parametrize("n", [0, 1, 10, 63, 64])
def test_slug_lengths(n):
    key = b"k" * 32
    p = pseudonym.pseudonym("HOSTNAME", key, b"web01.corp", n).decode()
    if n == 0:
        assert p == "[HOSTNAME]"
    else:
        assert re.match(r"^\[HOSTNAME_[0-9a-f]{%d}\]$" % n, p)
        assert p[10:-1] == pseudonym.hmac_hex(key, b"web01.corp")[:n]


def test_slug_length_out_of_range():
    with pytest.raises(ValueError):
        pseudonym.pseudonym("X", b"k", b"e", 65)


def test_same_entity_same_pseudonym_across_records_and_batches():
    key = synth.make_key(3)
    text = b"Host: 10.0.0.1\nIP: 10.0.0.1 and 10.0.0.2"
    out = pseudonym.pseudonymize_batch(text + text, [0, len(text), 2 * len(text)],
                                       np.array([[0, 1, 6, 14], [0, 1, 19, 27], [1, 1, 6, 14], [0, 1, 32, 40]]),
                                       2, ["IP_ADDRESS"], key, 10)
    a = pseudonym.pseudonym("IP_ADDRESS", key, b"10.0.0.1", 10)
    b = pseudonym.pseudonym("IP_ADDRESS", key, b"10.0.0.2", 10)
    assert out[0] == b"Host: " + a + b"\nIP: " + a + b" and " + b
    assert out[1].startswith(b"Host: " + a)
    assert a != b


def test_output_length_identity_and_unchanged_bytes():
    key = synth.make_key(0)
    rb = synth.generate_records(20, ("uniform", 16, 200), 8, 30522, 4)
    outs = pseudonym.pseudonymize_batch(rb.text, rb.cu_bytes, rb.gold_spans, rb.n_records, rb.type_names, key, 10)
    for r in range(rb.n_records):
        sp = rb.gold_spans[rb.gold_spans[:, 0] == r]
        plen = sum(len(rb.type_names[t - 1]) + 3 + 10 for t in sp[:, 1])
        assert len(outs[r]) == len(rb.record_text(r)) - int((sp[:, 3] - sp[:, 2]).sum()) + plen
        if len(sp) == 0:
            assert outs[r] == rb.record_text(r)


def test_substitute_rejects_overlapping_spans():
    with pytest.raises(ValueError):
        pseudonym.substitute(b"abcdef", [(1, 0, 3), (1, 2, 4)], ["T"], b"k", 4)


def test_confident_spans_hand_made():
    # one record of 8 tokens, two types: spans at tokens 1-2 (type 1), 4 (type 2), 7 (type 1)
    lab = np.array([0, 1, 2, 0, 3, 0, 0, 1])
    off = np.array([[3 * i, 3 * i + 2] for i in range(8)])
    cu = np.array([0, 8])
    sp = spans.bio_decode(lab, off, cu, 2)
    assert sp.tolist() == [[0, 1, 3, 8], [0, 2, 12, 14], [0, 1, 21, 23]]
    margin = np.ones(8)
    margin[5] = 1e-3  # the token after the second span
    got = spans.confident_spans(sp, margin, off, cu)
    # the last span has no token after it inside the record
    assert got == [(0, 1, 3, 8), (0, 1, 21, 23)]
    assert spans.confident_spans(sp, margin, off, cu, exclude=[0]) == [(0, 1, 21, 23)]


def test_confident_span_gate_only_sees_confident_disagreements():
    """Brute force over random label pairs: labels that differ only on
    unconfident tokens never fail the gate; a difference on a confident token
    inside or next to a confident span does."""
    rng = np.random.default_rng(5)
    n_types = 3
    caught = 0
    for trial in range(300):
        lens = rng.integers(1, 12, 4)
        cu = np.concatenate([[0], np.cumsum(lens)])
        T = int(cu[-1])
        off = np.zeros((T, 2), dtype=np.int64)
        for r in range(4):
            k = np.arange(lens[r])
            off[cu[r]:cu[r + 1], 0], off[cu[r]:cu[r + 1], 1] = 3 * k, 3 * k + 2
        ref = rng.integers(0, 2 * n_types + 1, T)
        margin = np.where(rng.random(T) < 0.3, 1e-3, 1.0)
        other = ref.copy()
        soft = np.nonzero(margin <= 1e-2)[0]
        other[soft] = rng.integers(0, 2 * n_types + 1, len(soft))
        g = spans.confident_span_gate(other, ref, margin, off, cu, n_types)
        assert not g["missing_in_a"] and not g["missing_in_ref"], trial
        # change one confident token
        hard = np.nonzero(margin > 1e-2)[0]
        if len(hard):
            t = int(rng.choice(hard))
            other[t] = (ref[t] + 1 + rng.integers(0, 2 * n_types)) % (2 * n_types + 1)
            g = spans.confident_span_gate(other, ref, margin, off, cu, n_types)
            caught += bool(g["missing_in_a"] or g["missing_in_ref"])
    assert caught > 100
