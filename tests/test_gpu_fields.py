"""GPU parity of the schema-aware whole-field path (field_spans) against the
oracle: spans and substituted bytes bit-exact."""
import random

import numpy as np
import pytest

import synth
from oracle import fields as F, pseudonym as ops
from synth.records import TYPE_NAMES_17, RecordBatch, _FIELD_OF
from tests.gpu_common import make_cache, say

pytestmark = pytest.mark.gpu

CONFIG = {name.encode(): TYPE_NAMES_17.index(t) + 1 for t, names in _FIELD_OF.items() for name in names}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _text_batch(records, type_names):
    cu = np.concatenate([[0], np.cumsum([len(r) for r in records])]).astype(np.int64)
    B = len(records)
    return RecordBatch(b"".join(records), cu, np.zeros(0, np.int32), np.zeros((0, 2), np.int32),
                       np.zeros(B + 1, np.int32), np.zeros(0, np.uint8), np.zeros((0, 4), np.int64), list(type_names))


def _pipeline(cache, n_types):
    import torch
    from paper_2606_15650_amd.pipeline import Pipeline
    pl = Pipeline.__new__(Pipeline)
    pl.cache, pl.device, pl._ws, pl.n_types = cache, torch.device("cuda:0"), {}, n_types
    return pl


def _fields_gpu(rb, cache, config, span_cap=None):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, spans_to_numpy
    db = DeviceBatch(rb)
    pl = _pipeline(cache, len(rb.type_names))
    spans, cu, cap = pl.fields(db, config, span_cap=span_cap)
    torch.cuda.synchronize()
    cu_h = cu.cpu().numpy().astype(np.int64)
    arr = spans_to_numpy(spans, int(min(cu_h[-1], cap)))
    out = []
    for b in range(rb.n_records):
        rows = arr[cu_h[b]:min(cu_h[b + 1], len(arr))]
        assert (rows[:, 0] == b).all()
        out.append([(int(t), int(s), int(e)) for _, t, s, e in rows])
    return cu_h, out


def test_field_spans_on_generated_records(torch_dev):
    rb = synth.generate_records(400, ("lognormal", 5.2, 0.6, 16, 512), len(TYPE_NAMES_17), 30522, 21)
    cache = make_cache(rb.type_names)
    say(f"[fields] {rb.n_records} records, {len(rb.text)} bytes")
    _, got = _fields_gpu(rb, cache, CONFIG)
    want = F.field_spans_batch(rb.text, rb.cu_bytes, CONFIG)
    assert sum(map(len, want)) > 300
    assert got == want


def test_field_spans_on_adversarial_lines(torch_dev):
    """Lines built from names, colons, spaces and breaks, records that end
    mid-line and empty records."""
    pieces = [b"Host", b"IP", b": ", b":", b" ", b"\n", b"x", b"See Also", b"a:b", b"1.2", b"\n\n", b"Port", b"MAC",
              b"Hash: ", b"Host: 10.0.0.1"]
    rng = random.Random(3)
    recs = [b"" if i % 23 == 0 else b"".join(rng.choice(pieces) for _ in range(rng.randint(1, 30)))
            for i in range(500)]
    rb = _text_batch(recs, TYPE_NAMES_17)
    cache = make_cache(TYPE_NAMES_17)
    _, got = _fields_gpu(rb, cache, CONFIG)
    want = F.field_spans_batch(rb.text, rb.cu_bytes, CONFIG)
    assert sum(map(len, want)) > 200
    assert got == want


def test_field_path_substitution_matches_oracle(torch_dev):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, outputs_to_list
    rb = synth.generate_records(200, ("lognormal", 5.2, 0.6, 16, 512), len(TYPE_NAMES_17), 30522, 22)
    cache = make_cache(rb.type_names)
    pl = _pipeline(cache, len(rb.type_names))
    db = DeviceBatch(rb)
    _, _, out, cu_out = pl.step_fields(db, CONFIG)
    torch.cuda.synchronize()
    got = outputs_to_list(out, cu_out)
    key = synth.make_key(0)
    want = [ops.substitute(rb.text[int(rb.cu_bytes[b]):int(rb.cu_bytes[b + 1])], sp, rb.type_names, key, cache.slug)
            for b, sp in enumerate(F.field_spans_batch(rb.text, rb.cu_bytes, CONFIG))]
    assert got == want


def test_field_errors_capacity_and_empty(torch_dev):
    from paper_2606_15650_amd import api
    rb = _text_batch([b"Host: 1.2.3.4\nMAC: aa\n", b"", b"IP: x"], TYPE_NAMES_17)
    cache = make_cache(TYPE_NAMES_17)
    api.device_errors(0, clear=True)
    cu_h, got = _fields_gpu(rb, cache, CONFIG, span_cap=1)
    assert cu_h.tolist() == [0, 2, 2, 3]
    assert got[0] == [(1, 6, 13)]
    assert api.device_errors(0, clear=True) & api.ERR_SPAN_CAP
    rb2 = _text_batch([b"Host: a", b"IP: b"], TYPE_NAMES_17)
    rb2.cu_bytes = np.array([0, 7, 9], np.int64)  # does not end at n_bytes
    _fields_gpu(rb2, cache, CONFIG)
    assert api.device_errors(0, clear=True) & api.ERR_TEXT
    with pytest.raises(RuntimeError):
        _fields_gpu(rb, cache, {b"Ho:st": 1})
    with pytest.raises(RuntimeError):
        _fields_gpu(rb, cache, {b"Host": 99})
    cu_h, got = _fields_gpu(_text_batch([], TYPE_NAMES_17), cache, CONFIG)
    assert cu_h.tolist() == [0] and got == []
