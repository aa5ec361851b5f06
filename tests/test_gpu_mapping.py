"""GPU parity of per-type preservation and of the mapping export against the oracle."""
import numpy as np
import pytest

import synth
from oracle import pseudonym as ops
from tests.gpu_common import make_cache, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _pseudo(rb, spans, cache):
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list
    db = DeviceBatch(rb)
    n = len(spans)
    raw = np.zeros((max(n, 1), 3), np.int64)
    if n:
        raw[:n, 0] = (spans[:, 0] & 0xFFFFFFFF) | (spans[:, 1] << 32)
        raw[:n, 1] = spans[:, 2]
        raw[:n, 2] = spans[:, 3]
    counts = np.bincount(spans[:, 0], minlength=rb.n_records) if n else np.zeros(rb.n_records, np.int64)
    cu = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)).cuda()
    pl = Pipeline.__new__(Pipeline)
    pl.cache, pl.device, pl._ws = cache, torch.device("cuda:0"), {}
    out, cu_out = pl.pseudonymize(db, torch.from_numpy(raw).cuda(), cu, max(n, 1))
    torch.cuda.synchronize()
    return outputs_to_list(out, cu_out)


def test_preserved_types_are_left_in_place(torch_dev):
    rb = synth.generate_records(200, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 51)
    cache = make_cache(rb.type_names)
    key = synth.make_key(0)
    keep = ["IP_ADDRESS", "HASH"]
    idx = [rb.type_names.index(t) + 1 for t in keep]
    cache.set_preserve(keep)
    say(f"[preserve] {keep}")
    got = _pseudo(rb, rb.gold_spans, cache)
    sp = rb.gold_spans[~np.isin(rb.gold_spans[:, 1], idx)]
    want = ops.pseudonymize_batch(rb.text, rb.cu_bytes, sp, rb.n_records, rb.type_names, key, cache.slug)
    assert got == want
    cache.set_preserve([])
    want_all = ops.pseudonymize_batch(rb.text, rb.cu_bytes, rb.gold_spans, rb.n_records, rb.type_names, key,
                                      cache.slug)
    assert _pseudo(rb, rb.gold_spans, cache) == want_all
    with pytest.raises(RuntimeError):
        cache.set_preserve([99])


def test_mapping_export_after_three_calls(torch_dev):
    """Batch A, batch B, batch A again (entities repeat across and within
    calls; some exceed the 96-byte table entry)."""
    names = synth.TYPE_NAMES_17
    A = synth.generate_records(150, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 61)
    B = synth.generate_records(150, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 62)
    key = synth.make_key(0)
    cache = make_cache(names, slug=12, capacity=1 << 17)  # two export chunks
    cache.set_preserve(["PORT"])
    port = names.index("PORT") + 1
    # long spans: whole lines of some records (beyond the table's 96 bytes)
    def with_long(rb):
        extra = []
        for r in range(0, rb.n_records, 25):
            n = int(rb.cu_bytes[r + 1] - rb.cu_bytes[r])
            if n > 120 and not (rb.gold_spans[:, 0] == r).any():
                extra.append([r, 2, 0, 110])
        sp = np.concatenate([rb.gold_spans, np.array(extra, np.int64).reshape(-1, 4)])
        return sp[np.lexsort((sp[:, 2], sp[:, 0]))]
    calls = [(A, with_long(A)), (B, with_long(B)), (A, with_long(A))]
    for rb, sp in calls:
        got = _pseudo(rb, sp, cache)
        keep = sp[sp[:, 1] != port]
        assert got == ops.pseudonymize_batch(rb.text, rb.cu_bytes, keep, rb.n_records, names, key, 12)
    rows = cache.export()
    want = ops.mapping_rows([(rb.text, rb.cu_bytes, sp) for rb, sp in calls], names, key, 12, preserve=(port,))
    say(f"[mapping] {len(rows)} rows")
    assert len(want) > 200
    assert rows == want
    # a clear empties the table and restarts the call count
    cache.clear()
    assert cache.export() == []
    _pseudo(B, calls[1][1], cache)
    rows = cache.export()
    assert rows and all(r["first_seen"] == 1 and r["last_seen"] == 1 for r in rows)


def test_many_duplicate_inserts_of_one_entity_in_one_call(torch_dev):
    """20,000 spans of one entity (plus a few others) in one call: every probe
    of the first call races to insert the same key.  The output equals the
    oracle's, the counters add up, the table ends with one row for the
    entity after the export merges racing inserts, and a second call is
    served from the table."""
    from synth.records import RecordBatch
    hot = b"10.20.30.40"
    others = [b"db01.corp", b"CVE-2021-44228", b"alice@example.org"]
    texts, spans = [], []
    for r in range(2000):
        parts, sp = [], []
        pos = 0
        for k in range(10):
            ent = hot if (k + r) % 11 else others[(k + r) % 3]
            pre = b"host " if k else b""
            parts += [pre, ent, b" "]
            pos += len(pre)
            sp.append((r, 1 if ent == hot else 2, pos, pos + len(ent)))
            pos += len(ent) + 1
        texts.append(b"".join(parts))
        spans += sp
    text = b"".join(texts)
    cu_bytes = np.concatenate([[0], np.cumsum([len(t) for t in texts])]).astype(np.int64)
    # one token per record (the pseudonymizer reads text and spans only)
    rb = RecordBatch(text, cu_bytes, np.zeros(2000, np.int32), np.zeros((2000, 2), np.int32),
                     np.arange(2001, dtype=np.int32), np.zeros(2000, np.uint8), np.zeros((0, 4), np.int64),
                     ["IP_ADDRESS", "HOSTNAME", "CVE_ID", "EMAIL_ADDRESS"])
    spans = np.array(spans, np.int64)
    n_hot = int((spans[:, 1] == 1).sum())
    say(f"[pcache] {len(spans)} spans, {n_hot} of them the same entity, one call")
    cache = make_cache(rb.type_names, capacity=1 << 12)
    got = _pseudo(rb, spans, cache)
    want = ops.pseudonymize_batch(rb.text, rb.cu_bytes, spans, rb.n_records, rb.type_names, synth.make_key(0), 10)
    assert got == want
    st = cache.stats()
    say(f"  first call: {st}")
    assert st["lookups"] == len(spans)
    assert 4 <= st["entries"] <= st["lookups"] - st["hits"]
    rows = cache.export()
    hot_rows = [r for r in rows if r["original"] == hot]
    assert len(hot_rows) == 1 and hot_rows[0]["entity_type"] == "IP_ADDRESS"
    assert sorted(r["original"] for r in rows) == sorted([hot] + others)
    got2 = _pseudo(rb, spans, cache)
    assert got2 == want
    st2 = cache.stats()
    assert st2["hits"] - st["hits"] == len(spans)
    cache.close()


def test_concurrent_calls_on_two_streams_share_one_table(torch_dev):
    """Two calls enqueued back to back on two streams with one table (as the
    server's slots run them; whether their kernels overlap is up to the
    device, and the first pair's hit count shows it): the same batch on both,
    then another batch beside a repeat of the first (misses beside hits).
    Every output equals the oracle's, the counters add up, and the export
    holds each distinct cached entity once."""
    import torch
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list
    rb_a = synth.generate_records(400, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 61)
    rb_c = synth.generate_records(300, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 62)
    cache = make_cache(rb_a.type_names)
    key = synth.make_key(0)

    def prep(rb):
        sp = rb.gold_spans
        raw = np.zeros((max(len(sp), 1), 3), np.int64)
        raw[:len(sp), 0] = (sp[:, 0] & 0xFFFFFFFF) | (sp[:, 1] << 32)
        raw[:len(sp), 1:] = sp[:, 2:4]
        counts = np.bincount(sp[:, 0], minlength=rb.n_records)
        cu = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        return DeviceBatch(rb), torch.from_numpy(raw).cuda(), torch.from_numpy(cu).cuda(), max(len(sp), 1)

    def pipe():
        pl = Pipeline.__new__(Pipeline)
        pl.cache, pl.device, pl._ws = cache, torch.device("cuda:0"), {}
        return pl

    a, c = prep(rb_a), prep(rb_c)
    # only entities of at most 96 bytes are looked up (longer ones are hashed every time)
    n_a = int(((rb_a.gold_spans[:, 3] - rb_a.gold_spans[:, 2]) <= 96).sum())
    n_c = int(((rb_c.gold_spans[:, 3] - rb_c.gold_spans[:, 2]) <= 96).sum())
    want_a = ops.pseudonymize_batch(rb_a.text, rb_a.cu_bytes, rb_a.gold_spans, rb_a.n_records, rb_a.type_names,
                                    key, cache.slug)
    want_c = ops.pseudonymize_batch(rb_c.text, rb_c.cu_bytes, rb_c.gold_spans, rb_c.n_records, rb_c.type_names,
                                    key, cache.slug)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    p1, p2 = pipe(), pipe()
    torch.cuda.synchronize()
    say(f"[pcache] two streams: {len(rb_a.gold_spans)} spans on each, one table")
    o1 = p1.pseudonymize(a[0], a[1], a[2], a[3], stream=s1)
    o2 = p2.pseudonymize(a[0], a[1], a[2], a[3], stream=s2)
    torch.cuda.synchronize()
    assert outputs_to_list(*o1) == want_a
    assert outputs_to_list(*o2) == want_a
    st = cache.stats()
    say(f"  first pair: {st}")
    assert st["lookups"] == 2 * n_a
    assert st["entries"] <= st["lookups"] - st["hits"]
    # a new batch beside a repeat of the first
    p1, p2 = pipe(), pipe()
    o1 = p1.pseudonymize(c[0], c[1], c[2], c[3], stream=s1)
    o2 = p2.pseudonymize(a[0], a[1], a[2], a[3], stream=s2)
    torch.cuda.synchronize()
    assert outputs_to_list(*o1) == want_c
    assert outputs_to_list(*o2) == want_a
    st2 = cache.stats()
    say(f"  second pair: {st2}")
    assert st2["lookups"] == st["lookups"] + n_a + n_c
    assert st2["hits"] - st["hits"] >= n_a  # the repeat meets only cached entities
    # the export: each distinct entity of at most 96 bytes once
    ents = set()
    for rb in (rb_a, rb_c):
        for r, _, b, e in rb.gold_spans:
            if e - b <= 96:
                ents.add(bytes(rb.text[rb.cu_bytes[r] + b:rb.cu_bytes[r] + e]))
    rows = cache.export()
    originals = [r["original"] for r in rows]
    assert len(originals) == len(set(originals))
    assert set(originals) == ents
