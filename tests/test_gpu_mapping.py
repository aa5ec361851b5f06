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
