"""decode_spans_noalloc (no workspace, no allocation) against decode_spans.

Two calls in a row on the same GPU, the second on a smaller batch, each
compared bit for bit with decode_spans on the same labels; a batch above the
scratch array's token limit is refused before any launch."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import spans as ospans
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _both(rb, labels, n_types, span_cap):
    import torch
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, spans_to_numpy
    db = DeviceBatch(rb)
    lab = torch.from_numpy(np.ascontiguousarray(labels, np.uint8)).cuda()
    out = []
    for noalloc in (False, True):
        spans = torch.full((max(span_cap, 1), 3), -7, dtype=torch.int64, device="cuda")
        cu_spans = torch.full((rb.n_records + 1,), -7, dtype=torch.int32, device="cuda")
        if noalloc:
            api.decode_spans_noalloc(lab, db.tok_off, db.cu, rb.n_records, rb.n_tokens, n_types, spans, span_cap,
                                     cu_spans)
        else:
            ws = torch.empty(api.decode_workspace_size(rb.n_tokens, rb.n_records), dtype=torch.uint8, device="cuda")
            api.decode_spans(lab, db.tok_off, db.cu, rb.n_records, rb.n_tokens, n_types, spans, span_cap, cu_spans,
                             ws, ws.numel())
        torch.cuda.synchronize()
        cs = cu_spans.cpu().numpy()
        out.append((spans_to_numpy(spans, min(int(cs[-1]), span_cap)), cs))
    return out


def test_noalloc_decode_equals_decode_spans_on_two_calls(torch_dev):
    rng = np.random.default_rng(31)
    big = synth.generate_records(600, ("lognormal", 5.2, 0.6, 16, 512), 8, 30522, 41)
    small = synth.generate_records(37, ("uniform", 1, 90), 8, 30522, 42)
    for name, rb in (("first call", big), ("second call, smaller", small)):
        lab = rng.integers(0, 17, rb.n_tokens).astype(np.uint8)
        (sp_ref, cu_ref), (sp_na, cu_na) = _both(rb, lab, 8, rb.n_tokens)
        say(f"[noalloc] {name}: T={rb.n_tokens} B={rb.n_records} spans={int(cu_ref[-1])}")
        np.testing.assert_array_equal(cu_na, cu_ref)
        np.testing.assert_array_equal(sp_na, sp_ref)
        np.testing.assert_array_equal(sp_na, ospans.bio_decode(lab, rb.tok_off, rb.cu_seqlens, 8))


def test_noalloc_capacity_report_and_limit(torch_dev):
    import torch
    from paper_2606_15650_amd import api
    rb = synth.generate_records(20, ("uniform", 16, 64), 4, 8192, 2)
    lab = np.ones(rb.n_tokens, np.uint8)  # every token opens a span
    (sp_ref, cu_ref), (sp_na, cu_na) = _both(rb, lab, 4, 10)
    assert cu_na[-1] == rb.n_tokens and len(sp_na) == 10
    np.testing.assert_array_equal(sp_na, sp_ref)
    # above the scratch limit: refused on the host, nothing launched
    T = api.NOALLOC_MAX_TOKENS + 1
    d = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="exceeds"):
        api.decode_spans_noalloc(d, d, d, 1, T, 4, d, 0, d)
