"""Serving loop (anon_submit / anon_poll) on the GPU: continuous batching must
not change any request's result, and bad requests fail cleanly."""
import time

import numpy as np
import pytest

import synth
from oracle import pipeline as opipe
from synth.configs import TINY
from tests.gpu_common import make_cache, make_model, say

pytestmark = pytest.mark.gpu


def _requests(rb, sizes):
    out, r0 = [], 0
    for n in sizes:
        out.append(rb.subset(range(r0, r0 + n)))
        r0 += n
    return out


def _submit(sv, req):
    return sv.submit(req.ids, req.cu_seqlens, req.tok_off, req.text, req.cu_bytes)


def _wait(sv, ticket, timeout=60.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        r = sv.poll(ticket)
        if r is not None:
            return r
        time.sleep(0.001)
    raise TimeoutError(ticket)


@pytest.fixture(scope="module")
def server():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_15650_amd import api
    W, m = make_model(TINY, "bf16", 0)
    cache = make_cache(synth.TYPE_NAMES_9)
    sv = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=4096, n_streams=3, max_queue=256)
    yield W, m, cache, sv
    sv.stop()


def test_results_alone_equal_results_in_the_mix(server):
    W, m, cache, sv = server
    rb = synth.generate_records(90, ("uniform", 16, 128), 4, TINY.vocab, 41)
    sizes = [1, 7, 3, 12, 20, 5, 9, 2, 15, 16]
    reqs = _requests(rb, sizes)
    say(f"[server] {len(reqs)} requests one at a time")
    alone = []
    for q in reqs:
        t = _submit(sv, q)
        r = _wait(sv, t)
        assert r["status"] == 0
        alone.append(r)
        sv.release(t)
    say("[server] the same requests submitted together")
    tickets = [_submit(sv, q) for q in reqs]
    mixed = [_wait(sv, t) for t in tickets]
    for t in tickets:
        sv.release(t)
    for a, b, q in zip(alone, mixed, reqs):
        assert b["status"] == 0
        np.testing.assert_array_equal(a["labels"], b["labels"])
        np.testing.assert_array_equal(a["spans"], b["spans"])
        assert a["out"] == b["out"]
        np.testing.assert_array_equal(a["cu_out"], b["cu_out"])
        assert b["n_records"] == q.n_records


def test_server_output_equals_oracle_tail_on_gpu_labels(server):
    W, m, cache, sv = server
    rb = synth.generate_records(10, ("uniform", 16, 128), 4, TINY.vocab, 42)
    say("[server] one request vs the oracle's spans and substitution on the same labels")
    t = _submit(sv, rb)
    r = _wait(sv, t)
    sv.release(t)
    res = opipe.run(W, TINY, rb, synth.make_key(0), 10, labels_override=r["labels"])
    np.testing.assert_array_equal(r["spans"], res.spans)
    cu = r["cu_out"]
    outs = [r["out"][cu[i]:cu[i + 1]] for i in range(rb.n_records)]
    assert outs == res.outputs


def test_bad_requests_are_rejected(server):
    from paper_2606_15650_amd import api
    W, m, cache, sv = server
    rb = synth.generate_records(2, ("uniform", 16, 32), 4, TINY.vocab, 43)
    say("[server] malformed requests")
    bad_ids = rb.ids.copy()
    bad_ids[0] = TINY.vocab + 5
    with pytest.raises(api.AnonError):
        sv.submit(bad_ids, rb.cu_seqlens, rb.tok_off, rb.text, rb.cu_bytes)
    bad_cu = rb.cu_seqlens.copy()
    bad_cu[1] = bad_cu[0]  # empty record
    with pytest.raises(api.AnonError):
        sv.submit(rb.ids, bad_cu, rb.tok_off, rb.text, rb.cu_bytes)
    big = synth.generate_records(40, np.full(40, 128), 4, TINY.vocab, 44)  # 5120 tokens > micro-batch
    with pytest.raises(api.AnonError):
        _submit(sv, big)
    with pytest.raises(api.AnonError):
        sv.poll(987654321)
    # token byte ranges that overlap, or run past their record, are refused
    # before anything reaches the GPU (a bad range would make an entity span
    # leave its record or overlap another, and its bytes would stay in clear)
    bad_off = rb.tok_off.copy()
    bad_off[3, 0] = bad_off[2, 0]
    with pytest.raises(api.AnonError):
        sv.submit(rb.ids, rb.cu_seqlens, bad_off, rb.text, rb.cu_bytes)
    bad_off = rb.tok_off.copy()
    bad_off[int(rb.cu_seqlens[1]) - 1, 1] = int(rb.cu_bytes[1] - rb.cu_bytes[0]) + 1
    with pytest.raises(api.AnonError):
        sv.submit(rb.ids, rb.cu_seqlens, bad_off, rb.text, rb.cu_bytes)
    bad_off = rb.tok_off.copy()
    bad_off[0] = (5, 2)
    with pytest.raises(api.AnonError):
        sv.submit(rb.ids, rb.cu_seqlens, bad_off, rb.text, rb.cu_bytes)
    # the server still serves after the refusals
    r = _wait(sv, _submit(sv, rb))
    assert r["status"] == 0


def test_admission_by_activation_budget():
    """With a budget that holds one full micro-batch (and not two), micro-batches
    never run concurrently although three slots are free, the arena in use
    never exceeds the budget, and every result equals the one a roomy server
    gives."""
    from paper_2606_15650_amd import api
    W, m = make_model(TINY, "bf16", 0)
    cache = make_cache(synth.TYPE_NAMES_9)
    # requests of 960 tokens: one per 1024-token micro-batch, each taking
    # most of a full micro-batch's footprint, so two never fit 1.5 of them
    rb = synth.generate_records(96, np.full(96, 120), 4, TINY.vocab, 46)
    reqs = _requests(rb, [8] * 12)
    roomy = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=1024, n_streams=3, max_queue=256)
    full = roomy.stats()["arena_bytes"] // 3  # one full micro-batch
    ref = [_wait(roomy, _submit(roomy, q)) for q in reqs]
    st_roomy = roomy.stats()
    roomy.stop()
    tight = api.Server(m, cache, hbm_budget_bytes=full + full // 2, max_batch_tokens=1024, n_streams=3,
                       max_queue=256)
    tickets = [_submit(tight, q) for q in reqs]
    got = [_wait(tight, t) for t in tickets]
    st = tight.stats()
    tight.stop()
    say(f"[server] roomy {st_roomy}; tight {st}")
    assert st["arena_bytes"] <= full + full // 2
    assert st["peak_arena_bytes"] <= st["arena_bytes"]
    assert st["max_concurrent"] == 1
    for a, b in zip(ref, got):
        assert b["status"] == 0
        np.testing.assert_array_equal(a["labels"], b["labels"])
        assert a["out"] == b["out"]
    m.close()
    cache.close()


def test_stop_with_work_in_flight_finishes_cleanly():
    import torch
    from paper_2606_15650_amd import api
    W, m = make_model(TINY, "fp32", 1)
    cache = make_cache(synth.TYPE_NAMES_9)
    sv = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=2048, n_streams=2, max_queue=64)
    rb = synth.generate_records(60, ("uniform", 16, 64), 4, TINY.vocab, 45)
    reqs = _requests(rb, [6] * 10)
    say("[server] stop while requests are queued/in flight")
    tickets = [_submit(sv, q) for q in reqs]
    r0 = _wait(sv, tickets[0])
    assert r0["status"] == 0
    sv.stop()
    torch.cuda.synchronize()


def test_budget_too_small_fails_at_start():
    from paper_2606_15650_amd import api
    W, m = make_model(TINY, "fp32", 1)
    cache = make_cache(synth.TYPE_NAMES_9)
    say("[server] start with a budget below one slot")
    with pytest.raises(api.AnonError):
        api.Server(m, cache, hbm_budget_bytes=1 << 20, max_batch_tokens=4096, n_streams=2)


def test_graph_bucket_server_equals_eager_server_alone_and_mixed():
    """Graph buckets on, base-width model (two layers, 17 labels): every forward
    runs as a graph replay; each request's labels, spans and bytes are the same
    alone, in the mix and from the eager server."""
    from paper_2606_15650_amd import api
    from synth.configs import ModelConfig
    base2 = ModelConfig(n_layers=2, hidden=768, n_heads=12, ffn=3072, vocab=30522, n_labels=17)
    W, m = make_model(base2, "bf16", 2)
    cache = make_cache(synth.TYPE_NAMES_17[:8])
    rb = synth.generate_records(90, ("uniform", 16, 512), 8, base2.vocab, 47)
    reqs = _requests(rb, [1, 7, 3, 12, 20, 5, 9, 2, 15, 16])
    eager = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=16384, n_streams=3, max_queue=256)
    say("[server] eager server, requests together")
    ref = [_wait(eager, t) for t in [_submit(eager, q) for q in reqs]]
    eager.stop()
    sv = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=16384, n_streams=3, max_queue=256,
                    graph_buckets=6)
    say("[server] graph buckets, requests one at a time")
    alone = []
    for q in reqs:
        t = _submit(sv, q)
        alone.append(_wait(sv, t))
        sv.release(t)
    say("[server] graph buckets, requests together")
    tickets = [_submit(sv, q) for q in reqs]
    mixed = [_wait(sv, t) for t in tickets]
    st = sv.stats()
    sv.stop()
    say(f"[server] graph-bucket server stats {st}")
    assert st["graph_launches"] == st["micro_batches"] > len(reqs)
    for a, b, c, q in zip(alone, mixed, ref, reqs):
        for r in (a, b, c):
            assert r["status"] == 0
        for r in (a, b):
            np.testing.assert_array_equal(r["labels"], c["labels"])
            np.testing.assert_array_equal(r["spans"], c["spans"])
            assert r["out"] == c["out"]
            np.testing.assert_array_equal(r["cu_out"], c["cu_out"])
    m.close()
    cache.close()


def test_graph_bucket_server_start_errors():
    from paper_2606_15650_amd import api
    W, m = make_model(TINY, "bf16", 0)
    cache = make_cache(synth.TYPE_NAMES_9)
    with pytest.raises(api.AnonError):
        api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=4096, n_streams=2, graph_buckets=17)
    # the fixed slot buffers count against the budget: one that holds the
    # eager server's arena does not hold them as well
    eager = api.Server(m, cache, hbm_budget_bytes=8 << 30, max_batch_tokens=4096, n_streams=2, max_queue=8)
    need = eager.stats()["arena_bytes"]
    eager.stop()
    with pytest.raises(api.AnonError):
        api.Server(m, cache, hbm_budget_bytes=need // 2 + (need // 2) // 4, max_batch_tokens=4096, n_streams=2,
                   graph_buckets=4)
    m.close()
    cache.close()
