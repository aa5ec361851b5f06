"""The NER forward pass recorded as one HIP graph (ner_forward_capture): every
replay equals ner_forward on the same buffers bit for bit, with eager work and
synchronisations between replays, and a new batch of the same shape written
into the captured buffers gives that batch's results."""
import numpy as np
import pytest

from synth.configs import TINY, ModelConfig
from tests.gpu_common import make_model, say

pytestmark = pytest.mark.gpu

BASE2 = ModelConfig(n_layers=2, hidden=768, n_heads=12, ffn=3072, vocab=30522, n_labels=17)


def _lengths_batch(lengths, vocab, seed):
    import torch
    rng = np.random.default_rng(seed)
    cu = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    ids = rng.integers(0, vocab, int(cu[-1]), dtype=np.int32)
    return torch.from_numpy(ids).cuda(), torch.from_numpy(cu).cuda()


def _outputs(T, L):
    import torch
    return (torch.empty(T, dtype=torch.uint8, device="cuda"), torch.empty(T, L, dtype=torch.float32, device="cuda"),
            torch.empty(T, dtype=torch.float32, device="cuda"))


def _eager(m, ids, cu, B, T):
    import torch
    from paper_2606_15650_amd import api
    lab, z, mg = _outputs(T, m.cfg.n_labels)
    ws_bytes = m.workspace_size(T, B)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    api.ner_forward(m, ids, cu, B, T, lab, z, mg, ws, ws_bytes)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), z.cpu().numpy(), mg.cpu().numpy()


def _replays_match_eager(m, lengths, seed):
    import torch
    from paper_2606_15650_amd import api
    B, T = len(lengths), int(np.sum(lengths))
    ids, cu = _lengths_batch(lengths, m.cfg.vocab, seed)
    want = _eager(m, ids, cu, B, T)
    lab, z, mg = _outputs(T, m.cfg.n_labels)
    ws_bytes = m.workspace_size(T, B)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    g = api.ner_forward_capture(m, ids, cu, B, T, lab, z, mg, ws, ws_bytes)
    torch.cuda.synchronize()
    other_ids, other_cu = _lengths_batch(lengths[::-1], m.cfg.vocab, seed + 1)
    for rep in range(3):
        lab.fill_(255)
        z.fill_(float("nan"))
        mg.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        got = (lab.cpu().numpy(), z.cpu().numpy(), mg.cpu().numpy())
        for a, b in zip(got, want):
            assert np.array_equal(a, b), f"replay {rep}"
        # eager work of another batch between replays
        _eager(m, other_ids, other_cu, B, T)
    # a new batch of the same shape written into the captured buffers
    perm = np.random.default_rng(seed + 2).permutation(len(lengths))
    new_ids, new_cu = _lengths_batch(np.asarray(lengths)[perm], m.cfg.vocab, seed + 3)
    ids.copy_(new_ids)
    cu.copy_(new_cu)
    g.launch()
    torch.cuda.synchronize()
    want2 = _eager(m, new_ids, new_cu, B, T)
    got = (lab.cpu().numpy(), z.cpu().numpy(), mg.cpu().numpy())
    for a, b in zip(got, want2):
        assert np.array_equal(a, b), "new batch"
    assert not np.array_equal(want[0], want2[0])
    g.close()


def test_tiny_fp32_graph_replays():
    _, m = make_model(TINY, "fp32", 0)
    lengths = np.random.default_rng(0).integers(16, 129, 64)
    say(f"[graph] tiny fp32, {len(lengths)} records, {lengths.sum()} tokens")
    _replays_match_eager(m, lengths, 10)


def test_bf16_base_width_graph_replays():
    """Base widths (two layers): the MFMA GEMM tiles and every attention length
    class, lengths 1..512."""
    _, m = make_model(BASE2, "bf16", 1)
    rng = np.random.default_rng(1)
    lengths = np.clip(np.round(rng.lognormal(5.2, 0.6, 300)), 1, 512).astype(np.int64)
    lengths[:4] = [1, 128, 129, 512]
    say(f"[graph] base-width bf16, {len(lengths)} records, {lengths.sum()} tokens")
    _replays_match_eager(m, lengths, 20)


def test_capture_errors():
    import torch
    from paper_2606_15650_amd import api
    _, m = make_model(TINY, "fp32", 0)
    ids, cu = _lengths_batch([5, 7], TINY.vocab, 0)
    lab, z, mg = _outputs(12, TINY.n_labels)
    ws_bytes = m.workspace_size(12, 2)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.AnonError) as e:
        api.ner_forward_capture(m, ids, cu, 2, 12, lab, z, mg, ws, ws_bytes - 1)
    assert e.value.status == -4  # ECAPACITY
    with pytest.raises(api.AnonError) as e:
        api.ner_forward_capture(m, ids, cu, 0, 0, lab, z, mg, ws, ws_bytes)
    assert e.value.status == -1  # EINVAL
    api.prof_enable("ffn1", True)
    try:
        with pytest.raises(api.AnonError) as e:
            api.ner_forward_capture(m, ids, cu, 2, 12, lab, z, mg, ws, ws_bytes)
        assert e.value.status == -1  # EINVAL
    finally:
        api.prof_enable("ffn1", False)
    # the library stays usable after refused captures
    g = api.ner_forward_capture(m, ids, cu, 2, 12, lab, z, mg, ws, ws_bytes)
    g.launch()
    torch.cuda.synchronize()
    want = _eager(m, ids, cu, 2, 12)
    assert np.array_equal(lab.cpu().numpy(), want[0])
    g.close()


def _bucket_replays_match_eager(m, T_cap, batches, seed):
    """One graph captured for a token bucket of T_cap tokens and T_cap records;
    batches of other sizes are written into its buffers (boundaries padded
    with empty records, the count in device memory) and replayed twice each,
    with eager work of the same batch between the replays.  Every replay
    equals ner_forward on that batch alone, bit for bit, and leaves the rows
    past the batch untouched."""
    import torch
    from paper_2606_15650_amd import api
    L = m.cfg.n_labels
    ids = torch.zeros(T_cap, dtype=torch.int32, device="cuda")
    cu = torch.zeros(T_cap + 1, dtype=torch.int32, device="cuda")
    n_tok = torch.zeros(1, dtype=torch.int32, device="cuda")
    lab, z, mg = _outputs(T_cap, L)
    ws_bytes = m.workspace_size(T_cap, T_cap)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    g = api.ner_forward_capture_bucket(m, ids, cu, n_tok, T_cap, T_cap, lab, z, mg, ws, ws_bytes)
    torch.cuda.synchronize()
    for i, lengths in enumerate(batches):
        B, T = len(lengths), int(np.sum(lengths))
        assert B <= T_cap and T <= T_cap
        say(f"[graph] bucket {T_cap}: batch {i}, {B} records, {T} tokens")
        b_ids, b_cu = _lengths_batch(lengths, m.cfg.vocab, seed + i)
        for rep in range(2):
            want = _eager(m, b_ids, b_cu, B, T)
            lab.fill_(255)
            z.fill_(float("nan"))
            mg.fill_(float("nan"))
            ids[:T].copy_(b_ids)
            cu[:B + 1].copy_(b_cu)
            cu[B + 1:].fill_(T)
            n_tok.fill_(T)
            g.launch()
            torch.cuda.synchronize()
            got = (lab[:T].cpu().numpy(), z[:T].cpu().numpy(), mg[:T].cpu().numpy())
            for a, b in zip(got, want):
                assert np.array_equal(a, b), f"batch {i} replay {rep}"
            assert (lab[T:].cpu().numpy() == 255).all(), "rows past the batch were written"
    assert api.device_errors(0, clear=True) == 0
    # a count past the bucket raises the sequence-length bit; nothing faults
    # (records of 64 tokens that fill the bucket: only the count is wrong)
    cu.copy_(torch.clamp(torch.arange(T_cap + 1, dtype=torch.int32, device="cuda") * 64, max=T_cap))
    n_tok.fill_(T_cap + 5)
    g.launch()
    torch.cuda.synchronize()
    assert api.device_errors(0, clear=True) & api.ERR_SEQLENS
    g.close()


def test_tiny_fp32_bucket_graph_replays():
    _, m = make_model(TINY, "fp32", 0)
    rng = np.random.default_rng(3)
    batches = [[1], [3, 17, 1], rng.integers(16, 129, 40), np.full(32, 128)]
    _bucket_replays_match_eager(m, 4096, batches, 30)


def test_bf16_base_width_bucket_graph_replays():
    """Base widths (two layers), a 16384-token bucket: batches from one token
    to the full bucket, lengths at the attention tile edges."""
    _, m = make_model(BASE2, "bf16", 1)
    rng = np.random.default_rng(4)
    ragged = np.clip(np.round(rng.lognormal(5.2, 0.6, 40)), 1, 512).astype(np.int64)
    ragged[:4] = [1, 128, 129, 512]
    batches = [[1], ragged, [512] * 32, [7, 300, 64]]
    _bucket_replays_match_eager(m, 16384, batches, 40)


def test_bucket_capture_errors():
    import torch
    from paper_2606_15650_amd import api
    _, m = make_model(TINY, "fp32", 0)
    ids = torch.zeros(64, dtype=torch.int32, device="cuda")
    cu = torch.zeros(65, dtype=torch.int32, device="cuda")
    n_tok = torch.zeros(1, dtype=torch.int32, device="cuda")
    lab, z, mg = _outputs(64, TINY.n_labels)
    ws_bytes = m.workspace_size(64, 64)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.AnonError) as e:
        api.ner_forward_capture_bucket(m, ids, cu, None, 64, 64, lab, z, mg, ws, ws_bytes)
    assert e.value.status == -1  # EINVAL: no count
    with pytest.raises(api.AnonError) as e:
        api.ner_forward_capture_bucket(m, ids, cu, n_tok, 0, 64, lab, z, mg, ws, ws_bytes)
    assert e.value.status == -1  # EINVAL: empty bucket
    with pytest.raises(api.AnonError) as e:
        api.ner_forward_capture_bucket(m, ids, cu, n_tok, 64, 64, lab, z, mg, ws, ws_bytes - 1)
    assert e.value.status == -4  # ECAPACITY
