"""Throughput of the NER + pseudonymize path on one MI355X.

A step is one pass of the whole path over one resident batch: ner_forward
(embedding, 12 post-LN encoder layers, classifier), decode_spans and
pseudonymize, all on one stream.  Inputs (token ids, offsets, text) are in HBM
before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload base_bf16]

Prints one JSON line.  Besides the headline tokens/s it reports the plain FP32
path on the same batch (the speedup baseline), per-step p50/p99 latency, the
dominant kernel against the MFMA roofline (timed with HIP events on its launch
stream during the timed steps), the serving loop's p50/p99 request latency at
100 req/s (6 s of Poisson arrivals), and the FP64 oracle's throughput on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense): FLOP/s per operand type, HBM bytes/s
PEAK_FLOPS = {"bf16": 2.5e15, "fp8": 5.0e15, "fp32": 157.3e12}
PEAK_HBM = 8.0e12


# kernel class -> source file whose kernels it launches
KERNEL_SOURCE = {"qkv": "k_gemm.hip", "oproj": "k_gemm.hip", "ffn1": "k_gemm.hip", "ffn2": "k_gemm.hip",
                 "attn": "k_attn.hip"}


def counter_traffic(workload: str, kernel: str, tile: str | None):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE runs, each scaled by the reading of a
    1 GiB copy), or None when there is none, it was taken on another tile, or
    the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_{kernel}_counters.json")
    src = KERNEL_SOURCE.get(kernel)
    if not src or not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        c = json.load(f)
    with open(os.path.join(ROOT, "paper_2606_15650_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if c.get("source_sha256") != sha:
        return None, f"{src} changed since the counters were taken"
    # one entry per tile and tile order the counters were taken on
    entries = c.get("entries", [c])
    for e in entries:
        if tile is None or e.get("tile") == tile:
            return float(e["bytes_per_launch"]), f"{os.path.relpath(path, ROOT)} ({e.get('tile')})"
    return None, f"counters taken on tiles {[e.get('tile') for e in entries]}, this run chose {tile}"


def attention_flops(cu: np.ndarray, cfg) -> float:
    """Algorithmic attention FLOPs of one layer: QK^T and PV over each record."""
    L = np.diff(cu).astype(np.float64)
    return float((4.0 * L * L * cfg.hidden).sum())


def gemm_flops_per_token(cfg) -> dict:
    h, f = cfg.hidden, cfg.ffn
    return {"qkv": 2 * h * 3 * h, "oproj": 2 * h * h, "ffn1": 2 * h * f, "ffn2": 2 * f * h}


def path_flops(cfg, cu: np.ndarray) -> float:
    T = float(cu[-1])
    g = sum(gemm_flops_per_token(cfg).values())
    return cfg.n_layers * (g * T + attention_flops(cu, cfg)) + 2.0 * cfg.hidden * cfg.n_labels * T


def modern_flops(cfg, cu: np.ndarray) -> dict:
    """Algorithmic FLOPs of one pass of the ModernBERT-style encoder, per
    kernel class: the GEMMs per token, attention from the pairs each query
    sees (all keys of its record on global layers, those at most
    local_window/2 away on local ones), the head and classifier."""
    h, I = cfg.hidden, cfg.intermediate
    T = float(cu[-1])
    L = np.diff(cu).astype(np.int64)
    w = cfg.local_window // 2
    full = float((L.astype(np.float64) ** 2).sum())
    # pairs |i - j| <= w in a record of n tokens
    n = L.astype(np.float64)
    ww = np.minimum(w, n - 1)
    band = float((n * (2 * ww + 1) - ww * (ww + 1)).sum())
    n_glob = sum(1 for l in range(cfg.n_layers) if l % cfg.global_every == 0)
    att = 4.0 * h * (n_glob * full + (cfg.n_layers - n_glob) * band)
    gl = cfg.n_layers
    return {"qkv": gl * 2.0 * h * 3 * h * T, "oproj": gl * 2.0 * h * h * T, "ffn1": gl * 2.0 * h * 2 * I * T,
            "ffn2": gl * 2.0 * I * h * T, "attn": att, "cls": 2.0 * h * h * T + 2.0 * h * cfg.n_labels * T}


def modern_bench(steps: int, warmup: int, keep: bool, log=None) -> dict:
    """The ModernBERT-style encoder (22 layers, h768, GeGLU 1152, local and
    global attention) on the base workload's records: the whole path (NER,
    spans, pseudonyms) timed like the headline, its kernels, the dominant
    kernel against the BF16 MFMA peak."""
    import torch

    import synth
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline

    wl = synth.workload("modern_bf16")
    cfg = wl.model
    rb = synth.generate_records(wl.n_records, wl.lengths, cfg.n_types, cfg.vocab, wl.seed)
    W = synth.make_weights(cfg, wl.weight_seed, wl.o_target)
    key = synth.make_key(0)
    model = api.ModernModel(cfg, synth.weights_blob(cfg, W), "bf16")
    cache = api.PseudonymCache(key, 10, rb.type_names, 1 << 20)
    pl = Pipeline(model, cache)
    db = DeviceBatch(rb)
    T = rb.n_tokens
    for _ in range(warmup):
        cache.clear()
        pl.step(db)
    torch.cuda.synchronize()
    classes = ["qkv", "attn", "oproj", "ffn1", "ffn2", "ln", "embed", "cls"]
    for k in classes:
        api.prof_enable(k, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        cache.clear()  # a cold pseudonym table every step, as on the base path
        pl.step(db)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = {k: api.prof_read(k) for k in classes}
    for k in classes:
        api.prof_enable(k, False)
    fl = modern_flops(cfg, rb.cu_seqlens.astype(np.int64))
    breakdown = {}
    for k, v in kern.items():
        if v["launches"]:
            f = fl.get(k)
            per_launch = f / (v["launches"] / steps) if f else None
            breakdown[k] = {"launches": v["launches"], "ms_per_step": v["ms"] / steps,
                            "tflops": (per_launch * v["launches"] / (v["ms"] * 1e-3) / 1e12) if f else None}
    dom = max((k for k in breakdown if fl.get(k)), key=lambda k: kern[k]["ms"])
    d = kern[dom]
    avg_ms = d["ms"] / d["launches"]
    per_launch = fl[dom] / (d["launches"] / steps)
    total = sum(fl.values())
    out = {"workload": wl.name, "value": T * steps / wall, "unit": "tokens/s", "ms_per_step": wall / steps * 1e3,
           "steps": steps, "dtype": "bf16",
           "config": {"records": rb.n_records, "tokens": T, "layers": cfg.n_layers, "hidden": cfg.hidden,
                      "heads": cfg.n_heads, "intermediate": cfg.intermediate, "vocab": cfg.vocab,
                      "local_window": cfg.local_window, "global_every": cfg.global_every,
                      "lengths": list(wl.lengths)},
           "roofline": {"bound": "mfma", "kernel": dom, "achieved": per_launch / (avg_ms * 1e-3) / 1e12,
                        "peak": PEAK_FLOPS["bf16"] / 1e12, "unit": "TFLOP/s",
                        "frac": per_launch / (avg_ms * 1e-3) / PEAK_FLOPS["bf16"], "avg_launch_ms": avg_ms,
                        "flops_per_launch": per_launch},
           "path_tflops": total / (wall / steps) / 1e12, "path_mfma_frac": total / (wall / steps) / PEAK_FLOPS["bf16"],
           "kernels": breakdown, "pcache": cache.stats()}
    ctx = None
    if keep:
        _, z, _ = pl.ner(db, logits=True)
        torch.cuda.synchronize()
        ctx = {"wl": wl, "rb": rb, "W": W, "z": z[:T].cpu().numpy()}
    model.close()
    cache.close()
    return out, ctx


def modern_parity(ctx: dict, budget_s: float) -> dict:
    """Logit error and label agreement of the ModernBERT-style path on its
    first records against the pure FP64 oracle and the rounding oracle (part
    of the CPU baseline leg)."""
    from oracle import encoder, modernbert as mb
    wl, rb, W, zg_all = ctx["wl"], ctx["rb"], ctx["W"], ctx["z"]
    cfg = wl.model
    zs, zqs, nrec = [], [], 0
    t0 = time.perf_counter()
    while nrec < rb.n_records and time.perf_counter() - t0 < budget_s:
        sub = rb.subset([nrec])
        zs.append(mb.forward(W, cfg, sub.ids, sub.cu_seqlens)[0])
        zqs.append(mb.forward(W, cfg, sub.ids, sub.cu_seqlens, encoder.Precision("bf16"))[0])
        nrec += 1
    n = int(rb.cu_seqlens[nrec])
    zg = zg_all[:n].astype(np.float64)
    lg = encoder.argmax_margin(zg)[0]
    out = {"records": nrec, "tokens": n}
    for name, zr in (("vs_pure_fp64_oracle", np.concatenate(zs)), ("vs_rounding_oracle", np.concatenate(zqs))):
        lr, mr = encoder.argmax_margin(zr)
        d = np.abs(zg - zr)
        conf = mr > 1e-2
        out[name] = {"max_abs_logit_err": float(d.max()), "rms_logit_err": float(np.sqrt((d ** 2).mean())),
                     "label_agreement_all": float((lg == lr).mean()),
                     "label_agreement_confident": float((lg[conf] == lr[conf]).mean()) if conf.any() else 1.0,
                     "confident_label_mismatches": int((conf & (lg != lr)).sum()),
                     "tokens_margin_le_1e-2": int((~conf).sum())}
    return out


def cpu_baseline(wl, rb, W, key, budget_s: float = 12.0):
    """The FP64 oracle on the first records of the workload, until ~budget_s of
    CPU work.  Returns the baseline entry and the oracle's logits, labels and
    outputs of the records it ran (the parity leg compares the GPU with them)."""
    from oracle import pipeline as opipe
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    tok = 0
    nrec = 0
    zs, outs = [], []
    t0 = time.perf_counter()
    step = 2
    while nrec < rb.n_records and time.perf_counter() - t0 < budget_s:
        sub = rb.subset(range(nrec, min(nrec + step, rb.n_records)))
        res = opipe.run(W, wl.model, sub, key, 10)
        zs.append(res.logits)
        outs.extend(res.outputs)
        tok += sub.n_tokens
        nrec += sub.n_records
    dt = time.perf_counter() - t0
    entry = {"value": tok / dt, "unit": "tokens/s", "cores": int(threads), "kind": "oracle",
             "sample": f"first {nrec} records ({tok} tokens) of the {wl.name} workload through the FP64 oracle "
                       f"(NER, spans, HMAC substitution) in {dt:.1f} s"}
    return entry, {"nrec": nrec, "z": np.concatenate(zs), "outputs": outs}


def parity_leg(wl, rb, W, pure: dict, gpu: dict, scales=None, key: bytes | None = None) -> dict:
    """Logit error and label agreement of the GPU path on the oracle's sample
    records (part of the CPU baseline leg): against the pure FP64 oracle and,
    for BF16/FP8, against the oracle that rounds where the GPU stores.  With
    the key, also the span and record gates: every span whose tokens and two
    neighbours are confident (oracle margin > 1e-2) is the same on both sides,
    and every record whose tokens are all confident has byte-identical output
    (tokens the perturbed oracle shows ambiguous count as not confident)."""
    from oracle import encoder, pipeline as opipe, spans as ospans
    MARGIN = 1e-2
    nrec = pure["nrec"]
    n = int(rb.cu_seqlens[nrec])
    zg, lg = gpu["z"][:n].astype(np.float64), gpu["labels"][:n]
    sub = rb.subset(range(nrec))

    def gates(lr, mr, outs_ref, exclude=()):
        g = ospans.confident_span_gate(lg, lr, mr, sub.tok_off, sub.cu_seqlens, wl.model.n_types, MARGIN, exclude)
        ok = mr > MARGIN
        if len(exclude):
            ok[np.asarray(list(exclude), dtype=np.int64)] = False
        cu = sub.cu_seqlens
        recs = [b for b in range(nrec) if ok[cu[b]:cu[b + 1]].all()]
        return {"confident_oracle_spans": g["confident_ref_spans"],
                "confident_oracle_spans_missing_on_gpu": len(g["missing_in_a"]),
                "confident_gpu_spans": g["confident_a_spans"],
                "confident_gpu_spans_not_in_oracle": len(g["missing_in_ref"]),
                "confident_records": len(recs),
                "confident_records_bytes_equal": int(sum(gpu["outputs"][b] == outs_ref[b] for b in recs))}

    def compare(zr):
        lr, mr = encoder.argmax_margin(zr)
        d = np.abs(zg - zr)
        conf = mr > MARGIN
        return {"max_abs_logit_err": float(d.max()), "rms_logit_err": float(np.sqrt((d ** 2).mean())),
                "rel_frobenius": float(np.linalg.norm(zg - zr) / max(np.linalg.norm(zr), 1e-30)),
                "label_agreement_all": float((lg == lr).mean()),
                "label_agreement_confident": float((lg[conf] == lr[conf]).mean()) if conf.any() else 1.0,
                "confident_label_mismatches": int((conf & (lg != lr)).sum()),
                "tokens_margin_le_1e-2": int((~conf).sum())}

    out = {"records": nrec, "tokens": n, "vs_pure_fp64_oracle": compare(pure["z"])}
    if key is not None:
        lp, mp = encoder.argmax_margin(pure["z"])
        out["vs_pure_fp64_oracle"].update(gates(lp, mp, pure["outputs"]))
    if wl.precision != "fp32":
        prec = encoder.Precision(wl.precision, [list(map(float, r)) for r in np.asarray(scales).reshape(-1, 4)]
                                 if scales is not None else [])
        t0 = time.perf_counter()
        zq, lq, mq = encoder.forward(W, wl.model, sub.ids, sub.cu_seqlens, prec)
        out["vs_rounding_oracle"] = r = compare(zq)
        r["oracle_s"] = time.perf_counter() - t0
        # the confident mismatches: ambiguous ones are those where the oracle
        # perturbed by 1e-7 before each rounding (3 seeds, run on the records
        # that hold them) also gives the GPU's label or a margin below its own
        # deviation
        bad = np.nonzero((mq > MARGIN) & (lg != lq))[0]
        accepted = []
        if len(bad):
            from oracle import sensitivity
            recs = sorted(set(int(np.searchsorted(rb.cu_seqlens, t, side="right") - 1) for t in bad))
            for rec in recs:
                a, b = int(rb.cu_seqlens[rec]), int(rb.cu_seqlens[rec + 1])
                one = rb.subset([rec])
                runs = [sensitivity.perturbed_forward(W, wl.model, one.ids, one.cu_seqlens, wl.precision, sd,
                                                      act_scales=prec.act_scales or None) for sd in (1, 2, 3)]
                tok = [int(t) - a for t in bad if a <= t < b]
                accepted += [a + int(t) for t in sensitivity.ambiguous_tokens(lg[a:b], zq[a:b], tok, runs)]
            r["confident_mismatches_ambiguous"] = len(accepted)
            r["confident_mismatches_unexplained"] = int(len(bad) - len(accepted))
        if key is not None:
            outs_q = opipe.run(W, wl.model, sub, key, 10, labels_override=lq).outputs
            r.update(gates(lq, mq, outs_q, accepted))
    out["outputs_equal_pure_oracle"] = int(sum(a == b for a, b in zip(gpu["outputs"][:nrec], pure["outputs"])))
    return out


def serve_bench(rates, seconds: float, warm_s: float, seed: int = 0, log=None, streams: int = 3,
                max_tok: int = 131072, graph_buckets: int = 8) -> dict:
    """Continuous-batching server under Poisson arrivals (serving workload).

    Requests hold U{1..200} records with the base workload's length
    distribution (drawn from a generated pool of records); arrivals are
    Poisson at each rate for `seconds` after `warm_s` of warm-up traffic.
    Latency = completion - submission per request.  With graph_buckets > 0
    every micro-batch's NER forward is one replay of a token-bucket graph.
    """
    import threading

    import synth
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import Pipeline

    wl = synth.workload("base_bf16")
    cfg = wl.model
    pool = synth.generate_records(4096, wl.lengths, cfg.n_types, cfg.vocab, seed + 1000)
    W = synth.make_weights(cfg, wl.weight_seed, wl.o_target)
    model = api.Model(cfg, synth.weights_blob(cfg, W), "bf16")
    cache = api.PseudonymCache(synth.make_key(0), 10, pool.type_names, 1 << 20)
    Pipeline(model, cache).autotune(max_tok, 1)
    results = []
    for rate in rates:
        sv = api.Server(model, cache, hbm_budget_bytes=64 << 30, max_batch_tokens=max_tok, n_streams=streams,
                        max_queue=100000, graph_buckets=graph_buckets)
        rng = np.random.default_rng(seed + int(rate))
        # request = a run of consecutive pool records (wrapping), U{1..200} long
        reqs = []
        t_total = warm_s + seconds
        t = 0.0
        while t < t_total:
            t += rng.exponential(1.0 / rate)
            n = int(rng.integers(1, 201))
            r0 = int(rng.integers(0, pool.n_records - n))
            reqs.append((t, pool.subset(range(r0, r0 + n))))
        done: list = []
        tickets: list = []
        lock = threading.Lock()
        stop = threading.Event()

        def poller():
            pending = []
            while not stop.is_set() or pending or len(done) < len(tickets):
                with lock:
                    pending.extend(tickets[len(done) + len(pending):])
                still = []
                for (tk, t_arr, ntok) in pending:
                    r = sv.poll(tk)
                    if r is None:
                        still.append((tk, t_arr, ntok))
                    else:
                        done.append((t_arr, r["t_submit"], r["t_done"], ntok, r["status"]))
                        sv.release(tk)
                pending = still
                if stop.is_set() and not pending and len(done) >= len(tickets):
                    break
                time.sleep(0.0005)

        th = threading.Thread(target=poller)
        th.start()
        t0 = time.perf_counter()
        for (t_arr, q) in reqs:
            dt = t_arr - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tk = sv.submit(q.ids, q.cu_seqlens, q.tok_off, q.text, q.cu_bytes)
            with lock:
                tickets.append((tk, t_arr, q.n_tokens))
        stop.set()
        th.join()
        wall = time.perf_counter() - t0
        sst = sv.stats()
        sv.stop()
        meas = [d for d in done if d[0] >= warm_s and d[4] == 0]
        lat = np.array([d[2] - d[1] for d in meas]) * 1e3
        t_first = min(d[1] for d in meas)
        t_last = max(d[2] for d in meas)
        tok = sum(d[3] for d in meas)
        offered = sum(q.n_tokens for (ta, q) in reqs if ta >= warm_s) / seconds
        results.append({"rate_req_s": rate, "requests": len(meas), "p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                        "tokens_per_s": tok / (t_last - t_first), "offered_tokens_per_s": offered,
                        "failed": sum(1 for d in done if d[4] != 0), "wall_s": wall,
                        "micro_batches": sst["micro_batches"], "graph_launches": sst["graph_launches"]})
        print(json.dumps({"serve_partial": results[-1]}), file=log or sys.stdout, flush=True)
    model.close()
    cache.close()
    return {"metric": "serving p50/p99 request latency", "unit": "ms", "workload": "serve_bf16",
            "config": {"model": "12L h768 BF16", "requests": "Poisson arrivals, U{1..200} records each, "
                       "lengths as base_bf16", "hbm_budget": "64 GiB", "max_batch_tokens": max_tok,
                       "streams": streams, "graph_buckets": graph_buckets}, "rates": results}


def stream_bench(max_chunk_tokens: int = 2_000_000, warm_chunks: int | None = None) -> dict:
    """Dataset-scale streaming workload: 70,951 records (~550 MB) windowed at
    512 tokens with 64-token overlap, processed in chunks with every input
    resident in HBM and one pseudonym table across chunks."""
    import torch

    import synth
    from synth.records import generate_records_fast
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline

    wl = synth.workload("stream_bf16")
    cfg = wl.model
    t0 = time.perf_counter()
    rb = generate_records_fast(wl.n_records, wl.lengths, cfg.n_types, cfg.vocab, wl.seed, zipf_pool=wl.zipf_pool,
                               zipf_s=wl.zipf_s)
    W = synth.make_weights(cfg, wl.weight_seed, wl.o_target)
    gen_s = time.perf_counter() - t0
    model = api.Model(cfg, synth.weights_blob(cfg, W), "bf16")
    cache = api.PseudonymCache(synth.make_key(0), 10, rb.type_names, 1 << 20)
    pl = Pipeline(model, cache)
    cu = rb.cu_seqlens.astype(np.int64)
    cb = rb.cu_bytes
    # chunks of consecutive records under a token budget
    chunks, r0 = [], 0
    while r0 < rb.n_records:
        r1 = r0 + 1
        while r1 < rb.n_records and cu[r1 + 1] - cu[r0] <= max_chunk_tokens:
            r1 += 1
        chunks.append((r0, r1))
        r0 = r1
    dev = torch.device("cuda:0")
    ids = torch.from_numpy(rb.ids).to(dev)
    tok_off = torch.from_numpy(rb.tok_off).to(dev)
    text = torch.from_numpy(np.frombuffer(rb.text, np.uint8).copy()).to(dev)
    h_cus = [(cu[a:b + 1] - cu[a]).astype(np.int32) for a, b in chunks]
    d_cus = [torch.from_numpy(c).to(dev) for c in h_cus]
    d_cbs = [torch.from_numpy((cb[a:b + 1] - cb[a]).astype(np.int64)).to(dev) for a, b in chunks]
    max_ws = max(model.windowed_workspace_size(c, 512, 448) for c in h_cus)
    pl.autotune(min(max_chunk_tokens, 1 << 20), 1)
    ws = torch.empty(max_ws, dtype=torch.uint8, device=dev)
    pl._ws["ner_win"] = ws

    class Chunk:
        pass

    def run(stream_pass: bool, n_chunks: int | None = None):
        n_spans = 0
        for k, (a, b) in enumerate(chunks[:n_chunks]):
            c = Chunk()
            c.B, c.T = b - a, int(cu[b] - cu[a])
            c.n_bytes = int(cb[b] - cb[a])
            c.h_cu = h_cus[k]
            c.ids = ids[int(cu[a]):int(cu[b])]
            c.cu = d_cus[k]
            c.tok_off = tok_off[int(cu[a]):int(cu[b])]
            c.text = text[int(cb[a]):int(cb[b])]
            c.cu_bytes = d_cbs[k]
            labels, _, _ = pl.ner(c, logits=False, margin=False, window=512, stride=448)
            spans, cu_spans, cap = pl.spans(c, labels)
            pl.pseudonymize(c, spans, cu_spans, cap)
            if k % 8 == 0:
                print(f"[stream] {'timed' if stream_pass else 'warm-up'} chunk {k + 1}/{len(chunks)}",
                      file=sys.stderr, flush=True)
        return n_spans

    run(False, warm_chunks)  # warm-up (the table is cleared before the timed pass)
    cache.clear()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    st = cache.stats()
    # hit rate of the table on the gold (Zipf-distributed) entity spans
    gold_cache = api.PseudonymCache(synth.make_key(0), 10, rb.type_names, 1 << 20)
    gsp = rb.gold_spans
    raw = np.zeros((max(len(gsp), 1), 3), np.int64)
    raw[:len(gsp), 0] = (gsp[:, 0] & 0xFFFFFFFF) | (gsp[:, 1] << 32)
    raw[:len(gsp), 1:] = gsp[:, 2:]
    d_gsp = torch.from_numpy(raw).to(dev)
    counts = np.bincount(gsp[:, 0], minlength=rb.n_records)
    d_gcu = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)).to(dev)
    full = Chunk()
    full.B, full.T, full.n_bytes = rb.n_records, rb.n_tokens, len(rb.text)
    full.text, full.cu_bytes = text, torch.from_numpy(cb).to(dev)
    gp = Pipeline(model, gold_cache)
    tg = time.perf_counter()
    gp.pseudonymize(full, d_gsp, d_gcu, len(gsp))
    torch.cuda.synchronize()
    tg = time.perf_counter() - tg
    gst = gold_cache.stats()
    # the schema-configured path (no NER) over the whole dataset in one call:
    # field spans of the generator's field names, then substitution
    from synth.records import _FIELD_OF
    config = {n: rb.type_names.index(t) + 1 for t, names in _FIELD_OF.items() if t in rb.type_names
              for n in names}
    fcache = api.PseudonymCache(synth.make_key(0), 10, rb.type_names, 1 << 22)
    fp = Pipeline(model, fcache)
    fp.step_fields(full, config)  # warm-up
    fcache.clear()
    torch.cuda.synchronize()
    tf = time.perf_counter()
    _, cu_f, _, _ = fp.step_fields(full, config)
    torch.cuda.synchronize()
    tf = time.perf_counter() - tf
    fst = fcache.stats()
    schema = {"seconds": tf, "text_bytes_per_s": len(rb.text) / tf, "spans": int(cu_f[-1].item()),
              "fields": len(config), "pcache": {**fst, "hit_rate": fst["hits"] / max(fst["lookups"], 1)},
              "paper_context": "with the schema configuration the paper reports 12.55 s for D2-CSV "
                               "(34,341 KB/s) on an RTX 5060 Ti + Ryzen 5 8600G (Table VI)"}
    # the recognizers alone (no NER spans) over the whole dataset in one call,
    # then substitution
    rcache = api.PseudonymCache(synth.make_key(0), 10, rb.type_names, 1 << 22)
    rp = Pipeline(model, rcache)
    sp_r, cu_r, cap_r = rp.recognize(full)  # warm-up
    rp.pseudonymize(full, sp_r, cu_r, cap_r)
    rcache.clear()
    torch.cuda.synchronize()
    tr = time.perf_counter()
    sp_r, cu_r, cap_r = rp.recognize(full)
    rp.pseudonymize(full, sp_r, cu_r, cap_r)
    torch.cuda.synchronize()
    tr = time.perf_counter() - tr
    recog_only = {"seconds": tr, "text_bytes_per_s": len(rb.text) / tr, "spans": int(cu_r[-1].item())}
    del fp, rp, sp_r
    fcache.close()
    rcache.close()
    L = np.diff(cu)
    nw = np.where(L > 512, 1 + -(-(L - 512) // 448), 1)
    win_pos = int(np.sum(np.where(L > 512, (nw - 1) * 512 + (L - (nw - 1) * 448), L)))
    out = {"metric": "NER+pseudonymize tokens/sec/GPU (dataset-scale stream)", "value": rb.n_tokens / wall,
           "unit": "tokens/s", "dtype": "bf16", "data": "synthetic", "wall_s": wall,
           "config": {"workload": wl.name, "records": rb.n_records, "tokens": rb.n_tokens,
                      "text_mb": len(rb.text) / 1e6, "window": 512, "stride": 448, "window_positions": win_pos,
                      "chunks": len(chunks), "max_chunk_tokens": max_chunk_tokens, "zipf_pool": wl.zipf_pool,
                      "zipf_s": wl.zipf_s},
           "pcache_predicted_spans": {**st, "hit_rate": st["hits"] / max(st["lookups"], 1)},
           "pcache_gold_spans": {**gst, "hit_rate": gst["hits"] / max(gst["lookups"], 1), "spans": int(len(gsp)),
                                 "seconds": tg},
           "schema_fields": schema,
           "recognizers_only": recog_only,
           "input_gen_s": gen_s,
           "paper_context": "550.54 MB / 70,951 records in 453.1 s on an RTX 5060 Ti + Ryzen 5 8600G, "
                            "full pipeline, precision not stated (Table VI)"}
    model.close()
    cache.close()
    gold_cache.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="base_bf16")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--serve", default="", help="comma-separated request rates: run the serving benchmark")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-streams", type=int, default=3, help="server slots (HIP streams)")
    ap.add_argument("--serve-max-tokens", type=int, default=131072, help="tokens per micro-batch at most")
    ap.add_argument("--serve-graphs", type=int, default=8,
                    help="token-bucket graphs per server slot (0: launch the forward kernel by kernel)")
    ap.add_argument("--calib-copy", action="store_true", help="run a 1 GiB device copy first (counter scale)")
    ap.add_argument("--ffn1-group", type=int, default=-1,
                    help="profiling runs: the FFN1 tile order after the autotuner (0 = by shape, N = groups of N "
                         "row blocks; default: the autotuner's)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short serving run (100 req/s) of the default line")
    ap.add_argument("--no-recognizers", action="store_true",
                    help="skip the timings of the recognizer and schema-field paths")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 path on the large workload")
    ap.add_argument("--no-modern", action="store_true", help="skip the ModernBERT-style encoder's path")
    ap.add_argument("--no-stream", action="store_true", help="skip the dataset-scale stream")
    ap.add_argument("--fp8-steps", type=int, default=3)
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1 "
                                   "(records are independent and shard across GPUs without communication)"}))
        return 2
    if a.serve:
        rates = [float(x) for x in a.serve.split(",")]
        print(json.dumps(serve_bench(rates, a.serve_seconds, a.serve_warmup, streams=a.serve_streams,
                                     max_tok=a.serve_max_tokens, graph_buckets=a.serve_graphs)), flush=True)
        return 0
    if a.workload == "stream_bf16":
        print(json.dumps(stream_bench()), flush=True)
        return 0
    if a.calib_copy:
        # a plain device copy of known size (1 GiB read + 1 GiB write), used to
        # scale the FETCH_SIZE / WRITE_SIZE counters of a profiled run
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    import torch

    import synth
    from paper_2606_15650_amd import api
    from paper_2606_15650_amd.pipeline import DeviceBatch, Pipeline, outputs_to_list

    def path_bench(wl_name: str, steps: int, warmup: int, extras: bool, fp32: bool, keep_logits: bool) -> dict:
        """One workload: generate it, time `steps` whole-path steps (the path in
        the workload's precision), the dominant kernel against its roofline,
        optionally the recognizer / schema-field / graph timings and the FP32
        path on the same batch; with keep_logits the GPU logits, labels and
        outputs of one more step are returned for the parity leg."""
        wl = synth.workload(wl_name)
        cfg = wl.model
        t_gen = time.perf_counter()
        rb = synth.generate_records(wl.n_records, wl.lengths, cfg.n_types, cfg.vocab, wl.seed)
        W = synth.make_weights(cfg, wl.weight_seed, wl.o_target)
        key = synth.make_key(0)
        blob = synth.weights_blob(cfg, W)
        gen_s = time.perf_counter() - t_gen
        T, B = rb.n_tokens, rb.n_records
        cu = rb.cu_seqlens.astype(np.int64)
        scales = None
        if wl.precision == "fp8":
            # static per-tensor activation scales, calibrated once by the oracle
            with open(os.path.join(ROOT, "tests", "golden", f"fp8_scales_{wl.name}.json")) as f:
                scales = np.asarray(json.load(f)["scales"], np.float32).reshape(-1)
        kept = {}

        def run_path(precision: str, steps: int, warmup: int, prof: bool, extras: bool = False):
            model = api.Model(cfg, blob, precision, act_scales=scales if precision == "fp8" else None)
            cache = api.PseudonymCache(key, 10, rb.type_names, 1 << 20)
            pl = Pipeline(model, cache)
            db = DeviceBatch(rb)
            stream = torch.cuda.current_stream()
            tiles, _ = pl.autotune(T, B)
            if a.ffn1_group >= 0:  # a fixed FFN1 tile order (counter runs cover every order)
                g = model.get_tiles()[1]
                g[2] = a.ffn1_group
                model.set_tile_groups(g)
            attn_pick, attn_times = pl.autotune_attention(db)
            kept["attn_config"] = {"chosen": model.attn_configs()[attn_pick] if attn_pick >= 0 else "fp32",
                                   "times_ms": {n: float(t) for n, t in zip(model.attn_configs(), attn_times)
                                                if t >= 0}}
            groups = model.get_tiles()[1]
            tiles = [f"{model.tile_configs()[t]}_g{g if g else 'auto'}" for t, g in zip(tiles, groups)]
            # every step pseudonymizes the batch as a new one: the pseudonym
            # table starts empty (a fill kernel on the stream, inside the timed
            # region), so each distinct entity of the batch is hashed every step
            for _ in range(warmup):
                cache.clear(stream)
                pl.step(db)
            torch.cuda.synchronize()
            classes = ["qkv", "attn", "oproj", "ffn1", "ffn2", "ln", "embed", "cls"]
            if prof:
                for k in classes:
                    api.prof_enable(k, True)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev[0].record(stream)
            for i in range(steps):
                cache.clear(stream)
                pl.step(db)
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
            kern = {}
            if prof:
                for k in classes:
                    kern[k] = api.prof_read(k)
                    api.prof_enable(k, False)
            st = cache.stats()
            if keep_logits and precision == wl.precision:
                # one more (untimed) pass for the parity leg: logits, labels, outputs
                _, z, _ = pl.ner(db, logits=True)
                labels, spans, cu_spans, out, cu_out = pl.step(db)
                torch.cuda.synchronize()
                kept["z"] = z[:T].cpu().numpy()
                kept["labels"] = labels[:T].cpu().numpy()
                kept["outputs"] = outputs_to_list(out, cu_out)
            rx = recognizer_timing(pl, db, stream, max(2, steps // 2)) if extras else None
            fd = field_timing(pl, db, stream, 10) if extras else None
            gr = graph_timing(pl, db, stream, max(2, steps // 2)) if extras else None
            model.close()
            cache.close()
            return wall, per, kern, st, tiles, rx, fd, gr

        def graph_timing(pl, db, stream, steps: int) -> dict:
            """ner_forward over the batch as one HIP graph (ner_forward_capture)
            against the same call launched kernel by kernel; labels compared."""
            lab_e, _, mg_e = pl.ner(db, stream=stream)
            ws = pl._buf("ner_graph", pl.model.workspace_size(db.T, db.B))
            lab_g = torch.empty_like(lab_e)
            mg_g = torch.empty_like(mg_e)
            g = api.ner_forward_capture(pl.model, db.ids, db.cu, db.B, db.T, lab_g, None, mg_g, ws, ws.numel())
            g.launch(stream)
            torch.cuda.synchronize()
            same = bool(torch.equal(lab_e, lab_g) and torch.equal(mg_e, mg_g))
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record(stream)
            for _ in range(steps):
                pl.ner(db, stream=stream)
            ev[1].record(stream)
            ev[2].record(stream)
            for _ in range(steps):
                g.launch(stream)
            ev[3].record(stream)
            torch.cuda.synchronize()
            g.close()
            return {"eager_ner_ms": ev[0].elapsed_time(ev[1]) / steps,
                    "graph_ner_ms": ev[2].elapsed_time(ev[3]) / steps, "labels_and_margins_equal": same}

        def field_timing(pl, db, stream, steps: int) -> dict:
            """The schema-configured path (whole-field spans of the generator's
            field names, then substitution; no NER) over the same batch."""
            from synth.records import _FIELD_OF
            config = {n: rb.type_names.index(t) + 1 for t, names in _FIELD_OF.items() if t in rb.type_names
                      for n in names}
            pl.step_fields(db, config)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
            for i in range(steps):
                ev[2 * i].record(stream)
                spans, cu_f, out, cu_out = pl.step_fields(db, config, stream=stream)
                ev[2 * i + 1].record(stream)
            torch.cuda.synchronize()
            ms = float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)]))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pl.fields(db, config, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            return {"value": db.n_bytes / (ms * 1e-3), "unit": "text bytes/s", "ms_per_step": ms,
                    "field_spans_ms": e0.elapsed_time(e1), "text_bytes": db.n_bytes, "records": db.B,
                    "spans": int(cu_f[-1].item()), "fields": len(config),
                    "paper_context": "with the schema configuration the paper reports 34,341 KB/s (D2, CSV) and "
                                     "31,272 KB/s (D3) on an RTX 5060 Ti + Ryzen 5 8600G (Table VI)"}

        def recognizer_timing(pl, db, stream, steps: int) -> dict:
            """The same step with the pattern recognizers merged into the NER spans,
            and recognize_spans alone (HIP events on its stream) over the batch text."""
            pl.step(db, recognizers=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                pl.step(db, recognizers=True)
            torch.cuda.synchronize()
            wall_r = time.perf_counter() - t0
            labels, _, _ = pl.ner(db, logits=False, margin=False, stream=stream)
            spans, cu_spans, cap = pl.spans(db, labels, stream=stream)
            reps = 10
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
            for i in range(reps):
                ev[2 * i].record(stream)
                _, cu_r, _ = pl.recognize(db, spans, cu_spans, cap, stream=stream)
                ev[2 * i + 1].record(stream)
            torch.cuda.synchronize()
            ms = float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]))
            return {"value": T * steps / wall_r, "unit": "tokens/s", "ms_per_step": wall_r / steps * 1e3,
                    "recognize_ms": ms, "text_bytes": db.n_bytes, "text_GBps": db.n_bytes / (ms * 1e-3) / 1e9,
                    "ner_spans": int(cu_spans[-1].item()), "merged_spans": int(cu_r[-1].item()),
                    "recognizers": api.RECOGNIZERS}

        wall, per, kern, cstats, tiles, rx, fd, gr = run_path(wl.precision, steps, warmup, prof=True, extras=extras)
        tokens_per_s = T * steps / wall
        # dominant kernel class (largest total time) against its roofline
        gemm_tok = gemm_flops_per_token(cfg)
        total_att = attention_flops(cu, cfg)
        dom = max(kern, key=lambda k: kern[k]["ms"])
        d = kern[dom]
        peak_key = wl.precision
        if dom in gemm_tok:
            flops_per_launch = gemm_tok[dom] * T
        elif dom == "attn":
            flops_per_launch = total_att
            peak_key = "bf16" if wl.precision != "fp32" else "fp32"   # attention runs on bf16 operands
        else:
            flops_per_launch = None
        peak = PEAK_FLOPS[peak_key]
        avg_ms = d["ms"] / max(d["launches"], 1)
        achieved = flops_per_launch / (avg_ms * 1e-3) if flops_per_launch else None
        tile_of = dict(zip(["qkv", "oproj", "ffn1", "ffn2"], tiles))
        traffic, traffic_src = counter_traffic(wl.name, dom, tile_of.get(dom))
        roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12, "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic, "traffic_source": traffic_src,
                    "avg_launch_ms": avg_ms, "flops_per_launch": flops_per_launch, "peak_dtype": peak_key}
        breakdown = {}
        for k, v in kern.items():
            if v["launches"]:
                f = gemm_tok[k] * T * v["launches"] if k in gemm_tok else (
                    total_att * v["launches"] if k == "attn" else 0)
                breakdown[k] = {"launches": v["launches"], "ms_per_step": v["ms"] / steps,
                                "tflops": (f / (v["ms"] * 1e-3) / 1e12) if f else None}
        flops = path_flops(cfg, cu)
        out = {
            "metric": "NER+pseudonymize tokens/sec/GPU",
            "value": tokens_per_s,
            "unit": "tokens/s",
            "n_gpus": 1,
            "steps": steps,
            "warmup": warmup,
            "ms_per_step": wall / steps * 1e3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": wl.precision,
            "data": "synthetic",
            "config": {"workload": wl.name, "records": B, "tokens": T, "layers": cfg.n_layers, "hidden": cfg.hidden,
                       "heads": cfg.n_heads, "ffn": cfg.ffn, "vocab": cfg.vocab, "labels": cfg.n_labels,
                       "lengths": list(wl.lengths), "packing": "varlen, no padding", "parallelism": "single GPU"},
            "roofline": roofline,
            "path_tflops": flops / (wall / steps) / 1e12,
            "path_mfma_frac": flops / (wall / steps) / PEAK_FLOPS[wl.precision],
            "step_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                                "mean": float(per.mean())},
            "kernels": breakdown,
            "pcache": {**cstats, "per_step": "table cleared before every timed step (cold: every distinct "
                                              "entity of the batch is hashed in every step)"},
            "gemm_tiles": dict(zip(["qkv", "oproj", "ffn1", "ffn2"], tiles)),
            "attention_tiles": kept.get("attn_config"),
            "input_gen_s": gen_s,
        }
        if rx is not None:
            out["with_recognizers"] = rx
        if fd is not None:
            out["schema_fields"] = fd
        if gr is not None:
            out["ner_graph"] = gr
        if fp32 and wl.precision != "fp32":
            w32, per32, _, _, _, _, _, _ = run_path("fp32", max(2, steps // 4), 1, prof=False)
            tps32 = T * max(2, steps // 4) / w32
            out["fp32_path"] = {"value": tps32, "unit": "tokens/s", "speedup": tokens_per_s / tps32}
        ctx = {"wl": wl, "rb": rb, "W": W, "key": key, "scales": scales, "gpu": kept}
        return out, ctx

    out, ctx = path_bench(a.workload, a.steps, a.warmup, extras=not a.no_recognizers, fp32=not a.no_fp32,
                          keep_logits=not a.no_cpu)
    if not a.no_serve and a.workload == "base_bf16":
        # request latency under streaming load: the serving workload at three
        # rates, 10 s of arrivals each after 1.5 s of warm-up, forward passes
        # as token-bucket graph replays; the middle rate again with kernel-by-
        # kernel launches; `--serve RATES` runs any sweep
        keys = ("rate_req_s", "requests", "p50_ms", "p99_ms", "mean_ms", "tokens_per_s", "offered_tokens_per_s",
                "failed", "micro_batches", "graph_launches")
        sv = serve_bench([50.0, 100.0, 200.0], 10.0, 1.5, log=sys.stderr, graph_buckets=8)
        ev = serve_bench([100.0], 10.0, 1.5, log=sys.stderr, graph_buckets=0)
        out["serving"] = {"workload": sv["workload"], "seconds_per_rate": 10.0, "config": sv["config"],
                          "rates": [{k: r[k] for k in keys} for r in sv["rates"]],
                          "eager_launches": [{k: r[k] for k in keys} for r in ev["rates"]]}
    if not a.no_stream and a.workload == "base_bf16":
        # the dataset-scale stream (70,951 records, 554 MB, windows of 512
        # every 448): one timed pass over the whole dataset
        print("[bench] dataset-scale stream", file=sys.stderr, flush=True)
        st = stream_bench(warm_chunks=1)
        out["stream_path"] = {k: st[k] for k in ("value", "unit", "wall_s", "config", "pcache_predicted_spans",
                                                 "pcache_gold_spans", "schema_fields", "recognizers_only",
                                                 "input_gen_s", "paper_context")}
    mctx = None
    if not a.no_modern and a.workload == "base_bf16":
        print("[bench] ModernBERT-style path", file=sys.stderr, flush=True)
        out["modernbert_path"], mctx = modern_bench(max(2, a.steps // 2), 1, keep=not a.no_cpu)
    fp8 = None
    if not a.no_fp8 and a.workload == "base_bf16":
        # the FP8-E4M3 path on its own workload (24 layers, h1024), a few steps
        print("[bench] large_fp8 path", file=sys.stderr, flush=True)
        fp8, fctx = path_bench("large_fp8", a.fp8_steps, 1, extras=False, fp32=False, keep_logits=not a.no_cpu)
        out["fp8_path"] = {k: fp8[k] for k in ("value", "unit", "ms_per_step", "steps", "config", "roofline",
                                               "path_tflops", "path_mfma_frac", "kernels", "gemm_tiles",
                                               "attention_tiles")}
    if not a.no_cpu:
        base, pure = cpu_baseline(ctx["wl"], ctx["rb"], ctx["W"], ctx["key"], a.cpu_budget)
        out["cpu_baseline"] = base
        out["parity"] = parity_leg(ctx["wl"], ctx["rb"], ctx["W"], pure, ctx["gpu"], ctx["scales"], ctx["key"])
        if mctx is not None:
            out["modernbert_path"]["parity"] = modern_parity(mctx, a.cpu_budget / 2)
        if fp8 is not None:
            # a short sample of the FP8 workload (24-layer oracle: a few records)
            _, fpure = cpu_baseline(fctx["wl"], fctx["rb"], fctx["W"], fctx["key"], a.cpu_budget / 3)
            out["fp8_path"]["parity"] = parity_leg(fctx["wl"], fctx["rb"], fctx["W"], fpure, fctx["gpu"],
                                                   fctx["scales"], fctx["key"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
