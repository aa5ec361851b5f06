"""Shared helpers of the GPU tests: model/cache construction and comparisons."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

import synth
from synth.configs import ModelConfig

MARGIN = 1e-2        # labels must agree where the reference margin exceeds this
FP32_LOGIT_RTOL = 1e-4

# Reduced precision: the largest logit deviation from the rounding oracle.
# At 2 layers the deviation stays near 1e-3.  Deeper models are held to twice
# the spread the oracle itself shows when every value it rounds to bf16 moves
# by 1e-7 first (the size of FP32 summation differences): no bf16 evaluation
# can be held closer.  The spreads are measured by oracle/sensitivity.py on
# the base (12-layer BF16) and large (24-layer FP8) models.  Labels are held
# to the oracle wherever its margin exceeds 1e-2 at every depth
# (reduced_label_gate).
def _probe_bound(name: str) -> float:
    with open(os.path.join(GOLDEN, f"sensitivity_{name}.json")) as f:
        return 2.0 * json.load(f)["perturbed_vs_rounding_oracle"]["max"]


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LOGIT_BOUND = {("bf16", 2): 5e-3, ("fp8", 2): 5e-3, ("bf16", 12): _probe_bound("base_bf16"),
               ("fp8", 24): _probe_bound("large_fp8")}
PERTURB_SEEDS = (1, 2, 3)


def oracle_ner(W, cfg, ids, cu_seqlens, make_prec=None, window: int = 0, stride: int = 0, workers: int | None = None,
               forward=None):
    """The oracle's NER (logits, labels, margins) over a packed batch, with its
    records split into contiguous groups of about equal token counts that run
    in parallel threads (numpy releases the GIL in its array work).  Each
    group is a packed batch of its own: the oracle's result for a record does
    not depend on its batch-mates (pinned on the CPU).  ``forward`` replaces
    the BERT-style oracle (e.g. oracle.modernbert.forward).  ``make_prec(g)`` gives
    group g its Precision (a fresh one per group, so that a stateful reading
    such as the perturbed one draws from its own stream)."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import pipeline as opipe
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    ids = np.asarray(ids)
    B = len(cu) - 1
    make_prec = make_prec or (lambda g: None)
    workers = workers or min(16, os.cpu_count() or 1)
    # group boundaries by token count; every token weighs at least its
    # record's share of attention (long records cost more per token)
    L = np.diff(cu).astype(np.float64)
    cost = np.cumsum(L * (1.0 + L / 256.0))
    n_groups = max(1, min(B, 2 * workers))
    bounds = [0]
    for g in range(1, n_groups):
        r = int(np.searchsorted(cost, cost[-1] * g / n_groups)) + 1
        if bounds[-1] < r < B:
            bounds.append(r)
    bounds.append(B)

    ner = forward or (lambda W_, c_, i_, cu_, p_: opipe.ner(W_, c_, i_, cu_, p_, window, stride))

    def run(g):
        a, b = bounds[g], bounds[g + 1]
        sub_cu = cu[a:b + 1] - cu[a]
        return ner(W, cfg, ids[cu[a]:cu[b]], sub_cu, make_prec(g))

    if B == 0:
        return ner(W, cfg, ids, cu, make_prec(0))
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(run, range(len(bounds) - 1)))
    z = np.concatenate([p[0] for p in parts])
    lab = np.concatenate([p[1] for p in parts])
    mg = np.concatenate([p[2] for p in parts])
    return z, lab, mg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_model(cfg: ModelConfig, precision: str, seed: int = 0, o_target=None, act_scales=None):
    from paper_2606_15650_amd import api
    W = synth.make_weights(cfg, seed, o_target)
    return W, api.Model(cfg, synth.weights_blob(cfg, W), precision, act_scales=act_scales)


def make_cache(type_names, slug=10, key_seed=0, capacity=1 << 16):
    from paper_2606_15650_amd import api
    return api.PseudonymCache(synth.make_key(key_seed), slug, type_names, capacity)


def logit_rel_err(z_gpu: np.ndarray, z_ref: np.ndarray) -> np.ndarray:
    """Per token: max |z_gpu - z_ref| / max(max |z_ref|, 1e-6)."""
    num = np.abs(z_gpu - z_ref).max(axis=1)
    den = np.maximum(np.abs(z_ref).max(axis=1), 1e-6)
    return num / den


def confident_labels_agree(lab_gpu, lab_ref, margin_ref):
    sel = margin_ref > MARGIN
    bad = np.nonzero(sel & (lab_gpu != lab_ref))[0]
    return bad, int(sel.sum())


def confident_records(margin_ref: np.ndarray, cu: np.ndarray) -> list[int]:
    return [b for b in range(len(cu) - 1) if (margin_ref[cu[b]:cu[b + 1]] > MARGIN).all()]


def reduced_label_gate(lab, zq, lq, mq, perturbed, seeds=PERTURB_SEEDS, batch=None, n_types=None) -> int:
    """Reduced-precision labels against the rounding oracle (zq, lq, mq).

    Every token whose oracle margin exceeds 1e-2 must carry the oracle's
    label, except a token shown ambiguous on its own: the oracle perturbed by
    1e-7 before each bf16 rounding (``perturbed(seed)`` -> logits, labels,
    margins on the same tokens; what FP32 accumulation amounts to) gives the
    GPU's label there for some seed, or that seed's margin at the token is
    below the seed's own largest logit deviation from the oracle.  The number
    of accepted tokens is printed, and may not exceed three times (at least
    two) the number of labels above 1e-2 that the perturbed oracle itself
    flips.  With ``batch`` (its tok_off and cu_seqlens) and ``n_types``, the
    span gate follows: every span whose tokens and two neighbours are all
    confident (accepted tokens count as not confident) is the same in the GPU's
    and the oracle's decoding, in both directions.  Returns the number of
    accepted tokens."""
    from oracle import sensitivity
    conf = mq > MARGIN
    bad = np.nonzero(conf & (lab != lq))[0]
    accepted, own_flips = [], 0
    if len(bad):
        runs = [perturbed(s) for s in seeds]
        for zn, ln, mn in runs:
            own_flips = max(own_flips, int((conf & (ln != lq)).sum()))
        accepted = sensitivity.ambiguous_tokens(lab, zq, bad, runs)
    rejected = sorted(set(bad.tolist()) - set(accepted))
    say(f"  label gate: {int(conf.sum())} tokens above margin 1e-2, {len(bad)} differ, "
        f"{len(accepted)} accepted as ambiguous (perturbed oracle flips {own_flips})")
    assert not rejected, f"labels differ above margin 1e-2 at tokens {rejected[:20]} (margins {mq[rejected[:20]]})"
    assert len(accepted) <= max(2, 3 * own_flips), (len(accepted), own_flips)
    if batch is not None:
        from oracle import spans
        g = spans.confident_span_gate(lab, lq, mq, batch.tok_off, batch.cu_seqlens, n_types, MARGIN, accepted)
        say(f"  span gate: {g['confident_ref_spans']} confident oracle spans, {len(g['missing_in_a'])} missing on "
            f"the GPU; {g['confident_a_spans']} confident GPU spans, {len(g['missing_in_ref'])} not the oracle's")
        assert not g["missing_in_a"] and not g["missing_in_ref"], g
    return len(accepted)
