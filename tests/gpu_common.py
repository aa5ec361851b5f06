"""Shared helpers of the GPU tests: model/cache construction and comparisons."""
from __future__ import annotations

import sys

import numpy as np

import synth
from synth.configs import ModelConfig

MARGIN = 1e-2        # labels must agree where the reference margin exceeds this
FP32_LOGIT_RTOL = 1e-4


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
