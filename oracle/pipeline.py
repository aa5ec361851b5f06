"""The whole path over a packed batch: NER, (window merge), spans, pseudonyms.

Test infrastructure only.  Composes oracle.encoder, oracle.spans and
oracle.pseudonym in the paper's order (Sec. II: detection, then HMAC
pseudonymisation and substitution).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import encoder, pseudonym, spans as spans_mod


@dataclass
class OracleResult:
    logits: np.ndarray      # [T, C] float64
    labels: np.ndarray      # [T] uint8
    margin: np.ndarray      # [T] float64
    spans: np.ndarray       # [S, 4] (record, type, begin, end)
    outputs: list           # per-record output bytes


def ner(W, cfg, ids, cu_seqlens, prec=None, window: int = 0, stride: int = 0):
    """Logits, labels and margins per record token, windowed if ``window`` > 0."""
    if not window:
        return encoder.forward(W, cfg, ids, cu_seqlens, prec)
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    win = spans_mod.windows(cu, window, stride)
    w_ids = np.concatenate([ids[cu[r] + s: cu[r] + s + n] for r, s, n in win.tolist()])
    w_cu = np.concatenate([[0], np.cumsum(win[:, 2])]).astype(np.int64)
    z_w, _, _ = encoder.forward(W, cfg, w_ids, w_cu, prec)
    z = np.empty((int(cu[-1]), z_w.shape[1]))
    wi = 0
    for r in range(len(cu) - 1):
        n = int(cu[r + 1] - cu[r])
        starts = spans_mod.window_starts(n, window, stride)
        own = spans_mod.owner_window(n, window, stride)
        for i in range(n):
            k = int(own[i])
            z[cu[r] + i] = z_w[w_cu[wi + k] + (i - starts[k])]
        wi += len(starts)
    labels, margin = encoder.argmax_margin(z)
    return z, labels, margin


def run(W, cfg, batch, key: bytes, slug_len: int, prec=None, window: int = 0, stride: int = 0,
        labels_override=None) -> OracleResult:
    """The whole path; with ``labels_override`` the NER stage is skipped and
    the given labels are decoded and substituted (logits and margins None)."""
    if labels_override is not None:
        z, labels, margin = None, np.asarray(labels_override), None
    else:
        z, labels, margin = ner(W, cfg, batch.ids, batch.cu_seqlens, prec, window, stride)
    sp = spans_mod.bio_decode(labels, batch.tok_off, batch.cu_seqlens, cfg.n_types)
    outs = pseudonym.pseudonymize_batch(batch.text, batch.cu_bytes, sp, batch.n_records,
                                        batch.type_names, key, slug_len)
    return OracleResult(z, labels, margin, sp, outs)
