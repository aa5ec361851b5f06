"""Labels to entity byte spans, and long records to windows (test infrastructure only).

BIO decoding.  Replacement (Sec. II, stage 3) acts on entity spans, so token
labels must be turned into byte ranges.  Label 0 is O; entity type t >= 1 has
B-t = 2t-1 and I-t = 2t.  Walking a record's tokens in order:

* O closes the open span;
* B-t always opens a new span of type t (closing any open one);
* I-t extends the open span if it has type t, otherwise it opens a new span
  of type t (the lenient reading of an I- tag without a matching B-);
* a span covers [begin of its first token, end of its last token).

Windows.  The encoder sees at most ``max_pos`` (512) positions, and the paper
names truncation of long inputs as a limitation (Sec. VI).  A record longer
than the window W is covered by windows starting at multiples of the stride S
(the last one may be shorter); every token takes its label from one owner
window: where windows k and k+1 overlap, the first half of the overlap belongs
to window k and the rest to window k+1.
"""
from __future__ import annotations

import numpy as np


def bio_decode_record(labels, tok_off, n_types: int) -> list[tuple[int, int, int]]:
    """Spans (type, begin, end) of one record from its labels and token byte offsets."""
    spans: list[list[int]] = []
    open_span = None
    for lab, (tb, te) in zip(np.asarray(labels).tolist(), np.asarray(tok_off).tolist()):
        if lab < 0 or lab > 2 * n_types:
            raise ValueError(f"label {lab} outside [0, {2 * n_types}]")
        if lab == 0:
            open_span = None
            continue
        typ = (lab + 1) // 2
        is_begin = (lab % 2) == 1
        if is_begin or open_span is None or open_span[0] != typ:
            open_span = [typ, tb, te]
            spans.append(open_span)
        else:
            open_span[2] = te
    return [tuple(s) for s in spans]


def bio_decode(labels, tok_off, cu_seqlens, n_types: int) -> np.ndarray:
    """Spans of a packed batch as rows (record, type, begin, end), record-major."""
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    rows = []
    for r in range(len(cu) - 1):
        a, b = int(cu[r]), int(cu[r + 1])
        rows += [(r, t, bb, ee) for (t, bb, ee) in bio_decode_record(labels[a:b], tok_off[a:b], n_types)]
    return np.asarray(rows, dtype=np.int64).reshape(-1, 4)


def window_starts(n: int, window: int, stride: int) -> list[int]:
    """Start offsets of the windows covering a record of n tokens."""
    if n <= window:
        return [0]
    k = 1 + -(-(n - window) // stride)
    return [stride * i for i in range(k)]


def owner_window(n: int, window: int, stride: int) -> np.ndarray:
    """For each of the n tokens, the index of the window that owns its label."""
    starts = window_starts(n, window, stride)
    half = (window - stride) // 2
    own = np.zeros(n, dtype=np.int64)
    for k in range(1, len(starts)):
        own[starts[k] + half:] = k
    return own


def windows(cu_seqlens, window: int, stride: int):
    """Window table of a packed batch: rows (record, start within record, length)."""
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    rows = []
    for r in range(len(cu) - 1):
        n = int(cu[r + 1] - cu[r])
        for s in window_starts(n, window, stride):
            rows.append((r, s, min(window, n - s)))
    return np.asarray(rows, dtype=np.int64).reshape(-1, 3)


def confident_spans(spans, margin, tok_off, cu_seqlens, threshold: float = 1e-2, exclude=()) -> list:
    """The spans (rows record, type, begin, end) whose tokens, and the token just
    before and just after them within their record, all have ``margin`` above
    ``threshold``; tokens listed in ``exclude`` (global indices) count as not
    confident.  Such a span is decided by confident labels only: BIO decoding
    of a span depends on the labels of its own tokens and its two neighbours.
    (Evaluation helper of the parity gates, not part of the method.)"""
    cu = np.asarray(cu_seqlens, dtype=np.int64)
    ok = np.asarray(margin) > threshold
    if len(exclude):
        ok = ok.copy()
        ok[np.asarray(list(exclude), dtype=np.int64)] = False
    tok_off = np.asarray(tok_off)
    out = []
    for r, t, b, e in np.asarray(spans, dtype=np.int64).reshape(-1, 4).tolist():
        a0, a1 = int(cu[r]), int(cu[r + 1])
        inside = np.nonzero((tok_off[a0:a1, 0] >= b) & (tok_off[a0:a1, 1] <= e))[0]
        if len(inside) == 0:
            continue
        lo, hi = max(a0 + int(inside[0]) - 1, a0), min(a0 + int(inside[-1]) + 1, a1 - 1)
        if ok[lo:hi + 1].all():
            out.append((r, t, b, e))
    return out


def confident_span_gate(labels_a, labels_ref, margin_ref, tok_off, cu_seqlens, n_types: int,
                        threshold: float = 1e-2, exclude=()) -> dict:
    """Span gate between labels ``labels_a`` and reference labels: every
    confident reference span (by the reference margins) must be among a's
    spans, and every confident span of a among the reference's.  Counts."""
    sa = bio_decode(labels_a, tok_off, cu_seqlens, n_types)
    sr = bio_decode(labels_ref, tok_off, cu_seqlens, n_types)
    ca = confident_spans(sa, margin_ref, tok_off, cu_seqlens, threshold, exclude)
    cr = confident_spans(sr, margin_ref, tok_off, cu_seqlens, threshold, exclude)
    set_a, set_r = set(map(tuple, sa.tolist())), set(map(tuple, sr.tolist()))
    return {"confident_ref_spans": len(cr), "missing_in_a": [s for s in cr if s not in set_a],
            "confident_a_spans": len(ca), "missing_in_ref": [s for s in ca if s not in set_r]}
