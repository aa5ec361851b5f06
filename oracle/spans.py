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
