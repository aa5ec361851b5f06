"""Deterministic byte-level tokenizer for synthetic scan records.

The paper runs a pretrained subword NER model (Sec. II, stage 2); neither its
vocabulary nor its weights are available, so inputs are tokenized by this small
project-defined scheme instead:

* a token is a run of ASCII letters, a run of ASCII digits, or one other
  non-whitespace byte; whitespace separates tokens and is dropped;
* letter and digit runs longer than 8 bytes are cut into pieces of at most 8;
* the id of a piece is ``4 + FNV-1a-32(piece) mod (vocab - 4)`` (ids 0..3 are
  reserved and never produced).

Every token carries its byte range ``[begin, end)`` inside its record, which
is what span decoding needs to map labels back to bytes.
"""
from __future__ import annotations

import re

import numpy as np

_PIECE = re.compile(rb"[A-Za-z]+|[0-9]+|[^\sA-Za-z0-9]")
MAX_PIECE = 8
N_RESERVED = 4


def fnv1a32(data: bytes) -> int:
    """FNV-1a, 32-bit (offset basis 2166136261, prime 16777619)."""
    h = 2166136261
    for b in data:
        h ^= b
        h = (h * 16777619) & 0xFFFFFFFF
    return h


def token_spans(text: bytes) -> tuple[np.ndarray, np.ndarray]:
    """Byte ranges of the tokens of ``text`` (begin and end arrays, int64)."""
    begins: list[int] = []
    ends: list[int] = []
    for m in _PIECE.finditer(text):
        b, e = m.span()
        while e - b > MAX_PIECE:
            begins.append(b)
            ends.append(b + MAX_PIECE)
            b += MAX_PIECE
        begins.append(b)
        ends.append(e)
    return np.asarray(begins, dtype=np.int64), np.asarray(ends, dtype=np.int64)


def piece_ids(text: bytes, begins: np.ndarray, ends: np.ndarray, vocab: int) -> np.ndarray:
    """Vectorised FNV-1a-32 of each piece, mapped into ``[4, vocab)``."""
    n = begins.shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.int32)
    buf = np.frombuffer(text, dtype=np.uint8)
    lens = (ends - begins).astype(np.int64)
    h = np.full(n, 2166136261, dtype=np.uint64)
    for k in range(MAX_PIECE):
        live = lens > k
        idx = np.where(live, begins + k, 0)
        byte = buf[idx].astype(np.uint64)
        nh = ((h ^ byte) * np.uint64(16777619)) & np.uint64(0xFFFFFFFF)
        h = np.where(live, nh, h)
    return (N_RESERVED + (h % np.uint64(vocab - N_RESERVED))).astype(np.int32)


def tokenize(text: bytes, vocab: int) -> tuple[np.ndarray, np.ndarray]:
    """Token ids (int32 [n]) and byte offsets (int32 [n, 2]) of one record."""
    b, e = token_spans(text)
    ids = piece_ids(text, b, e, vocab)
    off = np.stack([b, e], axis=1).astype(np.int32) if b.size else np.zeros((0, 2), np.int32)
    return ids, off
