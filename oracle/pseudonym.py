"""Deterministic pseudonyms and their substitution (test infrastructure only).

Sec. II, stage 3: each detected entity is replaced by an HMAC-SHA256 slug
computed under an operator-defined secret key; the slug keeps 0 to 64 hex
characters and the entity type stays as a prefix, giving ``[TYPE_slug]``
(the paper's example maps an IPv4 address to ``[IP_ADDRESS_`` followed by ten
lowercase hex digits and ``]``).  Referential integrity (Sec. II, Fig. 1
caption): the same entity under the same key always gets the same pseudonym.

Readings: the HMAC message is the entity's bytes exactly as they appear in the
record; the slug is the first n characters of the lowercase hex digest; with
n = 0 the pseudonym is ``[TYPE]``.  HMAC (RFC 2104) over SHA-256 (FIPS 180-4)
is taken from Python's standard library.
"""
from __future__ import annotations

import hashlib
import hmac

import numpy as np


def hmac_hex(key: bytes, msg: bytes) -> str:
    return hmac.new(key, msg, hashlib.sha256).hexdigest()


def pseudonym(type_name: str, key: bytes, entity: bytes, slug_len: int) -> bytes:
    if not 0 <= slug_len <= 64:
        raise ValueError("slug length must be in [0, 64]")
    if slug_len == 0:
        return f"[{type_name}]".encode()
    return f"[{type_name}_{hmac_hex(key, entity)[:slug_len]}]".encode()


def substitute(text: bytes, spans, type_names, key: bytes, slug_len: int) -> bytes:
    """Replace each span (type, begin, end) of one record, left to right."""
    out = []
    pos = 0
    for (t, b, e) in spans:
        if b < pos or e < b or e > len(text):
            raise ValueError("spans must be sorted, disjoint and inside the record")
        out.append(text[pos:b])
        out.append(pseudonym(type_names[t - 1], key, text[b:e], slug_len))
        pos = e
    out.append(text[pos:])
    return b"".join(out)


def pseudonymize_batch(text: bytes, cu_bytes, spans: np.ndarray, n_records: int, type_names,
                       key: bytes, slug_len: int) -> list[bytes]:
    """Output bytes of every record; ``spans`` rows are (record, type, begin, end)."""
    cu = np.asarray(cu_bytes, dtype=np.int64)
    per = [[] for _ in range(n_records)]
    for r, t, b, e in np.asarray(spans, dtype=np.int64).reshape(-1, 4).tolist():
        per[r].append((t, b, e))
    return [substitute(text[int(cu[r]):int(cu[r + 1])], per[r], type_names, key, slug_len)
            for r in range(n_records)]
