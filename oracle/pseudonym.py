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


# Per-type preservation and the entity <-> pseudonym mapping.
#
# The paper decouples detection from the replacement policy: chosen entity
# types can be preserved (Sec. II), and the mapping of entities to
# pseudonyms is persisted with the entity type, the original, the slug, the
# full hash and when the entity was first and last seen (Sec. II, stage 4).
# Readings: a preserved type's spans are left as they are; the mapping holds
# one row per distinct entity of at most 96 bytes (the device table's entry
# size) pseudonymized with the table enabled, with the smallest type index it
# was pseudonymized under (an entity's bytes, not its type, determine the
# hash), and "seen" counted in pseudonymize calls numbered from 1; rows are
# ordered by first call, then by bytes.

def preserve_spans(spans, preserve) -> list:
    """The spans (type, begin, end) whose type is not preserved."""
    keep = set(preserve)
    return [s for s in spans if s[0] not in keep]


MAX_TABLE_ENTITY = 96


def mapping_rows(calls, type_names, key: bytes, slug_len: int, preserve=()) -> list[dict]:
    """Mapping after a sequence of calls; each call is (text, cu_bytes, spans rows
    (record, type, begin, end)), every span valid."""
    rows: dict[bytes, dict] = {}
    keep_out = set(preserve)
    for c, (text, cu_bytes, spans) in enumerate(calls, start=1):
        for r, t, b, e in np.asarray(spans, dtype=np.int64).reshape(-1, 4).tolist():
            if t in keep_out:
                continue
            ent = text[int(cu_bytes[r]) + b:int(cu_bytes[r]) + e]
            if len(ent) > MAX_TABLE_ENTITY:
                continue
            row = rows.get(ent)
            if row is None:
                full = hmac_hex(key, ent)
                rows[ent] = {"entity_type": type_names[t - 1], "type": t, "original": ent,
                             "slug": full[:slug_len], "full_hash": full, "first_seen": c, "last_seen": c}
            else:
                if t < row["type"]:
                    row["type"], row["entity_type"] = t, type_names[t - 1]
                row["last_seen"] = c
    out = sorted(rows.values(), key=lambda d: (d["first_seen"], d["original"]))
    for d in out:
        del d["type"]
    return out
