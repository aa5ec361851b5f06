"""Schema-aware whole-field pseudonymization without NER (test infrastructure only).

The paper's schema-aware configuration maps named fields straight to
pseudonyms, bypassing inference; it is the paper's largest speedup (Sec. II;
Sec. IV-A and App. C, Table VI, D2 with and without the configuration).  Reading taken
here (the GPU path takes the same), for ``Field: value`` records:

* a line is a maximal run of bytes without ``\\n``;
* a line holds a field if its first ``:`` is directly followed by a space;
  the field name is the bytes before that ``:``, the value the bytes after
  ``": "`` up to the end of the line;
* a field whose name (exact bytes) is configured with an entity type, and
  whose value is not empty, gives one span of that type covering the value.

The spans then go through the same substitution as NER spans.
"""
from __future__ import annotations


def field_spans_record(t: bytes, config: dict[bytes, int]) -> list[tuple[int, int, int]]:
    """Spans (type, begin, end) of the configured fields of one record."""
    out = []
    i = 0
    n = len(t)
    while i < n:
        j = t.find(b"\n", i)
        e = n if j < 0 else j
        line = t[i:e]
        c = line.find(b":")
        if c >= 0 and c + 1 < len(line) and line[c + 1] == ord(" "):
            typ = config.get(line[:c], 0)
            if typ and c + 2 < len(line):
                out.append((typ, i + c + 2, e))
        i = e + 1
    return out


def field_spans_batch(text: bytes, cu_bytes, config: dict[bytes, int]) -> list[list[tuple[int, int, int]]]:
    return [field_spans_record(text[int(cu_bytes[b]):int(cu_bytes[b + 1])], config)
            for b in range(len(cu_bytes) - 1)]
