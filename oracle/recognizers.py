"""Pattern recognizers beside the NER model, and overlap resolution (test infrastructure only).

The paper's detector pairs the transformer with 21 regular-expression
recognizers for IPv4/IPv6, URLs, hostnames, hashes, CVE/CPE ids and more
(Sec. II, stage 2), but prints none of the patterns.  It also reports what a
missing overlap-resolution layer costs: independent detectors that find
overlapping spans truncate entities or emit extra pseudonyms, and a single
leaked occurrence is enough to re-identify (Sec. IV-B and App. D, accuracy
results and false negatives).

Readings taken here (the GPU path takes the same):

* Nine recognizers, each a rule over the bytes of one record, with W = the
  word bytes [A-Za-z0-9_], LABEL = [A-Za-z0-9-], LOCAL = [A-Za-z0-9._%+-]:

  URL       ``http://`` or ``https://`` at a word boundary, then the maximal
            run (>= 1) of non-whitespace bytes;
  EMAIL     a maximal LOCAL run, ``@``, one or more ``label.`` groups, then a
            top-level label of >= 2 letters not followed by a LABEL byte
            (the longest such domain);
  IPV4      four dot-separated decimal octets 0..255 without leading zeros,
            at word boundaries;
  MAC       six two-digit hex groups separated by ``:``, at word boundaries;
  HASH      a run of exactly 32, 40 or 64 hex digits at word boundaries;
  CVE       ``CVE-`` + 4 digits + ``-`` + 4..7 digits, at word boundaries;
  HOSTNAME  a dotted LABEL sequence not preceded by a LABEL byte or a dot,
            ending at a label equal to one of a fixed list of top-level
            labels and not followed by a LABEL byte (the longest such);
  IPV6      an IPv6 address in one of the text forms of RFC 4291 section 2.2:
            the maximal run of hex digits, ``:`` and ``.`` that starts at a
            hex digit or ``:`` not preceded by a word byte, ``:`` or ``.``,
            without its trailing dots, must be such an address and must not
            be followed by a word byte.  It emits the IP address type;
  CPE       a CPE name (the paper lists CPE strings among its entity kinds):
            ``cpe:/`` (URI binding) or ``cpe:2.3:`` (formatted string) at a
            word start, a part letter (``a``, ``h``, ``o``; in 2.3 also ``*``
            or ``-``) not followed by a component byte, then the maximal run
            of component bytes [A-Za-z0-9._~%*?!\\-] and ``:``.  It emits a
            ``CPE`` type, so it is off for label sets without one.

  Each rule but IPv6 is the match, at one start position, of a regular
  expression (``PATTERNS`` below; the tests compare rule and expression at
  every position of random texts); the IPv6 rule is pinned to Python's
  ``ipaddress`` parser instead.  Every position where a rule
  matches gives one candidate span.
* Overlap resolution: NER spans and recognizer candidates that share at
  least one byte are merged into their union (chains merge transitively;
  spans that only touch stay apart).  The merged span takes the type of its
  longest member; on equal lengths NER wins, then recognizers in the order
  above.  No byte of any detected entity is left outside a span.
"""
from __future__ import annotations

RECOGNIZERS = ["URL", "EMAIL_ADDRESS", "IP_ADDRESS", "MAC_ADDRESS", "HASH", "CVE_ID", "HOSTNAME", "IPV6", "CPE"]
# entity type each recognizer emits by default
RECOGNIZER_TYPE = {r: r for r in RECOGNIZERS} | {"IPV6": "IP_ADDRESS"}
TOP_LABELS = [b"corp", b"lan", b"intra", b"net", b"org", b"local", b"example", b"internal"]

_W = frozenset(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789_")
_LABEL = frozenset(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-")
_LOCAL = frozenset(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789._%+-")
_LETTER = frozenset(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz")
_DIGIT = frozenset(b"0123456789")
_HEX = frozenset(b"0123456789abcdefABCDEF")
_SPACE = frozenset(b" \t\n\r\f\v")

# The regular expressions the rules state (bytes patterns, ASCII classes).
PATTERNS = {
    "URL": rb"\bhttps?://\S+",
    "EMAIL_ADDRESS": rb"(?<![A-Za-z0-9._%+-])[A-Za-z0-9._%+-]+@(?:[A-Za-z0-9-]+\.)+[A-Za-z]{2,}(?![A-Za-z0-9-])",
    "IP_ADDRESS": rb"\b(?:(?:25[0-5]|2[0-4][0-9]|1[0-9][0-9]|[1-9]?[0-9])\.){3}"
                  rb"(?:25[0-5]|2[0-4][0-9]|1[0-9][0-9]|[1-9]?[0-9])\b",
    "MAC_ADDRESS": rb"\b[0-9A-Fa-f]{2}(?::[0-9A-Fa-f]{2}){5}\b",
    "HASH": rb"\b(?:[0-9A-Fa-f]{64}|[0-9A-Fa-f]{40}|[0-9A-Fa-f]{32})\b",
    "CVE_ID": rb"\bCVE-[0-9]{4}-[0-9]{4,7}\b",
    "HOSTNAME": rb"(?<![A-Za-z0-9.-])(?:[A-Za-z0-9-]+\.)+(?:" + b"|".join(TOP_LABELS) + rb")(?![A-Za-z0-9-])",
    "CPE": rb"\bcpe:(?:/[aho]|2\.3:[aho*-])(?![A-Za-z0-9._~%*?!\\-])[A-Za-z0-9._~%*?!\\:-]*",
}


def _run(t: bytes, i: int, cls) -> int:
    """End of the maximal run of bytes in ``cls`` starting at i."""
    n = len(t)
    while i < n and t[i] in cls:
        i += 1
    return i


def _word_start(t: bytes, p: int) -> bool:
    """A word byte at p with no word byte before it (a regex \\b before a word byte)."""
    return t[p] in _W and (p == 0 or t[p - 1] not in _W)


def _word_end(t: bytes, q: int) -> bool:
    """No word byte at q (a regex \\b after a word byte)."""
    return q == len(t) or t[q] not in _W


def _dotted_groups(t: bytes, i: int) -> tuple[list[tuple[int, int]], int]:
    """Labels followed by a dot from i on, and the position after the last dot."""
    groups = []
    while True:
        j = _run(t, i, _LABEL)
        if j > i and j < len(t) and t[j] == ord("."):
            groups.append((i, j))
            i = j + 1
        else:
            return groups, i


def match_url(t: bytes, p: int) -> int:
    if not _word_start(t, p):
        return -1
    for scheme in (b"https://", b"http://"):
        if t.startswith(scheme, p):
            q = p + len(scheme)
            e = q
            while e < len(t) and t[e] not in _SPACE:
                e += 1
            return e if e > q else -1
    return -1


def match_email(t: bytes, p: int) -> int:
    if t[p] not in _LOCAL or (p > 0 and t[p - 1] in _LOCAL):
        return -1
    q = _run(t, p, _LOCAL)
    if q == len(t) or t[q] != ord("@"):
        return -1
    groups, tail = _dotted_groups(t, q + 1)
    # the top-level label is tried after all groups, then after one fewer, ...
    for j in range(len(groups), 0, -1):
        s = tail if j == len(groups) else groups[j][0]
        e = _run(t, s, _LETTER)
        if e - s >= 2 and (e == len(t) or t[e] not in _LABEL):
            return e
    return -1


def _octet(t: bytes, i: int) -> int:
    """End of a valid octet (0..255, no leading zero) spanning the whole digit run at i, else -1."""
    e = _run(t, i, _DIGIT)
    c = e - i
    if c < 1 or c > 3 or (c > 1 and t[i] == ord("0")) or int(t[i:e]) > 255:
        return -1
    return e


def match_ipv4(t: bytes, p: int) -> int:
    if t[p] not in _DIGIT or not _word_start(t, p):
        return -1
    i = p
    for k in range(4):
        e = _octet(t, i)
        if e < 0:
            return -1
        if k < 3:
            if e == len(t) or t[e] != ord("."):
                return -1
            i = e + 1
        else:
            return e if _word_end(t, e) else -1
    return -1


def match_mac(t: bytes, p: int) -> int:
    if not _word_start(t, p) or p + 17 > len(t):
        return -1
    for k in range(17):
        c = t[p + k]
        if (k % 3 == 2 and c != ord(":")) or (k % 3 != 2 and c not in _HEX):
            return -1
    return p + 17 if _word_end(t, p + 17) else -1


def match_hash(t: bytes, p: int) -> int:
    if t[p] not in _HEX or not _word_start(t, p):
        return -1
    e = _run(t, p, _HEX)
    return e if e - p in (32, 40, 64) and _word_end(t, e) else -1


def match_cve(t: bytes, p: int) -> int:
    if not _word_start(t, p) or not t.startswith(b"CVE-", p) or p + 9 > len(t):
        return -1
    if any(t[p + 4 + k] not in _DIGIT for k in range(4)) or t[p + 8] != ord("-"):
        return -1
    e = _run(t, p + 9, _DIGIT)
    return e if 4 <= e - (p + 9) <= 7 and _word_end(t, e) else -1


def match_hostname(t: bytes, p: int) -> int:
    if t[p] not in _LABEL or (p > 0 and (t[p - 1] in _LABEL or t[p - 1] == ord("."))):
        return -1
    groups, tail = _dotted_groups(t, p)
    for j in range(len(groups), 0, -1):
        s = tail if j == len(groups) else groups[j][0]
        for top in TOP_LABELS:
            e = s + len(top)
            if t.startswith(top, s) and (e == len(t) or t[e] not in _LABEL):
                return e
    return -1


def _dotted_quad(g: bytes) -> bool:
    parts = g.split(b".")
    return len(parts) == 4 and all(
        1 <= len(x) <= 3 and all(c in _DIGIT for c in x) and (len(x) == 1 or x[0] != ord("0")) and int(x) <= 255
        for x in parts)


def ipv6_text_valid(s: bytes) -> bool:
    """Whether s is an IPv6 address in a text form of RFC 4291 section 2.2:
    eight groups of 1-4 hex digits separated by ':', where one '::' may stand
    for one or more zero groups and the last 32 bits may be written as a
    dotted quad (octets without leading zeros)."""
    halves = s.split(b"::")
    if len(halves) > 2:
        return False
    groups = []
    for h in halves:
        groups.append(h.split(b":") if h else [])
    flat = [g for gs in groups for g in gs]
    n = 0
    for i, g in enumerate(flat):
        if b"." in g:
            # only the last group, and only where the text ends with it
            if i != len(flat) - 1 or not s.endswith(g) or not _dotted_quad(g):
                return False
            n += 2
        elif 1 <= len(g) <= 4 and all(c in _HEX for c in g):
            n += 1
        else:
            return False
    return n <= 7 if len(halves) == 2 else n == 8


def match_ipv6(t: bytes, p: int) -> int:
    if t[p] not in _HEX and t[p] != ord(":"):
        return -1
    if p > 0 and (t[p - 1] in _W or t[p - 1] in b":."):
        return -1
    e = p
    while e < len(t) and (t[e] in _HEX or t[e] in b":."):
        e += 1
    while e > p and t[e - 1] == ord("."):
        e -= 1
    if not ipv6_text_valid(t[p:e]) or not _word_end(t, e):
        return -1
    return e


_CPE = frozenset(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789._~%*?!\\-")


def match_cpe(t: bytes, p: int) -> int:
    if not _word_start(t, p):
        return -1
    if t.startswith(b"cpe:/", p):
        q, parts = p + 5, b"aho"
    elif t.startswith(b"cpe:2.3:", p):
        q, parts = p + 8, b"aho*-"
    else:
        return -1
    if q == len(t) or t[q] not in parts:
        return -1
    q += 1
    if q < len(t) and t[q] in _CPE:
        return -1
    while q < len(t) and (t[q] in _CPE or t[q] == ord(":")):
        q += 1
    return q


MATCHERS = {
    "URL": match_url, "EMAIL_ADDRESS": match_email, "IP_ADDRESS": match_ipv4, "MAC_ADDRESS": match_mac,
    "HASH": match_hash, "CVE_ID": match_cve, "HOSTNAME": match_hostname, "IPV6": match_ipv6, "CPE": match_cpe,
}


def recognizer_types(type_names) -> list[int]:
    """Type index (1-based, as in the label scheme) of each recognizer, 0 if the model has no such type."""
    names = list(type_names)
    return [names.index(RECOGNIZER_TYPE[r]) + 1 if RECOGNIZER_TYPE[r] in names else 0 for r in RECOGNIZERS]


def candidates(t: bytes, rec_types) -> list[tuple[int, int, int, int]]:
    """Every recognizer match in one record: (begin, end, type, priority), priority = 1 + recognizer index."""
    out = []
    for r, name in enumerate(RECOGNIZERS):
        if rec_types[r] == 0:
            continue
        m = MATCHERS[name]
        for p in range(len(t)):
            e = m(t, p)
            if e >= 0:
                out.append((p, e, rec_types[r], 1 + r))
    return out


def merge(spans) -> list[tuple[int, int, int]]:
    """Union of spans (begin, end, type, priority) sharing a byte; returns (type, begin, end).

    The merged span takes the type of its longest member, then of the lowest
    priority value (NER spans carry priority 0)."""
    out = []
    cur = None  # [begin, end, best_len, best_prio, best_type]
    for b, e, typ, prio in sorted(spans):
        if cur is not None and b < cur[1]:
            cur[1] = max(cur[1], e)
        else:
            if cur is not None:
                out.append((cur[4], cur[0], cur[1]))
            cur = [b, e, -1, 0, 0]
        if (e - b, -prio) > (cur[2], -cur[3]):
            cur[2], cur[3], cur[4] = e - b, prio, typ
    if cur is not None:
        out.append((cur[4], cur[0], cur[1]))
    return out


def resolve_record(t: bytes, ner_spans, rec_types) -> list[tuple[int, int, int]]:
    """NER spans (type, begin, end) of one record merged with its recognizer candidates."""
    spans = [(b, e, typ, 0) for typ, b, e in ner_spans]
    spans += candidates(t, rec_types)
    return merge(spans)


def resolve_batch(text: bytes, cu_bytes, ner_spans_per_record, type_names) -> list[list[tuple[int, int, int]]]:
    """resolve_record over a packed batch (text bytes back to back, cu_bytes offsets)."""
    rt = recognizer_types(type_names)
    return [resolve_record(text[int(cu_bytes[i]):int(cu_bytes[i + 1])], ner_spans_per_record[i], rt)
            for i in range(len(cu_bytes) - 1)]
