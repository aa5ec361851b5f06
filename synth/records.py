"""Seeded synthetic vulnerability-scan records with gold entity spans.

The paper's datasets (Sec. III, Table II) are either private (D2) or not in
this repository, so every input is generated here from a seeded template
grammar of scan-report fields: ``Field: value`` lines carrying IPv4 addresses,
hostnames, CVE ids, e-mail addresses, ports, URLs, MAC addresses and hex
digests, mixed with free "plugin text" drawn from a word list invented for
this project.  Entity types follow the paper's naming style (Sec. II, stage 3
shows ``IP_ADDRESS``).

A record is cut to an exact token count; gold BIO labels come from the
templates (label 0 = O, type t >= 1 has B = 2t-1 and I = 2t).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tokenizer import piece_ids, token_spans

TYPE_NAMES_17 = ["IP_ADDRESS", "HOSTNAME", "CVE_ID", "EMAIL_ADDRESS",
                 "PORT", "URL", "MAC_ADDRESS", "HASH"]
TYPE_NAMES_9 = TYPE_NAMES_17[:4]

# Invented vocabulary for free text (not taken from any scanner's output).
_WORDS = (
    "remote service version detected module banner listener endpoint daemon "
    "agent runtime package library handler request response session token "
    "cipher protocol handshake certificate option default configured enabled "
    "disabled outdated patched vulnerable exposure weakness upgrade vendor "
    "release branch build kernel firmware driver interface socket channel "
    "queue worker thread process memory buffer overflow injection traversal "
    "escalation bypass validation sanitized header cookie parameter payload "
    "archive backup mirror cluster replica primary secondary gateway proxy "
    "tunnel bridge segment subnet route policy audit scanner finding severity "
    "medium high low critical informational apply latest stable maintenance "
    "window schedule operator reviewed confirmed observed reported allows "
    "attacker local unauthenticated crafted message trigger condition may "
    "could should the a of on in to and with from for by via is was be"
).split()
_FIELDS_TEXT = ["Description", "Synopsis", "Solution", "Plugin Output", "Risk Factor",
                "Notes", "Summary", "Impact"]
_TLDS = ["corp", "lan", "intra", "net", "org", "local", "example", "internal"]
# line mix, tuned so that about 8% of tokens fall inside entities
P_FIELD_LINE = 0.09
P_INLINE = 0.08
_URL_PATHS = ["advisory", "docs", "kb", "patch", "release", "notes", "bulletin", "info"]


def _label(rng: np.random.Generator, lo: int = 3, hi: int = 8) -> str:
    n = int(rng.integers(lo, hi + 1))
    alphabet = "abcdefghijklmnopqrstuvwxyz0123456789"
    chars = [alphabet[int(i)] for i in rng.integers(0, 26, 1)]
    chars += [alphabet[int(i)] for i in rng.integers(0, 36, n - 1)]
    if n >= 5 and rng.random() < 0.3:
        chars[n // 2] = "-"
    return "".join(chars)


def _hostname(rng):
    k = int(rng.integers(2, 5))
    return ".".join([_label(rng) for _ in range(k - 1)] + [_TLDS[int(rng.integers(len(_TLDS)))]])


def _entity_text(t: str, rng: np.random.Generator) -> str:
    if t == "IP_ADDRESS":
        return ".".join(str(int(x)) for x in rng.integers(0, 256, 4))
    if t == "HOSTNAME":
        return _hostname(rng)
    if t == "CVE_ID":
        year = int(rng.integers(1999, 2026))
        num = int(rng.integers(1000, 100000)) if rng.random() < 0.6 else int(rng.integers(1000, 10000))
        return f"CVE-{year}-{num}"
    if t == "EMAIL_ADDRESS":
        local = _label(rng, 3, 10).replace("-", ".")
        return f"{local}@{_hostname(rng)}"
    if t == "PORT":
        return str(int(rng.integers(1, 65536)))
    if t == "URL":
        segs = "/".join(_URL_PATHS[int(i)] for i in rng.integers(0, len(_URL_PATHS), int(rng.integers(1, 4))))
        return f"https://{_hostname(rng)}/{segs}"
    if t == "MAC_ADDRESS":
        return ":".join(f"{int(x):02x}" for x in rng.integers(0, 256, 6))
    if t == "HASH":
        n = [32, 40, 64][int(rng.integers(3))]
        return "".join("0123456789abcdef"[int(x)] for x in rng.integers(0, 16, n))
    raise ValueError(t)


_FIELD_OF = {
    "IP_ADDRESS": ["Host", "IP", "Target"], "HOSTNAME": ["Hostname", "FQDN", "DNS Name"],
    "CVE_ID": ["CVE", "Reference"], "EMAIL_ADDRESS": ["Contact", "Owner"],
    "PORT": ["Port"], "URL": ["See Also"], "MAC_ADDRESS": ["MAC"], "HASH": ["Fingerprint", "Hash"],
}


class EntityPool:
    """A fixed pool of distinct entities drawn with Zipf(s) popularity."""

    def __init__(self, types: list[str], size: int, s: float, seed: int):
        rng = np.random.default_rng(seed + 7777)
        seen: set[str] = set()
        items: list[tuple[str, str]] = []
        while len(items) < size:
            t = types[int(rng.integers(len(types)))]
            e = _entity_text(t, rng)
            if e not in seen:
                seen.add(e)
                items.append((t, e))
        self.items = items
        w = 1.0 / np.arange(1, size + 1, dtype=np.float64) ** s
        self.cdf = np.cumsum(w) / w.sum()

    def draw(self, rng: np.random.Generator) -> tuple[str, str]:
        k = int(np.searchsorted(self.cdf, rng.random(), side="right"))
        return self.items[min(k, len(self.items) - 1)]


def _words(rng, lo, hi):
    return " ".join(_WORDS[int(i)] for i in rng.integers(0, len(_WORDS), int(rng.integers(lo, hi + 1))))


def _line(rng, types, pool):
    """One ``Field: value`` line as a list of (text, entity-type-or-None)."""
    r = rng.random()
    if r < P_FIELD_LINE:
        t, e = pool.draw(rng) if pool is not None else (None, None)
        if t is None:
            t = types[int(rng.integers(len(types)))]
            e = _entity_text(t, rng)
        name = _FIELD_OF[t][int(rng.integers(len(_FIELD_OF[t])))]
        parts = [(f"{name}: ", None), (e, t)]
        if t == "PORT":
            parts.append(("/tcp" if rng.random() < 0.8 else "/udp", None))
        return parts
    if r < P_FIELD_LINE + 0.08 and "PORT" not in types:
        # ports are plain text under the 4-type label set
        return [("Port: ", None), (f"{int(rng.integers(1, 65536))}/tcp", None)]
    name = _FIELDS_TEXT[int(rng.integers(len(_FIELDS_TEXT)))]
    parts = [(f"{name}: ", None), (_words(rng, 8, 22), None)]
    if rng.random() < P_INLINE:
        t, e = pool.draw(rng) if pool is not None else (None, None)
        if t is None:
            t = types[int(rng.integers(len(types)))]
            e = _entity_text(t, rng)
        parts += [(" on ", None), (e, t), (" ", None), (_words(rng, 2, 8), None)]
    parts.append((".", None))
    return parts


@dataclass
class RecordBatch:
    """A packed batch of records (no padding).

    ``text`` holds all record bytes back to back, record b occupying
    ``text[cu_bytes[b]:cu_bytes[b+1]]``.  ``ids``/``tok_off``/``gold_labels``
    are packed over tokens with ``cu_seqlens``; ``tok_off`` is relative to the
    token's own record.  ``gold_spans`` rows are (record, type, begin, end).
    """
    text: bytes
    cu_bytes: np.ndarray
    ids: np.ndarray
    tok_off: np.ndarray
    cu_seqlens: np.ndarray
    gold_labels: np.ndarray
    gold_spans: np.ndarray
    type_names: list[str]
    n_pool_draws: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_records(self) -> int:
        return int(self.cu_seqlens.shape[0] - 1)

    @property
    def n_tokens(self) -> int:
        return int(self.cu_seqlens[-1])

    def record_text(self, b: int) -> bytes:
        return self.text[int(self.cu_bytes[b]):int(self.cu_bytes[b + 1])]

    def subset(self, recs) -> "RecordBatch":
        """A new packed batch holding the given records, in the given order."""
        texts, ids, offs, labs, spans = [], [], [], [], []
        cu_b, cu_t = [0], [0]
        for nb, b in enumerate(recs):
            b = int(b)
            t0, t1 = int(self.cu_seqlens[b]), int(self.cu_seqlens[b + 1])
            texts.append(self.record_text(b))
            ids.append(self.ids[t0:t1]); offs.append(self.tok_off[t0:t1]); labs.append(self.gold_labels[t0:t1])
            sel = self.gold_spans[self.gold_spans[:, 0] == b].copy()
            sel[:, 0] = nb
            spans.append(sel)
            cu_b.append(cu_b[-1] + len(texts[-1])); cu_t.append(cu_t[-1] + (t1 - t0))
        return RecordBatch(
            text=b"".join(texts), cu_bytes=np.asarray(cu_b, np.int64),
            ids=np.concatenate(ids) if ids else np.zeros(0, np.int32),
            tok_off=np.concatenate(offs) if offs else np.zeros((0, 2), np.int32),
            cu_seqlens=np.asarray(cu_t, np.int32),
            gold_labels=np.concatenate(labs) if labs else np.zeros(0, np.uint8),
            gold_spans=np.concatenate(spans) if spans else np.zeros((0, 4), np.int64),
            type_names=self.type_names)


def draw_lengths(spec: tuple, n: int, rng: np.random.Generator) -> np.ndarray:
    """Token counts per record from ("uniform", lo, hi) or ("lognormal", mu, sigma, lo, hi)."""
    if spec[0] == "uniform":
        return rng.integers(spec[1], spec[2] + 1, n).astype(np.int64)
    if spec[0] == "lognormal":
        mu, sigma, lo, hi = spec[1:]
        return np.clip(np.round(np.exp(rng.normal(mu, sigma, n))), lo, hi).astype(np.int64)
    raise ValueError(spec)


def _one_record(rng, n_tok, types, pool, vocab):
    pieces: list[str] = []
    ents: list[tuple[int, int, int]] = []  # (begin, end, type index 1-based)
    pos = 0
    ntok = 0
    while ntok < n_tok:
        line = _line(rng, types, pool)
        line_txt = "".join(p for p, _ in line)
        lb = line_txt.encode()
        ntok += len(token_spans(lb)[0])
        for p, t in line:
            bb = len(p.encode())
            if t is not None:
                ents.append((pos, pos + bb, types.index(t) + 1))
            pos += bb
        pieces.append(line_txt)
        pieces.append("\n")
        pos += 1
    text = "".join(pieces).encode()
    b, e = token_spans(text)
    b, e = b[:n_tok], e[:n_tok]
    cut = int(e[-1]) if n_tok > 0 else 0
    text = text[:cut]
    ids = piece_ids(text, b, e, vocab)
    labels = np.zeros(n_tok, dtype=np.uint8)
    spans = []
    for (eb, ee, ti) in ents:
        if eb >= cut:
            continue
        inside = np.nonzero((b >= eb) & (e <= ee))[0]
        if inside.size == 0:
            continue
        labels[inside[0]] = 2 * ti - 1
        labels[inside[1:]] = 2 * ti
        spans.append((ti, int(b[inside[0]]), int(e[inside[-1]])))
    off = np.stack([b, e], axis=1).astype(np.int32)
    return text, ids, off, labels, spans


def _tokenize_line(parts, types, vocab):
    """Bytes, ids, offsets, labels and entity (type, begin, end) of one pool line."""
    text = "".join(p for p, _ in parts).encode()
    b, e = token_spans(text)
    ids = piece_ids(text, b, e, vocab)
    lab = np.zeros(len(b), np.uint8)
    ent = None
    pos = 0
    for p, t in parts:
        n = len(p.encode())
        if t is not None:
            inside = np.nonzero((b >= pos) & (e <= pos + n))[0]
            ti = types.index(t) + 1
            lab[inside[0]] = 2 * ti - 1
            lab[inside[1:]] = 2 * ti
            ent = (ti, pos, pos + n)
        pos += n
    return text, ids, np.stack([b, e], 1).astype(np.int32), lab, ent


def generate_records_fast(n_records: int, lengths, n_types: int, vocab: int, seed: int,
                          zipf_pool: int = 200_000, zipf_s: float = 1.1, text_pool: int = 20_000,
                          p_entity: float = 0.15) -> RecordBatch:
    """Dataset-scale records from pre-tokenized line pools (vectorized assembly).

    Lines are either free-text lines (a pool of ``text_pool`` distinct lines)
    or ``Field: entity`` lines whose entity is drawn with Zipf(s) popularity
    from ``zipf_pool`` distinct entities.  A record takes lines in order until
    it holds its target token count; the last line is cut at that token.
    """
    rng = np.random.default_rng(seed)
    lens = draw_lengths(lengths, n_records, rng) if isinstance(lengths, tuple) else np.asarray(lengths, np.int64)
    types = TYPE_NAMES_17[:n_types]
    lines = []
    for _ in range(text_pool):
        name = _FIELDS_TEXT[int(rng.integers(len(_FIELDS_TEXT)))]
        lines.append([(f"{name}: ", None), (_words(rng, 8, 22), None), (".", None)])
    pool = EntityPool(types, zipf_pool, zipf_s, seed)
    for t, e in pool.items:
        parts = [(f"{_FIELD_OF[t][0]}: ", None), (e, t)]
        if t == "PORT":
            parts.append(("/tcp", None))
        lines.append(parts)
    tok = [_tokenize_line(p, types, vocab) for p in lines]
    L_bytes = [t[0] for t in tok]
    L_nb = np.array([len(b) for b in L_bytes], np.int64)
    L_nt = np.array([len(t[1]) for t in tok], np.int64)
    L_t0 = np.concatenate([[0], np.cumsum(L_nt)])
    F_ids = np.concatenate([t[1] for t in tok])
    F_off = np.concatenate([t[2] for t in tok])
    F_lab = np.concatenate([t[3] for t in tok])
    L_ent = np.array([t[4] if t[4] is not None else (0, 0, 0) for t in tok], np.int64)

    # line stream: entity lines with probability p_entity (Zipf rank), else text lines
    need = int(lens.sum() / max(1.0, L_nt.mean()) * 1.3) + 1024
    kinds = rng.random(need) < p_entity
    ranks = np.minimum(np.searchsorted(pool.cdf, rng.random(need), side="right"), zipf_pool - 1)
    stream = np.where(kinds, text_pool + ranks, rng.integers(0, text_pool, need))
    cum = np.concatenate([[0], np.cumsum(L_nt[stream])])
    starts = np.empty(n_records, np.int64)
    ends = np.empty(n_records, np.int64)
    s = 0
    for r in range(n_records):
        e = int(np.searchsorted(cum, cum[s] + lens[r], side="left"))  # lines s..e-1 reach the target
        if e >= len(cum):
            raise RuntimeError("line stream too short")
        starts[r], ends[r] = s, e
        s = e
    # line instances of every record
    n_lines = ends - starts
    inst = np.concatenate([stream[a:b] for a, b in zip(starts, ends)]) if n_records else np.zeros(0, np.int64)
    inst_rec = np.repeat(np.arange(n_records), n_lines)
    first = np.concatenate([[0], np.cumsum(n_lines)])[:-1]
    # byte offset of each line inside its record (lines joined by "\n")
    inst_nb = L_nb[inst] + 1
    csum = np.cumsum(inst_nb) - inst_nb
    inst_boff = csum - np.repeat(csum[first], n_lines)
    # tokens: ragged gather of each line's tokens, then cut each record at its length
    inst_nt = L_nt[inst]
    tbase = np.cumsum(inst_nt) - inst_nt
    total = int(inst_nt.sum())
    src = np.repeat(L_t0[inst] - tbase, inst_nt) + np.arange(total)
    t_rec = np.repeat(inst_rec, inst_nt)
    t_shift = np.repeat(inst_boff, inst_nt)
    rec_t0 = np.concatenate([[0], np.cumsum(np.bincount(inst_rec, weights=inst_nt, minlength=n_records))])[:-1]
    t_idx = np.arange(total) - np.repeat(rec_t0.astype(np.int64), np.bincount(t_rec, minlength=n_records))
    keep = t_idx < lens[t_rec]
    ids = F_ids[src[keep]].astype(np.int32)
    off = (F_off[src[keep]] + t_shift[keep, None]).astype(np.int32)
    lab = F_lab[src[keep]].astype(np.uint8)
    cu_t = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cut = off[cu_t[1:] - 1, 1].astype(np.int64)  # end byte of each record's last token
    texts = []
    for r in range(n_records):
        texts.append(b"\n".join(L_bytes[i] for i in stream[starts[r]:ends[r]])[: cut[r]])
    cu_b = np.concatenate([[0], np.cumsum([len(t) for t in texts])]).astype(np.int64)
    # gold spans of entity lines that survive the cut
    ent = L_ent[inst]
    has = ent[:, 0] > 0
    sb = inst_boff + ent[:, 1]
    se = np.minimum(inst_boff + ent[:, 2], cut[inst_rec])
    ok = has & (sb < cut[inst_rec])
    spans = np.stack([inst_rec[ok], ent[ok, 0], sb[ok], se[ok]], 1).astype(np.int64)
    return RecordBatch(text=b"".join(texts), cu_bytes=cu_b, ids=ids, tok_off=off, cu_seqlens=cu_t,
                       gold_labels=lab, gold_spans=spans.reshape(-1, 4), type_names=list(types),
                       n_pool_draws=int(ok.sum()))


def generate_records(n_records: int, lengths, n_types: int, vocab: int, seed: int,
                     zipf_pool: int = 0, zipf_s: float = 1.1) -> RecordBatch:
    """Generate ``n_records`` records; ``lengths`` is a spec tuple or an int array."""
    rng = np.random.default_rng(seed)
    if isinstance(lengths, tuple):
        lens = draw_lengths(lengths, n_records, rng)
    else:
        lens = np.asarray(lengths, dtype=np.int64)
    types = TYPE_NAMES_17[:n_types]
    pool = EntityPool(types, zipf_pool, zipf_s, seed) if zipf_pool else None
    texts, ids, offs, labs, spans = [], [], [], [], []
    cu_b, cu_t = [0], [0]
    for r in range(n_records):
        text, i, o, l, sp = _one_record(rng, int(lens[r]), types, pool, vocab)
        texts.append(text); ids.append(i); offs.append(o); labs.append(l)
        spans.extend((r, t, bb, ee) for (t, bb, ee) in sp)
        cu_b.append(cu_b[-1] + len(text)); cu_t.append(cu_t[-1] + len(i))
    return RecordBatch(
        text=b"".join(texts), cu_bytes=np.asarray(cu_b, dtype=np.int64),
        ids=np.concatenate(ids) if ids else np.zeros(0, np.int32),
        tok_off=np.concatenate(offs) if offs else np.zeros((0, 2), np.int32),
        cu_seqlens=np.asarray(cu_t, dtype=np.int32),
        gold_labels=np.concatenate(labs) if labs else np.zeros(0, np.uint8),
        gold_spans=np.asarray(spans, dtype=np.int64).reshape(-1, 4),
        type_names=list(types))
