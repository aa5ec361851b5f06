"""Pins of the whole-field oracle: hand-made lines, equality with a regular
expression over random texts, and agreement with the generator's gold fields."""
import random
import re

import numpy as np

import synth
from oracle import fields as F
from synth.records import TYPE_NAMES_17, _FIELD_OF

CONFIG = {name.encode(): TYPE_NAMES_17.index(t) + 1 for t, names in _FIELD_OF.items() for name in names}


def test_written_lines():
    cfg = {b"Host": 1, b"See Also": 6, b"a": 2}
    t = b"Host: 10.0.0.1\nHost:10.0.0.2\nHost: \nSee Also: https://x.corp:8080/a\na:b: c\nHost: 1.2.3.4\r\nHost: z"
    got = F.field_spans_record(t, cfg)
    want = [(1, 6, 14), (6, 46, 67), (1, 81, 89), (1, 96, 97)]
    assert got == want, got
    assert [t[b:e] for _, b, e in got] == [b"10.0.0.1", b"https://x.corp:8080/a", b"1.2.3.4\r", b"z"]
    assert F.field_spans_record(b"", cfg) == []
    assert F.field_spans_record(b"\n\n", cfg) == []


def test_equals_regular_expression_on_random_texts():
    pat = re.compile(rb"^([^:\n]*): ([^\n]+)", re.M)
    pieces = [b"Host", b"IP", b": ", b":", b" ", b"\n", b"x", b"See Also", b"a:b", b"1.2", b"\n\n", b"Port"]
    cfg = {b"Host": 1, b"IP": 1, b"See Also": 6, b"Port": 5, b"": 3}
    rng = random.Random(7)
    hits = 0
    for _ in range(3000):
        t = b"".join(rng.choice(pieces) for _ in range(rng.randint(0, 20)))
        want = [(cfg[m.group(1)], m.start(2), m.end(2)) for m in pat.finditer(t) if m.group(1) in cfg]
        assert F.field_spans_record(t, cfg) == want, t
        hits += len(want)
    assert hits > 400


def test_generator_fields_are_gold_entities():
    """Every field span is a gold entity of its type (a port field also holds
    the protocol after the number: "443/tcp"), and every gold entity that
    stands alone as a configured field's value is found."""
    rb = synth.generate_records(64, np.full(64, 300), len(TYPE_NAMES_17), 30522, 12)
    port = TYPE_NAMES_17.index("PORT") + 1
    n_fields = 0
    for b in range(rb.n_records):
        t = rb.text[int(rb.cu_bytes[b]):int(rb.cu_bytes[b + 1])]
        spans = F.field_spans_record(t, CONFIG)
        gold = {(int(g[1]), int(g[2]), int(g[3])) for g in rb.gold_spans[rb.gold_spans[:, 0] == b]}
        # a record is cut to an exact token count: its last line may be cut short
        spans = [s for s in spans if s[2] < len(t)]
        for typ, sb, se in spans:
            if typ == port:
                assert any(g[0] == typ and g[1] == sb and g[2] < se for g in gold)
                assert t[sb:se].split(b"/")[1] in (b"tcp", b"udp")
            else:
                assert (typ, sb, se) in gold
        for typ, gb, ge in gold:
            ls = t.rfind(b"\n", 0, gb) + 1
            le = t.find(b"\n", ge)
            line = t[ls:len(t) if le < 0 else le]
            if le >= 0 and line[:gb - ls] in {k + b": " for k in CONFIG} and ge == ls + len(line):
                assert (typ, gb, ge) in spans
        n_fields += len(spans)
    assert n_fields > 50
