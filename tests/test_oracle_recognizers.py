"""Pins of the recognizer oracle: each rule against Python's regular-expression
engine at every position of seeded random texts, hand-made overlap-resolution
cases, and coverage of the generator's gold entities."""
import ipaddress
import random
import re

import numpy as np
import pytest

import synth
from oracle import recognizers as R

# Pieces that assemble into matches, near-misses and boundary cases.
PIECES = {
    "URL": [b"http://", b"https://", b"htp://", b"http:/", b" ", b"x", b".", b"\n", b"_", b"a/b", b"\t"],
    "EMAIL_ADDRESS": [b"ab", b"x1", b".", b"@", b"-", b"_", b"%", b"+", b" ", b"com", b"corp", b"c", b"a.b@",
                      b"@h.co", b"..", b"9"],
    "IP_ADDRESS": [b"1", b"25", b"255", b"256", b"0", b"01", b"199", b"2", b".", b".", b".", b" ", b"a", b"_",
                   b"1.2.3.4", b"10.0.0."],
    "MAC_ADDRESS": [b"0a", b"ff", b"1F", b":", b":", b"g", b" ", b"_", b"0a:1b:2c:3d:4e:5f", b"aa:bb:cc:dd:ee",
                    b":00"],
    "HASH": [b"0123456789abcdef", b"0123456789ABCDEF", b"abcd", b"01234567", b" ", b"g", b"_", b"."],
    "CVE_ID": [b"CVE-", b"2021", b"-", b"12345", b"1", b"a", b" ", b"CVE-2021-1234567", b"_", b"cve-"],
    "HOSTNAME": [b"a", b"b1", b"-", b".", b"corp", b"lan", b"local", b"net", b"org1", b" ", b"@", b"x.internal",
                 b"/", b"Corp"],
    "IPV6": [b"fe80", b"::", b":", b":", b"1", b"0db8", b"FFFF", b"0", b"12345", b"1.2.3.4", b"01.2.3.4", b".",
             b" ", b"g", b"_", b"2001:db8::1", b"0:0:0:0:0:0:0:1", b"a:b:c:d:e:f:1:2", b"::ffff:10.0.0.1", b"\n"],
    "CPE": [b"cpe:/", b"cpe:2.3:", b"cpe:/a:apache:http_server:2.4.41", b"a", b"h", b"o", b"x", b"*", b"-", b":",
            b"::", b"apache", b"2.4.41", b"\\:", b" ", b"_", b"cpe", b"CPE:/", b".", b"\n", b"~", b"/", b"?"],
}


@pytest.mark.parametrize("name", [n for n in R.RECOGNIZERS if n in R.PATTERNS])
def test_rule_equals_regular_expression_at_every_position(name):
    pat = re.compile(R.PATTERNS[name])
    rule = R.MATCHERS[name]
    rng = random.Random(R.RECOGNIZERS.index(name))
    hits = 0
    for _ in range(1500):
        t = b"".join(rng.choice(PIECES[name]) for _ in range(rng.randint(1, 16)))
        for p in range(len(t)):
            m = pat.match(t, p)
            want = m.end() if m else -1
            assert rule(t, p) == want, (name, t, p)
            hits += want >= 0
    assert hits > 100, hits  # the texts do exercise matches


def _ipaddress_accepts(s: bytes) -> bool:
    try:
        ipaddress.IPv6Address(s.decode("ascii"))
        return True
    except ValueError:
        return False


def test_ipv6_validator_equals_ipaddress():
    """The oracle's own reading of the RFC 4291 text forms accepts exactly
    what Python's ipaddress parser accepts: every string of up to 6 bytes
    over a small alphabet, and random assemblies of groups, colons and
    dotted quads."""
    alphabet = [b"0", b"f", b"1", b":", b"."]
    n_valid = 0
    strings = [b""]
    for _ in range(6):
        strings = [x + a for x in strings for a in alphabet]
        for x in strings:
            v = R.ipv6_text_valid(x)
            assert v == _ipaddress_accepts(x), x
            n_valid += v
    pieces = [b"0", b"1", b"ab", b"ffff", b"0db8", b"12345", b":", b":", b"::", b"1.2.3.4", b"255.0.0.1",
              b"256.1.1.1", b"01.2.3.4", b".", b"1.2.3"]
    rng = random.Random(17)
    for _ in range(40000):
        x = b"".join(rng.choice(pieces) for _ in range(rng.randint(1, 18)))
        v = R.ipv6_text_valid(x)
        assert v == _ipaddress_accepts(x), x
        n_valid += v
    assert n_valid > 1000, n_valid


_RUN = re.compile(rb"(?<![A-Za-z0-9_:.])[0-9A-Fa-f:][0-9A-Fa-f:.]*")


def test_ipv6_rule_equals_run_and_ipaddress_at_every_position():
    """The rule against a second formulation: a regular expression finds the
    run, the trailing dots are stripped, ipaddress judges the rest, and no
    word byte may follow."""
    rng = random.Random(23)
    hits = 0
    for _ in range(3000):
        t = b"".join(rng.choice(PIECES["IPV6"]) for _ in range(rng.randint(1, 14)))
        for p in range(len(t)):
            m = _RUN.match(t, p)
            want = -1
            if m:
                sub = m.group().rstrip(b".")
                e = p + len(sub)
                if _ipaddress_accepts(sub) and (e == len(t) or t[e] not in b"_" and not chr(t[e]).isalnum()):
                    want = e
            assert R.match_ipv6(t, p) == want, (t, p)
            hits += want >= 0
    assert hits > 300, hits


def test_rules_on_written_examples():
    cases = {
        "IP_ADDRESS": [(b"host 10.0.0.255 up", 5, 15), (b"v1.2.3.4", 1, -1), (b"1.2.3.256", 0, -1),
                       (b"01.2.3.4", 0, -1), (b"1.2.3.4.5", 0, 7), (b"1.2.3.4.5", 2, 9)],
        "CVE_ID": [(b"(CVE-2021-44228)", 1, 15), (b"CVE-2021-123", 0, -1), (b"CVE-2021-12345678", 0, -1)],
        "MAC_ADDRESS": [(b"mac 00:1a:2B:3c:4d:5e.", 4, 21), (b"00:1a:2b:3c:4d", 0, -1)],
        "HASH": [(b"x " + b"a" * 40 + b" y", 2, 42), (b"a" * 41, 0, -1), (b"a" * 32 + b"g", 0, -1)],
        "URL": [(b"see https://a.corp/kb now", 4, 21), (b"xhttps://a", 1, -1)],
        "EMAIL_ADDRESS": [(b"to j.doe@mail.example.", 3, 21), (b"a@b.c1", 0, -1), (b"a@b.corp.x1", 0, 8)],
        "HOSTNAME": [(b"at db-1.site.corp.", 3, 17), (b"a.b.org1", 0, -1), (b"a.corp.lan", 0, 10)],
        "IPV6": [(b"gw fe80::1%eth0", 3, 10), (b"(2001:db8::8a2e:370:7334).", 1, 24), (b"::", 0, 2),
                 (b"ip ::ffff:10.0.0.1.", 3, 18), (b"00:1a:2b:3c:4d:5e", 0, -1), (b"12:30:45", 0, -1),
                 (b"1:2:3:4:5:6:7:8", 0, 15), (b"1:2:3:4:5:6:7:8:9", 0, -1), (b"x::1", 1, -1),
                 (b"fe80::1g", 0, -1), (b"::ffff:01.2.3.4", 0, -1), (b"1::2::3", 0, -1)],
        "CPE": [(b"(cpe:/a:apache:http_server:2.4.41) ", 1, 33), (b"cpe:2.3:o:microsoft:windows_10:1909:*:*:*:*", 0, 43),
                (b"xcpe:/a:b", 1, -1), (b"cpe:/ab:c", 0, -1), (b"cpe:2.3:*", 0, 9), (b"cpe:/*:x", 0, -1),
                (b"cpe:/a", 0, 6), (b"cpe:/a/b", 0, 6), (b"CPE:/a:b", 0, -1)],
    }
    for name, rows in cases.items():
        for t, p, e in rows:
            assert R.MATCHERS[name](t, p) == e, (name, t, p)


def test_merge_unions_overlaps_and_keeps_touching_spans_apart():
    # (begin, end, type, priority); NER spans have priority 0
    assert R.merge([(0, 5, 1, 3), (5, 9, 2, 1)]) == [(1, 0, 5), (2, 5, 9)]          # touching: apart
    assert R.merge([(0, 30, 6, 1), (8, 17, 2, 7)]) == [(6, 0, 30)]                   # URL holds a hostname
    assert R.merge([(0, 6, 1, 0), (2, 12, 1, 3)]) == [(1, 0, 12)]                    # NER truncated an IP
    assert R.merge([(0, 4, 3, 2), (0, 4, 5, 0)]) == [(5, 0, 4)]                      # tie: NER type wins
    assert R.merge([(0, 4, 3, 2), (3, 8, 4, 5), (7, 20, 6, 1)]) == [(6, 0, 20)]      # chain, longest member
    assert R.merge([(0, 4, 3, 4), (0, 4, 2, 2)]) == [(2, 0, 4)]                      # tie: lower recognizer
    assert R.merge([]) == []


def test_truncated_ner_span_is_extended_to_the_whole_entity():
    t = b"Host: 100.111.20.23\n"
    rt = R.recognizer_types(synth.TYPE_NAMES_17)
    # an NER span covering only "100.111" would leak ".20.23"
    got = R.resolve_record(t, [(1, 6, 13)], rt)
    assert got == [(1, 6, 19)]


def test_generator_gold_entities_are_covered():
    """Every gold entity of a recognised type lies inside one resolved span
    (recognizers alone, no NER spans).  Records are cut to an exact token
    count, so an entity ending at the record's last byte may be truncated and
    is left out."""
    names = synth.TYPE_NAMES_17
    rb = synth.generate_records(48, np.full(48, 300), len(names), 30522, 11)
    rt = R.recognizer_types(names)
    covered = total = 0
    for i in range(rb.n_records):
        t = rb.text[int(rb.cu_bytes[i]):int(rb.cu_bytes[i + 1])]
        spans = R.resolve_record(t, [], rt)
        for g in rb.gold_spans[rb.gold_spans[:, 0] == i]:
            typ, b, e = int(g[1]), int(g[2]), int(g[3])
            if names[typ - 1] == "PORT" or e == len(t):
                continue  # a port is a bare number that no pattern names
            total += 1
            covered += any(sb <= b and e <= se for _, sb, se in spans)
    assert total > 50 and covered == total, (covered, total)


def test_recognizer_type_mapping():
    """IPv6 emits the IP address type; CPE is off unless the label set has a
    CPE type; the binding's mapping equals the oracle's."""
    from paper_2606_15650_amd import api
    names = synth.TYPE_NAMES_17
    rt = R.recognizer_types(names)
    assert len(rt) == len(R.RECOGNIZERS) == 9
    ip = names.index("IP_ADDRESS") + 1
    assert rt[R.RECOGNIZERS.index("IP_ADDRESS")] == rt[R.RECOGNIZERS.index("IPV6")] == ip
    assert rt[R.RECOGNIZERS.index("CPE")] == 0
    with_cpe = names + ["CPE"]
    assert R.recognizer_types(with_cpe)[R.RECOGNIZERS.index("CPE")] == len(with_cpe)
    assert api.RECOGNIZERS == R.RECOGNIZERS
    for ns in (names, synth.TYPE_NAMES_9, with_cpe):
        assert api.recognizer_types(ns) == R.recognizer_types(ns)
