"""Pins of the preservation and mapping oracle on hand-made calls."""
import numpy as np

from oracle import pseudonym as P

KEY = b"k" * 32
NAMES = ["IP_ADDRESS", "HOSTNAME", "CVE_ID"]


def test_preserve_leaves_the_type_in_place():
    t = b"a 10.0.0.1 b db.corp c"
    spans = [(1, 2, 10), (2, 13, 20)]
    kept = P.preserve_spans(spans, [1])
    assert kept == [(2, 13, 20)]
    out = P.substitute(t, kept, NAMES, KEY, 4)
    assert out.startswith(b"a 10.0.0.1 b [HOSTNAME_") and out.endswith(b"] c")


def test_mapping_over_three_calls():
    a = b"x 10.0.0.1 y db.corp"
    b = b"db.corp 10.0.0.2 " + b"h" * 97
    calls = [
        (a, [0, len(a)], np.array([[0, 1, 2, 10], [0, 2, 13, 20]])),
        (b, [0, len(b)], np.array([[0, 3, 0, 7], [0, 1, 8, 16], [0, 2, 17, 114]])),  # db.corp as type 3; 97 bytes
        (a, [0, len(a)], np.array([[0, 1, 2, 10]])),
    ]
    rows = P.mapping_rows(calls, NAMES, KEY, 10, preserve=())
    want = [  # ordered by first call, then bytes
        (b"10.0.0.1", "IP_ADDRESS", 1, 3),
        (b"db.corp", "HOSTNAME", 1, 2),      # smallest type index: 2 (HOSTNAME) < 3
        (b"10.0.0.2", "IP_ADDRESS", 2, 2),
    ]
    assert [(r["original"], r["entity_type"], r["first_seen"], r["last_seen"]) for r in rows] == want
    for r in rows:
        assert r["full_hash"] == P.hmac_hex(KEY, r["original"]) and r["slug"] == r["full_hash"][:10]
    # a preserved type never enters the mapping
    rows = P.mapping_rows(calls, NAMES, KEY, 10, preserve=(1,))
    assert [r["original"] for r in rows] == [b"db.corp"]
