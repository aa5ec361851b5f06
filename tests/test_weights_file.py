"""The versioned weights file (anon_weights_write / anon_weights_info /
anon_model_load): layout pinned byte by byte against an independent reading
with struct and a Python FNV-1a-64, and every malformed file rejected before
any device is touched.  CPU only; loading onto a GPU is tested in test_gpu_weights_file.py."""
import os
import struct

import numpy as np
import pytest

import synth
from synth.configs import TINY


def _fnv1a64(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for b in data:
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


@pytest.fixture(scope="module")
def written(tmp_path_factory):
    from paper_2606_15650_amd import api
    W = synth.make_weights(TINY, 3)
    blob = synth.weights_blob(TINY, W)
    path = str(tmp_path_factory.mktemp("w") / "tiny.anonw")
    api.write_weights(path, TINY, blob)
    return path, blob


def test_layout_and_hash(written):
    path, blob = written
    raw = open(path, "rb").read()
    assert len(raw) == 64 + 4 * blob.size
    magic, version, kind = struct.unpack_from("<8sII", raw, 0)
    cfg = struct.unpack_from("<7if", raw, 16)
    n, fnv = struct.unpack_from("<QQ", raw, 48)
    assert magic == b"ANONWTS1" and version == 1 and kind == 0
    assert cfg[:7] == (TINY.n_layers, TINY.hidden, TINY.n_heads, TINY.ffn, TINY.vocab, TINY.n_labels, TINY.max_pos)
    assert cfg[7] == np.float32(TINY.ln_eps)
    assert n == blob.size
    assert raw[64:] == blob.astype("<f4").tobytes()
    # the Python FNV-1a-64 itself, on the published empty and "a" vectors
    assert _fnv1a64(b"") == 0xcbf29ce484222325 and _fnv1a64(b"a") == 0xaf63dc4c8601ec8c


def test_hash_matches_python_fnv_on_a_small_model(tmp_path):
    from paper_2606_15650_amd import api
    from synth.configs import ModelConfig
    cfg = ModelConfig(n_layers=1, hidden=64, n_heads=1, ffn=128, vocab=8, n_labels=3, max_pos=4)
    blob = synth.weights_blob(cfg, synth.make_weights(cfg, 1))
    path = str(tmp_path / "small.anonw")
    api.write_weights(path, cfg, blob)
    raw = open(path, "rb").read()
    assert struct.unpack_from("<Q", raw, 56)[0] == _fnv1a64(raw[64:])
    got, n = api.weights_info(path)
    assert n == blob.size and got["hidden"] == 64 and got["vocab"] == 8


def test_info_reads_back_the_config(written):
    from paper_2606_15650_amd import api
    path, blob = written
    got, n = api.weights_info(path)
    assert n == blob.size
    assert (got["n_layers"], got["hidden"], got["n_heads"], got["ffn"], got["vocab"], got["n_labels"],
            got["max_pos"]) == (TINY.n_layers, TINY.hidden, TINY.n_heads, TINY.ffn, TINY.vocab, TINY.n_labels,
                                TINY.max_pos)


def _corrupt(src, dst, fn):
    raw = bytearray(open(src, "rb").read())
    raw = fn(raw)
    open(dst, "wb").write(bytes(raw))
    return dst


@pytest.mark.parametrize("what,fn,needle", [
    ("payload byte", lambda r: r[:100] + bytes([r[100] ^ 1]) + r[101:], "hash"),
    ("truncated", lambda r: r[:-4], "size"),
    ("magic", lambda r: b"ANONWTS2" + r[8:], "magic"),
    ("version", lambda r: r[:8] + struct.pack("<I", 2) + r[12:], "version"),
    ("kind", lambda r: r[:12] + struct.pack("<I", 1) + r[16:], "kind"),
    ("float count", lambda r: r[:48] + struct.pack("<Q", 7) + r[56:], "floats"),
    ("config", lambda r: r[:20] + struct.pack("<i", 100) + r[24:], ""),
    ("header only", lambda r: r[:40], "header"),
])
def test_malformed_files_are_rejected_before_any_device_call(written, tmp_path, what, fn, needle):
    from paper_2606_15650_amd import api
    path, _ = written
    bad = _corrupt(path, str(tmp_path / "bad.anonw"), fn)
    with pytest.raises(api.AnonError) as e:
        api.weights_info(bad)
    assert e.value.status == -1 and needle in str(e.value), (what, str(e.value))
    # anon_model_load runs the same checks first: EINVAL, not a device error
    with pytest.raises(api.AnonError) as e:
        api.Model(TINY, None, "fp32", path=bad)
    assert e.value.status == -1, (what, str(e.value))


def test_missing_file_and_wrong_sizes(tmp_path):
    from paper_2606_15650_amd import api
    with pytest.raises(api.AnonError) as e:
        api.weights_info(str(tmp_path / "none.anonw"))
    assert e.value.status == -1
    blob = synth.weights_blob(TINY, synth.make_weights(TINY, 0))
    with pytest.raises(api.AnonError) as e:
        api.write_weights(str(tmp_path / "x.anonw"), TINY, blob[:-1])
    assert e.value.status == -1
    assert not os.path.exists(str(tmp_path / "x.anonw"))
