"""ctypes binding of libanon.so (include/anon.h).

Argument marshalling only: every step of the NER + pseudonymize path runs in
the library's HIP kernels.  Device buffers are torch tensors on a ROCm device
(or raw integer device addresses); streams are torch streams (or raw
hipStream_t handles).  If libanon.so is missing the import of the library
fails loudly - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libanon.so")

ANON_OK, ANON_PENDING = 0, 1
STATUS = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECAPACITY",
          -5: "EBUSY", -6: "ENOTFOUND", -7: "EDATA"}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2}
ERR_TOKEN_ID, ERR_SEQLENS, ERR_LABEL, ERR_SPAN, ERR_SPAN_CAP, ERR_OUT_CAP, ERR_TEXT = 1, 2, 4, 8, 16, 32, 64
KCLASS = {"qkv": 0, "attn": 1, "oproj": 2, "ffn1": 3, "ffn2": 4, "ln": 5, "embed": 6, "cls": 7}


class AnonError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class ModelConfigC(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("hidden", C.c_int32), ("n_heads", C.c_int32), ("ffn", C.c_int32),
                ("vocab", C.c_int32), ("n_labels", C.c_int32), ("max_pos", C.c_int32), ("ln_eps", C.c_float)]


class ModernConfigC(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("hidden", C.c_int32), ("n_heads", C.c_int32),
                ("intermediate", C.c_int32), ("vocab", C.c_int32), ("n_labels", C.c_int32),
                ("max_pos", C.c_int32), ("ln_eps", C.c_float), ("local_window", C.c_int32),
                ("global_every", C.c_int32), ("theta_global", C.c_float), ("theta_local", C.c_float)]


class SpanC(C.Structure):
    _fields_ = [("record", C.c_int32), ("type", C.c_int32), ("begin", C.c_int64), ("end", C.c_int64)]


SPAN_BYTES = C.sizeof(SpanC)  # 24


class ServerConfigC(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_batch_tokens", C.c_int32), ("n_streams", C.c_int32),
                ("max_queue", C.c_int32), ("max_request_tokens", C.c_int32), ("graph_buckets", C.c_int32)]


class RequestC(C.Structure):
    _fields_ = [("n_records", C.c_int32), ("ids", C.POINTER(C.c_int32)), ("cu_seqlens", C.POINTER(C.c_int32)),
                ("tok_off", C.POINTER(C.c_int32)), ("text", C.POINTER(C.c_uint8)),
                ("cu_bytes", C.POINTER(C.c_int64))]


class ServerCountersC(C.Structure):
    _fields_ = [("arena_bytes", C.c_int64), ("peak_arena_bytes", C.c_int64), ("micro_batches", C.c_int64),
                ("max_concurrent", C.c_int32), ("graph_launches", C.c_int64)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_records", C.c_int32), ("n_tokens", C.c_int32), ("n_spans", C.c_int32),
                ("out", C.POINTER(C.c_uint8)), ("cu_out", C.POINTER(C.c_int64)), ("labels", C.POINTER(C.c_uint8)),
                ("spans", C.POINTER(SpanC)), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


_lib = None
vp, sz, i32, i64, u64 = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64, C.c_uint64
_SIGS = {
    "anon_last_error": ([], C.c_char_p),
    "anon_version": ([], i32),
    "anon_device_errors": ([i32, C.POINTER(C.c_uint32), i32], i32),
    "anon_model_create": ([C.POINTER(ModelConfigC), vp, sz, i32, vp, i32, C.POINTER(vp)], i32),
    "anon_model_free": ([vp], None),
    "anon_weights_write": ([C.c_char_p, C.POINTER(ModelConfigC), vp, sz], i32),
    "anon_weights_info": ([C.c_char_p, C.POINTER(ModelConfigC), C.POINTER(sz)], i32),
    "anon_model_load": ([C.c_char_p, i32, vp, i32, C.POINTER(vp)], i32),
    "anon_ner_workspace_size": ([vp, i32, i32, C.POINTER(sz)], i32),
    "ner_forward": ([vp, vp, vp, i32, i32, vp, vp, vp, vp, sz, vp], i32),
    "anon_encoder_hidden": ([vp, vp, vp, i32, i32, i32, vp, vp, sz, vp], i32),
    "ner_forward_capture": ([vp, vp, vp, i32, i32, vp, vp, vp, vp, sz, C.POINTER(vp)], i32),
    "ner_forward_capture_bucket": ([vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, sz, C.POINTER(vp)], i32),
    "anon_graph_launch": ([vp, vp], i32),
    "anon_graph_free": ([vp], None),
    "anon_ner_windowed_workspace_size": ([vp, vp, i32, i32, i32, C.POINTER(sz)], i32),
    "ner_forward_windowed": ([vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, sz, vp], i32),
    "anon_decode_workspace_size": ([i32, i32, C.POINTER(sz)], i32),
    "decode_spans": ([vp, vp, vp, i32, i32, i32, vp, i32, vp, vp, sz, vp], i32),
    "anon_autotune_attention": ([vp, vp, i32, i32, vp, sz, vp, C.POINTER(i32), C.POINTER(C.c_float), i32], i32),
    "anon_model_set_attn_config": ([vp, i32], i32),
    "anon_model_get_attn_config": ([vp], i32),
    "anon_attn_config_count": ([], i32),
    "anon_attn_config_name": ([i32], C.c_char_p),
    "anon_modern_create": ([vp, vp, sz, i32, i32, C.POINTER(vp)], i32),
    "anon_modern_free": ([vp], None),
    "anon_modern_workspace_size": ([vp, i32, i32, C.POINTER(sz)], i32),
    "modern_ner_forward": ([vp, vp, vp, i32, i32, vp, vp, vp, vp, sz, vp], i32),
    "anon_modern_hidden": ([vp, vp, vp, i32, i32, i32, vp, vp, sz, vp], i32),
    "anon_modern_set_tiles": ([vp, C.POINTER(i32), i32], i32),
    "anon_modern_get_tiles": ([vp, C.POINTER(i32), C.POINTER(i32)], i32),
    "decode_spans_noalloc": ([vp, vp, vp, i32, i32, i32, vp, i32, vp, vp], i32),
    "anon_recognize_workspace_size": ([i64, i32, C.POINTER(sz)], i32),
    "anon_field_workspace_size": ([i64, i32, C.POINTER(sz)], i32),
    "field_spans": ([vp, vp, i32, i64, C.POINTER(C.c_char_p), C.POINTER(i32), i32, i32, vp, i32, vp, vp, sz, vp],
                    i32),
    "recognize_spans": ([vp, vp, i32, i64, C.POINTER(i32), i32, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
    "anon_pcache_create": ([vp, sz, i32, C.POINTER(C.c_char_p), i32, i64, i32, C.POINTER(vp)], i32),
    "anon_pcache_free": ([vp], None),
    "anon_pcache_clear": ([vp, vp], i32),
    "anon_pcache_set_enabled": ([vp, i32], i32),
    "anon_pcache_stats": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)], i32),
    "anon_pcache_set_preserve": ([vp, C.POINTER(i32), i32], i32),
    "anon_pcache_export": ([vp, vp, i64, C.POINTER(i64)], i32),
    "anon_pseudonymize_workspace_size": ([i32, i32, C.POINTER(sz)], i32),
    "pseudonymize": ([vp, vp, vp, i32, vp, vp, i32, vp, i64, vp, vp, sz, vp], i32),
    "anon_server_start": ([vp, vp, C.POINTER(ServerConfigC), C.POINTER(vp)], i32),
    "anon_submit": ([vp, C.POINTER(RequestC), C.POINTER(u64)], i32),
    "anon_poll": ([vp, u64, C.POINTER(ResultC)], i32),
    "anon_release": ([vp, u64], i32),
    "anon_server_stop": ([vp], i32),
    "anon_server_stats": ([vp, C.POINTER(ServerCountersC)], i32),
    "anon_autotune": ([vp, i32, vp, sz, vp, C.POINTER(i32), C.POINTER(C.c_float), i32], i32),
    "anon_model_set_tiles": ([vp, C.POINTER(i32)], i32),
    "anon_model_set_tile_groups": ([vp, C.POINTER(i32)], i32),
    "anon_model_get_tiles": ([vp, C.POINTER(i32), C.POINTER(i32)], i32),
    "anon_tile_config_count": ([i32], i32),
    "anon_tile_config_name": ([i32, i32], C.c_char_p),
    "anon_prof_enable": ([i32, i32], i32),
    "anon_prof_read": ([i32, C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(C.c_double)], i32),
}
EXPORTED = sorted(_SIGS)


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2606_15650_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        if os.environ.get("ANON_TRACE", "") not in ("", "0"):
            _start_trace()
    return _lib


def _start_trace():
    """ANON_TRACE=1: time every kernel class from the first use of the library
    on (HIP events on the launch streams) and print the totals to stderr at
    exit.  While it is on, forward graphs cannot be captured (the capture
    calls refuse with ANON_EINVAL)."""
    import atexit
    import sys
    for k in KCLASS:
        lib().anon_prof_enable(KCLASS[k], 1)

    def report():
        rows = []
        for k in KCLASS:
            r = prof_read(k)
            if r["launches"]:
                tf = r["flops"] / (r["ms"] * 1e-3) / 1e12 if r["flops"] and r["ms"] else None
                rows.append(f"  {k:6s} launches {r['launches']:7d}  total {r['ms']:10.3f} ms  "
                            f"mean {r['ms'] / r['launches']:8.4f} ms" + (f"  {tf:7.1f} TFLOP/s" if tf else ""))
        print("[ANON_TRACE] kernel time per class\n" + "\n".join(rows), file=sys.stderr, flush=True)

    atexit.register(report)


def _check(fn: str, st: int) -> int:
    if st < 0:
        raise AnonError(fn, st, lib().anon_last_error().decode(errors="replace"))
    return st


def ptr(x) -> int | None:
    """Device address of a torch tensor / integer / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def stream_handle(stream=None) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ model --
def _config_c(cfg) -> ModelConfigC:
    return ModelConfigC(cfg.n_layers, cfg.hidden, cfg.n_heads, cfg.ffn, cfg.vocab, cfg.n_labels, cfg.max_pos,
                        cfg.ln_eps)


def write_weights(path: str, cfg, weights_blob: np.ndarray):
    """anon_weights_write: the versioned weights file of an encoder."""
    blob = np.ascontiguousarray(weights_blob, dtype=np.float32)
    c = _config_c(cfg)
    _check("anon_weights_write", lib().anon_weights_write(os.fsencode(path), C.byref(c), blob.ctypes.data,
                                                          blob.size))


def weights_info(path: str) -> tuple[dict, int]:
    """anon_weights_info: (config fields, float count) of a checked weights file."""
    c, n = ModelConfigC(), sz()
    _check("anon_weights_info", lib().anon_weights_info(os.fsencode(path), C.byref(c), C.byref(n)))
    return {f: getattr(c, f) for f, _ in ModelConfigC._fields_}, n.value


class Model:
    """An encoder uploaded to one device (``anon_model_create``; ``Model.load``
    for ``anon_model_load`` of a weights file)."""

    def __init__(self, cfg, weights_blob: np.ndarray | None, precision: str = "bf16", act_scales=None,
                 device: int = 0, path: str | None = None):
        self.cfg = cfg
        self.precision = precision
        sc = None
        if act_scales is not None:
            self._scales = np.ascontiguousarray(np.asarray(act_scales, dtype=np.float32).reshape(-1))
            sc = self._scales.ctypes.data
        h = vp()
        if path is not None:
            _check("anon_model_load", lib().anon_model_load(os.fsencode(path), PRECISION[precision], sc, device,
                                                            C.byref(h)))
        else:
            blob = np.ascontiguousarray(weights_blob, dtype=np.float32)
            c = _config_c(cfg)
            _check("anon_model_create", lib().anon_model_create(C.byref(c), blob.ctypes.data, blob.size,
                                                                PRECISION[precision], sc, device, C.byref(h)))
        self.handle = h.value
        self.device = device

    @classmethod
    def load(cls, path: str, cfg, precision: str = "bf16", act_scales=None, device: int = 0) -> "Model":
        """The encoder of a weights file; ``cfg`` (the caller's description of
        it) must match the file's config."""
        got, _ = weights_info(path)
        want = {f: getattr(_config_c(cfg), f) for f, _ in ModelConfigC._fields_}
        if got != want:
            raise AnonError("anon_model_load", -1, f"weights file config {got} differs from {want}")
        return cls(cfg, None, precision, act_scales, device, path=path)

    def workspace_size(self, T: int, B: int) -> int:
        n = sz()
        _check("anon_ner_workspace_size", lib().anon_ner_workspace_size(self.handle, T, B, C.byref(n)))
        return n.value

    def windowed_workspace_size(self, cu_seqlens: np.ndarray, window: int, stride: int) -> int:
        cu = np.ascontiguousarray(cu_seqlens, dtype=np.int32)
        n = sz()
        _check("anon_ner_windowed_workspace_size",
               lib().anon_ner_windowed_workspace_size(self.handle, cu.ctypes.data, cu.size - 1, window, stride,
                                                      C.byref(n)))
        return n.value

    def tile_configs(self) -> list[str]:
        p = PRECISION[self.precision]
        return [lib().anon_tile_config_name(p, i).decode() for i in range(lib().anon_tile_config_count(p))]

    def autotune(self, T: int, d_workspace, ws_bytes: int, stream=None):
        """Pick the fastest GEMM tiles on T rows; returns (chosen[4], times_ms[4][n])."""
        n = len(self.tile_configs())
        chosen = (i32 * 4)()
        times = (C.c_float * (4 * n))()
        _check("anon_autotune", lib().anon_autotune(self.handle, T, ptr(d_workspace), ws_bytes,
                                                    stream_handle(stream), chosen, times, n))
        return list(chosen), np.array(times[:], dtype=np.float32).reshape(4, n)

    @staticmethod
    def attn_configs() -> list[str]:
        return [lib().anon_attn_config_name(i).decode() for i in range(lib().anon_attn_config_count())]

    def autotune_attention(self, d_cu_seqlens, B: int, T: int, d_workspace, ws_bytes: int, stream=None):
        """Pick the fastest attention tiles on this batch's lengths; returns (chosen, times_ms[n])."""
        n = len(self.attn_configs())
        chosen = i32()
        times = (C.c_float * n)()
        _check("anon_autotune_attention",
               lib().anon_autotune_attention(self.handle, ptr(d_cu_seqlens), B, T, ptr(d_workspace), ws_bytes,
                                             stream_handle(stream), C.byref(chosen), times, n))
        return chosen.value, np.array(times[:], dtype=np.float32)

    def set_attn_config(self, config: int):
        _check("anon_model_set_attn_config", lib().anon_model_set_attn_config(self.handle, int(config)))

    def attn_config(self) -> int:
        return lib().anon_model_get_attn_config(self.handle)

    def set_tiles(self, tiles):
        t = (i32 * 4)(*[int(x) for x in tiles])
        _check("anon_model_set_tiles", lib().anon_model_set_tiles(self.handle, t))

    def set_tile_groups(self, groups):
        g = (i32 * 4)(*[int(x) for x in groups])
        _check("anon_model_set_tile_groups", lib().anon_model_set_tile_groups(self.handle, g))

    def get_tiles(self) -> tuple[list[int], list[int]]:
        """(tile configuration, tile group) of each encoder GEMM."""
        t, g = (i32 * 4)(), (i32 * 4)()
        _check("anon_model_get_tiles", lib().anon_model_get_tiles(self.handle, t, g))
        return list(t), list(g)

    def close(self):
        if getattr(self, "handle", None):
            lib().anon_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ner_forward(model, d_ids, d_cu_seqlens, B: int, T: int, d_labels, d_logits=None, d_margin=None,
                d_workspace=None, ws_bytes: int = 0, stream=None):
    if isinstance(model, ModernModel):
        _check("modern_ner_forward", lib().modern_ner_forward(model.handle, ptr(d_ids), ptr(d_cu_seqlens), B, T,
                                                              ptr(d_labels), ptr(d_logits), ptr(d_margin),
                                                              ptr(d_workspace), ws_bytes, stream_handle(stream)))
        return
    _check("ner_forward", lib().ner_forward(model.handle, ptr(d_ids), ptr(d_cu_seqlens), B, T, ptr(d_labels),
                                            ptr(d_logits), ptr(d_margin), ptr(d_workspace), ws_bytes,
                                            stream_handle(stream)))


class ModernModel:
    """A ModernBERT-style encoder uploaded to one device (``anon_modern_create``)."""

    def __init__(self, cfg, weights_blob: np.ndarray, precision: str = "bf16", device: int = 0):
        blob = np.ascontiguousarray(weights_blob, dtype=np.float32)
        self.cfg = cfg
        self.precision = precision
        c = ModernConfigC(cfg.n_layers, cfg.hidden, cfg.n_heads, cfg.intermediate, cfg.vocab, cfg.n_labels,
                          cfg.max_pos, cfg.ln_eps, cfg.local_window, cfg.global_every, cfg.theta_global,
                          cfg.theta_local)
        h = vp()
        _check("anon_modern_create", lib().anon_modern_create(C.byref(c), blob.ctypes.data, blob.size,
                                                              PRECISION[precision], device, C.byref(h)))
        self.handle = h.value

    def workspace_size(self, T: int, B: int) -> int:
        n = sz()
        _check("anon_modern_workspace_size", lib().anon_modern_workspace_size(self.handle, T, B, C.byref(n)))
        return n.value

    def hidden(self, d_ids, d_cu_seqlens, B: int, T: int, n_layers: int, d_hidden, d_workspace, ws_bytes: int,
               stream=None):
        _check("anon_modern_hidden", lib().anon_modern_hidden(self.handle, ptr(d_ids), ptr(d_cu_seqlens), B, T,
                                                              n_layers, ptr(d_hidden), ptr(d_workspace), ws_bytes,
                                                              stream_handle(stream)))

    def set_tiles(self, tiles, attn_config: int = -1):
        t = (i32 * 5)(*[int(x) for x in tiles])
        _check("anon_modern_set_tiles", lib().anon_modern_set_tiles(self.handle, t, int(attn_config)))

    def get_tiles(self) -> tuple[list[int], int]:
        t, a = (i32 * 5)(), i32()
        _check("anon_modern_get_tiles", lib().anon_modern_get_tiles(self.handle, t, C.byref(a)))
        return list(t), a.value

    def tile_configs(self) -> list[str]:
        p = PRECISION[self.precision]
        return [lib().anon_tile_config_name(p, i).decode() for i in range(lib().anon_tile_config_count(p))]

    attn_configs = staticmethod(Model.attn_configs)

    def close(self):
        if getattr(self, "handle", None):
            lib().anon_modern_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ForwardGraph:
    """ner_forward recorded as one HIP graph (``ner_forward_capture``): each
    ``launch`` runs the layer stack on the capture's buffers as they are at
    that time.  Keeps the model and the buffers alive while it exists."""

    def __init__(self, handle: int, keep: tuple):
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None):
        _check("anon_graph_launch", lib().anon_graph_launch(self.handle, stream_handle(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().anon_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ner_forward_capture(model: Model, d_ids, d_cu_seqlens, B: int, T: int, d_labels, d_logits=None,
                        d_margin=None, d_workspace=None, ws_bytes: int = 0) -> ForwardGraph:
    h = vp()
    _check("ner_forward_capture",
           lib().ner_forward_capture(model.handle, ptr(d_ids), ptr(d_cu_seqlens), B, T, ptr(d_labels),
                                     ptr(d_logits), ptr(d_margin), ptr(d_workspace), ws_bytes, C.byref(h)))
    return ForwardGraph(h.value, (model, d_ids, d_cu_seqlens, d_labels, d_logits, d_margin, d_workspace))


def ner_forward_capture_bucket(model: Model, d_ids, d_cu_seqlens, d_n_tokens, B_cap: int, T_cap: int, d_labels,
                               d_logits=None, d_margin=None, d_workspace=None, ws_bytes: int = 0) -> ForwardGraph:
    h = vp()
    _check("ner_forward_capture_bucket",
           lib().ner_forward_capture_bucket(model.handle, ptr(d_ids), ptr(d_cu_seqlens), ptr(d_n_tokens), B_cap,
                                            T_cap, ptr(d_labels), ptr(d_logits), ptr(d_margin), ptr(d_workspace),
                                            ws_bytes, C.byref(h)))
    return ForwardGraph(h.value, (model, d_ids, d_cu_seqlens, d_n_tokens, d_labels, d_logits, d_margin,
                                  d_workspace))


def encoder_hidden(model: Model, d_ids, d_cu_seqlens, B: int, T: int, n_layers: int, d_hidden, d_workspace,
                   ws_bytes: int, stream=None):
    _check("anon_encoder_hidden", lib().anon_encoder_hidden(model.handle, ptr(d_ids), ptr(d_cu_seqlens), B, T,
                                                            n_layers, ptr(d_hidden), ptr(d_workspace), ws_bytes,
                                                            stream_handle(stream)))


def ner_forward_windowed(model: Model, d_ids, d_cu_seqlens, h_cu_seqlens: np.ndarray, B: int, T: int, window: int,
                         stride: int, d_labels, d_logits=None, d_margin=None, d_workspace=None, ws_bytes: int = 0,
                         stream=None):
    cu = np.ascontiguousarray(h_cu_seqlens, dtype=np.int32)
    _check("ner_forward_windowed",
           lib().ner_forward_windowed(model.handle, ptr(d_ids), ptr(d_cu_seqlens), cu.ctypes.data, B, T, window,
                                      stride, ptr(d_labels), ptr(d_logits), ptr(d_margin), ptr(d_workspace),
                                      ws_bytes, stream_handle(stream)))


def decode_workspace_size(T: int, B: int) -> int:
    n = sz()
    _check("anon_decode_workspace_size", lib().anon_decode_workspace_size(T, B, C.byref(n)))
    return n.value


def decode_spans(d_labels, d_tok_off, d_cu_seqlens, B: int, T: int, n_types: int, d_spans, span_cap: int,
                 d_cu_spans, d_workspace, ws_bytes: int, stream=None):
    _check("decode_spans", lib().decode_spans(ptr(d_labels), ptr(d_tok_off), ptr(d_cu_seqlens), B, T, n_types,
                                              ptr(d_spans), span_cap, ptr(d_cu_spans), ptr(d_workspace), ws_bytes,
                                              stream_handle(stream)))


NOALLOC_MAX_TOKENS = 1 << 20  # ANON_NOALLOC_MAX_TOKENS


def decode_spans_noalloc(d_labels, d_tok_off, d_cu_seqlens, B: int, T: int, n_types: int, d_spans, span_cap: int,
                         d_cu_spans, stream=None):
    """decode_spans with the library's per-device scratch array (no workspace, no allocation)."""
    _check("decode_spans_noalloc", lib().decode_spans_noalloc(ptr(d_labels), ptr(d_tok_off), ptr(d_cu_seqlens), B, T,
                                                              n_types, ptr(d_spans), span_cap, ptr(d_cu_spans),
                                                              stream_handle(stream)))


# Recognizer order of recognize_spans (the type each emits is chosen per call),
# and the entity type each emits by default.
RECOGNIZERS = ["URL", "EMAIL_ADDRESS", "IP_ADDRESS", "MAC_ADDRESS", "HASH", "CVE_ID", "HOSTNAME", "IPV6", "CPE"]
RECOGNIZER_TYPE = {r: r for r in RECOGNIZERS} | {"IPV6": "IP_ADDRESS"}


def recognizer_types(type_names) -> list[int]:
    """Type index (1-based) each recognizer emits for a model's type names; 0 = off."""
    names = list(type_names)
    return [names.index(RECOGNIZER_TYPE[r]) + 1 if RECOGNIZER_TYPE[r] in names else 0 for r in RECOGNIZERS]


def recognize_workspace_size(n_bytes: int, B: int) -> int:
    n = sz()
    _check("anon_recognize_workspace_size", lib().anon_recognize_workspace_size(n_bytes, B, C.byref(n)))
    return n.value


def recognize_spans(d_text, d_cu_bytes, B: int, n_bytes: int, rec_types, n_types: int, d_ner_spans, d_ner_cu,
                    ner_cap: int, d_spans, span_cap: int, d_cu_spans, d_workspace, ws_bytes: int, stream=None):
    if len(rec_types) != len(RECOGNIZERS):
        raise ValueError(f"rec_types needs {len(RECOGNIZERS)} entries, one per recognizer")
    rt = (i32 * len(RECOGNIZERS))(*[int(x) for x in rec_types])
    _check("recognize_spans", lib().recognize_spans(ptr(d_text), ptr(d_cu_bytes), B, n_bytes, rt, n_types,
                                                    ptr(d_ner_spans), ptr(d_ner_cu), ner_cap, ptr(d_spans),
                                                    span_cap, ptr(d_cu_spans), ptr(d_workspace), ws_bytes,
                                                    stream_handle(stream)))


def field_workspace_size(n_bytes: int, B: int) -> int:
    n = sz()
    _check("anon_field_workspace_size", lib().anon_field_workspace_size(n_bytes, B, C.byref(n)))
    return n.value


def field_spans(d_text, d_cu_bytes, B: int, n_bytes: int, fields: dict, n_types: int, d_spans, span_cap: int,
                d_cu_spans, d_workspace, ws_bytes: int, stream=None):
    """fields: {field name (str or bytes): type index 1..n_types}."""
    items = list(fields.items())
    names = (C.c_char_p * max(1, len(items)))(*[k if isinstance(k, bytes) else k.encode() for k, _ in items])
    types = (i32 * max(1, len(items)))(*[int(v) for _, v in items])
    _check("field_spans", lib().field_spans(ptr(d_text), ptr(d_cu_bytes), B, n_bytes, names, types, len(items),
                                            n_types, ptr(d_spans), span_cap, ptr(d_cu_spans), ptr(d_workspace),
                                            ws_bytes, stream_handle(stream)))


# ------------------------------------------------------------- pseudonyms --
class _Mapping(C.Structure):
    _fields_ = [("type", i32), ("len", i32), ("bytes", C.c_uint8 * 96), ("digest", C.c_uint8 * 32),
                ("first_call", C.c_uint32), ("last_call", C.c_uint32)]


class PseudonymCache:
    """HMAC key, slug length, type names and the device entity->digest table."""

    def __init__(self, key: bytes, slug_hex: int, type_names, capacity: int = 1 << 20, device: int = 0):
        names = (C.c_char_p * len(type_names))(*[n.encode() for n in type_names])
        kb = (C.c_uint8 * max(1, len(key))).from_buffer_copy(key or b"\0")
        h = vp()
        _check("anon_pcache_create", lib().anon_pcache_create(C.addressof(kb), len(key), slug_hex, names,
                                                              len(type_names), capacity, device, C.byref(h)))
        self.handle = h.value
        self.type_names = list(type_names)
        self.slug = slug_hex

    def clear(self, stream=None):
        _check("anon_pcache_clear", lib().anon_pcache_clear(self.handle, stream_handle(stream)))

    def set_enabled(self, on: bool):
        _check("anon_pcache_set_enabled", lib().anon_pcache_set_enabled(self.handle, 1 if on else 0))

    def stats(self) -> dict:
        a, b, c = i64(), i64(), i64()
        _check("anon_pcache_stats", lib().anon_pcache_stats(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return {"lookups": a.value, "hits": b.value, "entries": c.value}

    def set_preserve(self, types):
        """Types (names or 1-based indices) whose spans are left as they are."""
        idx = [self.type_names.index(t) + 1 if isinstance(t, str) else int(t) for t in types]
        arr = (i32 * max(1, len(idx)))(*idx)
        _check("anon_pcache_set_preserve", lib().anon_pcache_set_preserve(self.handle, arr, len(idx)))

    def export(self) -> list[dict]:
        """The entity <-> pseudonym mapping held by the table (see anon_pcache_export)."""
        n = i64()
        _check("anon_pcache_export", lib().anon_pcache_export(self.handle, None, 0, C.byref(n)))
        rows = (_Mapping * max(1, n.value))()
        _check("anon_pcache_export", lib().anon_pcache_export(self.handle, C.addressof(rows), n.value, C.byref(n)))
        out = []
        for r in rows[:n.value]:
            full = bytes(r.digest).hex()
            out.append({"entity_type": self.type_names[r.type - 1], "original": bytes(r.bytes[:r.len]),
                        "slug": full[:self.slug], "full_hash": full, "first_seen": r.first_call,
                        "last_seen": r.last_call})
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().anon_pcache_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pseudonymize_workspace_size(B: int, span_cap: int) -> int:
    n = sz()
    _check("anon_pseudonymize_workspace_size", lib().anon_pseudonymize_workspace_size(B, span_cap, C.byref(n)))
    return n.value


def pseudonymize(cache: PseudonymCache, d_text, d_cu_bytes, B: int, d_spans, d_cu_spans, span_cap: int, d_out,
                 out_cap: int, d_cu_out, d_workspace, ws_bytes: int, stream=None):
    _check("pseudonymize", lib().pseudonymize(cache.handle, ptr(d_text), ptr(d_cu_bytes), B, ptr(d_spans),
                                              ptr(d_cu_spans), span_cap, ptr(d_out), out_cap, ptr(d_cu_out),
                                              ptr(d_workspace), ws_bytes, stream_handle(stream)))


def device_errors(device: int = 0, clear: bool = True) -> int:
    f = C.c_uint32()
    _check("anon_device_errors", lib().anon_device_errors(device, C.byref(f), 1 if clear else 0))
    return f.value


# ------------------------------------------------------------------ timing --
def prof_enable(kclass: str, on: bool = True):
    _check("anon_prof_enable", lib().anon_prof_enable(KCLASS[kclass], 1 if on else 0))


def prof_read(kclass: str) -> dict:
    n, ms, fl = i64(), C.c_double(), C.c_double()
    _check("anon_prof_read", lib().anon_prof_read(KCLASS[kclass], C.byref(n), C.byref(ms), C.byref(fl)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value}


# ------------------------------------------------------------------ server --
class Server:
    """Continuous-batching server (anon_server_start / submit / poll)."""

    def __init__(self, model: Model, cache: PseudonymCache, hbm_budget_bytes: int = 64 << 30,
                 max_batch_tokens: int = 131072, n_streams: int = 2, max_queue: int = 4096,
                 max_request_tokens: int = 0, graph_buckets: int = 0):
        cfg = ServerConfigC(hbm_budget_bytes, max_batch_tokens, n_streams, max_queue, max_request_tokens,
                            graph_buckets)
        h = vp()
        _check("anon_server_start", lib().anon_server_start(model.handle, cache.handle, C.byref(cfg), C.byref(h)))
        self.handle = h.value
        self._keep = (model, cache)

    def submit(self, ids: np.ndarray, cu_seqlens: np.ndarray, tok_off: np.ndarray, text: bytes,
               cu_bytes: np.ndarray) -> int:
        ids = np.ascontiguousarray(ids, np.int32)
        cu = np.ascontiguousarray(cu_seqlens, np.int32)
        off = np.ascontiguousarray(tok_off, np.int32)
        cb = np.ascontiguousarray(cu_bytes, np.int64)
        tb = np.frombuffer(text, dtype=np.uint8) if len(text) else np.zeros(1, np.uint8)
        req = RequestC(cu.size - 1, ids.ctypes.data_as(C.POINTER(C.c_int32)),
                       cu.ctypes.data_as(C.POINTER(C.c_int32)), off.ctypes.data_as(C.POINTER(C.c_int32)),
                       tb.ctypes.data_as(C.POINTER(C.c_uint8)), cb.ctypes.data_as(C.POINTER(C.c_int64)))
        t = u64()
        _check("anon_submit", lib().anon_submit(self.handle, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else a dict with the request's outputs (copied)."""
        r = ResultC()
        st = _check("anon_poll", lib().anon_poll(self.handle, ticket, C.byref(r)))
        if st == ANON_PENDING:
            return None
        out = {"status": r.status, "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done,
               "n_records": r.n_records}
        if r.status == ANON_OK:
            cu = np.ctypeslib.as_array(r.cu_out, shape=(r.n_records + 1,)).copy()
            n = int(cu[-1])
            out["cu_out"] = cu
            out["out"] = C.string_at(r.out, n) if n else b""
            out["labels"] = (np.ctypeslib.as_array(r.labels, shape=(r.n_tokens,)).copy()
                             if r.n_tokens else np.zeros(0, np.uint8))
            sp = np.zeros((r.n_spans, 4), np.int64)
            for i in range(r.n_spans):
                s = r.spans[i]
                sp[i] = (s.record, s.type, s.begin, s.end)
            out["spans"] = sp
        return out

    def release(self, ticket: int):
        _check("anon_release", lib().anon_release(self.handle, ticket))

    def stats(self) -> dict:
        """anon_server_stats: arena size, peak arena bytes in use, micro-batches
        launched, most micro-batches in flight at once, forward graph replays."""
        c = ServerCountersC()
        _check("anon_server_stats", lib().anon_server_stats(self.handle, C.byref(c)))
        return {"arena_bytes": c.arena_bytes, "peak_arena_bytes": c.peak_arena_bytes,
                "micro_batches": c.micro_batches, "max_concurrent": c.max_concurrent,
                "graph_launches": c.graph_launches}

    def stop(self):
        if getattr(self, "handle", None):
            _check("anon_server_stop", lib().anon_server_stop(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
