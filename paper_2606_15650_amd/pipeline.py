"""Device plumbing around the C ABI: torch allocates HBM buffers and streams,
the library does every step of the path.

``DeviceBatch`` uploads a packed batch of records; ``Pipeline`` owns the
workspaces and runs NER -> span decoding -> pseudonym substitution on one
stream.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class DeviceBatch:
    """A packed batch resident in HBM: ids, cu_seqlens, token offsets, text, cu_bytes."""

    def __init__(self, batch, device: str = "cuda:0"):
        self.B = int(batch.n_records)
        self.T = int(batch.n_tokens)
        self.n_bytes = len(batch.text)
        self.h_cu = np.ascontiguousarray(batch.cu_seqlens, np.int32)
        dev = torch.device(device)
        self.ids = torch.from_numpy(np.ascontiguousarray(batch.ids, np.int32)).to(dev)
        self.cu = torch.from_numpy(self.h_cu.copy()).to(dev)
        self.tok_off = torch.from_numpy(np.ascontiguousarray(batch.tok_off, np.int32).reshape(-1, 2)).to(dev)
        tb = np.frombuffer(batch.text, dtype=np.uint8) if self.n_bytes else np.zeros(1, np.uint8)
        self.text = torch.from_numpy(tb.copy()).to(dev)
        self.cu_bytes = torch.from_numpy(np.ascontiguousarray(batch.cu_bytes, np.int64)).to(dev)
        self.device = dev


def spans_to_numpy(spans: torch.Tensor, n: int) -> np.ndarray:
    """Device span rows (24-byte anon_span) -> int64 [n, 4] (record, type, begin, end)."""
    raw = spans[:n].cpu().numpy().reshape(-1, 3)
    rec = (raw[:, 0] & 0xFFFFFFFF).astype(np.int64)
    typ = (raw[:, 0] >> 32).astype(np.int64)
    return np.stack([rec, typ, raw[:, 1], raw[:, 2]], axis=1) if n else np.zeros((0, 4), np.int64)


class Pipeline:
    def __init__(self, model: api.Model, cache: api.PseudonymCache | None = None, device: str = "cuda:0"):
        self.model = model
        self.cache = cache
        self.device = torch.device(device)
        self._ws: dict[str, torch.Tensor] = {}
        self.n_types = (model.cfg.n_labels - 1) // 2

    def _buf(self, name: str, nbytes: int) -> torch.Tensor:
        t = self._ws.get(name)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws[name] = t
        return t

    def ner(self, db: DeviceBatch, logits: bool = False, margin: bool = True, window: int = 0, stride: int = 0,
            stream=None):
        C = self.model.cfg.n_labels
        labels = torch.empty(max(db.T, 1), dtype=torch.uint8, device=self.device)
        z = torch.empty((max(db.T, 1), C), dtype=torch.float32, device=self.device) if logits else None
        m = torch.empty(max(db.T, 1), dtype=torch.float32, device=self.device) if margin else None
        if window:
            n = self.model.windowed_workspace_size(db.h_cu, window, stride)
            ws = self._buf("ner_win", n)
            api.ner_forward_windowed(self.model, db.ids, db.cu, db.h_cu, db.B, db.T, window, stride, labels, z, m,
                                     ws, ws.numel(), stream)
        else:
            n = self.model.workspace_size(db.T, db.B)
            ws = self._buf("ner", n)
            api.ner_forward(self.model, db.ids, db.cu, db.B, db.T, labels, z, m, ws, ws.numel(), stream)
        return labels, z, m

    def autotune(self, T: int, B: int = 1, stream=None):
        """Let the library time the GEMM tiles on T rows and keep the fastest."""
        ws = self._buf("ner", self.model.workspace_size(T, max(B, 1)))
        return self.model.autotune(T, ws, ws.numel(), stream)

    def autotune_attention(self, db: DeviceBatch, stream=None):
        """Let the library time the attention tiles on this batch's lengths and keep the fastest."""
        ws = self._buf("ner", self.model.workspace_size(db.T, db.B))
        return self.model.autotune_attention(db.cu, db.B, db.T, ws, ws.numel(), stream)

    def hidden(self, db: DeviceBatch, n_layers: int, stream=None) -> torch.Tensor:
        out = torch.empty((max(db.T, 1), self.model.cfg.hidden), dtype=torch.float32, device=self.device)
        ws = self._buf("ner", self.model.workspace_size(db.T, db.B))
        api.encoder_hidden(self.model, db.ids, db.cu, db.B, db.T, n_layers, out, ws, ws.numel(), stream)
        return out

    def spans(self, db: DeviceBatch, labels: torch.Tensor, span_cap: int | None = None, stream=None):
        cap = db.T if span_cap is None else span_cap
        spans = torch.empty((max(cap, 1), 3), dtype=torch.int64, device=self.device)
        cu_spans = torch.empty(db.B + 1, dtype=torch.int32, device=self.device)
        ws = self._buf("dec", api.decode_workspace_size(db.T, db.B))
        api.decode_spans(labels, db.tok_off, db.cu, db.B, db.T, self.n_types, spans, cap, cu_spans, ws, ws.numel(),
                         stream)
        return spans, cu_spans, cap

    def recognize(self, db: DeviceBatch, ner_spans=None, ner_cu=None, ner_cap: int = 0, span_cap: int | None = None,
                  stream=None):
        """Recognizer candidates merged with the NER spans (if given) into whole-entity spans.

        The unions are disjoint and each holds an NER span or a recognizer
        match of at least 5 bytes, so ner_cap + n_bytes / 5 + 1 of them always
        fit."""
        cap = (ner_cap + db.n_bytes // 5 + 1) if span_cap is None else span_cap
        spans = torch.empty((max(cap, 1), 3), dtype=torch.int64, device=self.device)
        cu_spans = torch.empty(db.B + 1, dtype=torch.int32, device=self.device)
        ws = self._buf("rx", api.recognize_workspace_size(db.n_bytes, db.B))
        rt = api.recognizer_types(self.cache.type_names)
        api.recognize_spans(db.text, db.cu_bytes, db.B, db.n_bytes, rt, self.n_types, ner_spans, ner_cu, ner_cap,
                            spans, cap, cu_spans, ws, ws.numel(), stream)
        return spans, cu_spans, cap

    def fields(self, db: DeviceBatch, config: dict, span_cap: int | None = None, stream=None):
        """Whole-field spans of the configured ``Field: value`` lines, without NER
        (config: field name -> type index).  A field needs at least 4 bytes
        ("x: v" and a line break), so n_bytes / 4 + 1 spans always fit."""
        cap = (db.n_bytes // 4 + 1) if span_cap is None else span_cap
        spans = torch.empty((max(cap, 1), 3), dtype=torch.int64, device=self.device)
        cu_spans = torch.empty(db.B + 1, dtype=torch.int32, device=self.device)
        ws = self._buf("fd", api.field_workspace_size(db.n_bytes, db.B))
        api.field_spans(db.text, db.cu_bytes, db.B, db.n_bytes, config, self.n_types, spans, cap, cu_spans, ws,
                        ws.numel(), stream)
        return spans, cu_spans, cap

    def step_fields(self, db: DeviceBatch, config: dict, stream=None):
        """The schema-configured path: whole-field spans, then substitution (no NER)."""
        spans, cu_spans, cap = self.fields(db, config, stream=stream)
        out, cu_out = self.pseudonymize(db, spans, cu_spans, cap, stream=stream)
        return spans, cu_spans, out, cu_out

    def out_capacity(self, db: DeviceBatch, span_cap: int) -> int:
        longest = max(len(n) for n in self.cache.type_names)
        return db.n_bytes + span_cap * (2 + longest + 1 + self.cache.slug) + 1

    def pseudonymize(self, db: DeviceBatch, spans: torch.Tensor, cu_spans: torch.Tensor, span_cap: int,
                     out_cap: int | None = None, stream=None):
        cap = self.out_capacity(db, span_cap) if out_cap is None else out_cap
        out = self._buf("out", cap)
        cu_out = torch.empty(db.B + 1, dtype=torch.int64, device=self.device)
        ws = self._buf("ps", api.pseudonymize_workspace_size(db.B, span_cap))
        api.pseudonymize(self.cache, db.text, db.cu_bytes, db.B, spans, cu_spans, span_cap, out, cap, cu_out, ws,
                         ws.numel(), stream)
        return out, cu_out

    def step(self, db: DeviceBatch, window: int = 0, stride: int = 0, recognizers: bool = False, stream=None):
        """One pass of the whole path over a resident batch (all on one stream);
        with recognizers, the NER spans are merged with the pattern recognizers'
        before substitution."""
        labels, _, _ = self.ner(db, logits=False, margin=False, window=window, stride=stride, stream=stream)
        spans, cu_spans, cap = self.spans(db, labels, stream=stream)
        if recognizers:
            spans, cu_spans, cap = self.recognize(db, spans, cu_spans, cap, stream=stream)
        out, cu_out = self.pseudonymize(db, spans, cu_spans, cap, stream=stream)
        return labels, spans, cu_spans, out, cu_out


def outputs_to_list(out: torch.Tensor, cu_out: torch.Tensor) -> list[bytes]:
    cu = cu_out.cpu().numpy()
    data = out[: int(cu[-1])].cpu().numpy().tobytes()
    return [data[int(cu[i]):int(cu[i + 1])] for i in range(len(cu) - 1)]
