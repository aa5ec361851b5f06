"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generation only: scan-report-like records, the
tokenizer that turns them into token ids with byte offsets, gold BIO labels,
synthetic encoder weights and the HMAC key.  It contains none of the method's
arithmetic (no encoder math, no span decoding, no hashing of entities), so the
oracle and the GPU path can both consume it without sharing any computation.
"""
from .configs import ModelConfig, ModernConfig, WORKLOADS, workload
from .tokenizer import tokenize, fnv1a32
from .records import RecordBatch, generate_records, TYPE_NAMES_17, TYPE_NAMES_9
from .weights import make_weights, tensor_specs, weights_blob, make_key

__all__ = [
    "ModelConfig", "ModernConfig", "WORKLOADS", "workload", "tokenize", "fnv1a32",
    "RecordBatch", "generate_records", "TYPE_NAMES_17", "TYPE_NAMES_9",
    "make_weights", "tensor_specs", "weights_blob", "make_key",
]
