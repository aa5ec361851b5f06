"""Model shapes and workload recipes used by the tests and the benchmark.

The paper names its NER models (Sec. II, stage 2) but gives no architecture and
no trained weights; the encoder shapes below are the ones the build is measured
on, with synthetic N(0, 0.02) weights.  Each workload states the record count
and the token-length distribution of its synthetic scan-report records.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class ModelConfig:
    n_layers: int
    hidden: int
    n_heads: int
    ffn: int
    vocab: int
    n_labels: int
    max_pos: int = 512
    ln_eps: float = 1e-5

    @property
    def head_dim(self) -> int:
        return self.hidden // self.n_heads

    @property
    def n_types(self) -> int:
        return (self.n_labels - 1) // 2


@dataclass(frozen=True)
class ModernConfig:
    """A ModernBERT-style encoder: pre-LayerNorm layers without biases,
    rotary position embeddings, global attention every ``global_every``
    layers (from layer 0) and a sliding window elsewhere (a token sees keys at
    most ``local_window // 2`` positions away), a gated GELU MLP
    (``intermediate`` wide), a final LayerNorm and a dense + GELU + LayerNorm
    head before the token classifier."""
    n_layers: int
    hidden: int
    n_heads: int
    intermediate: int
    vocab: int
    n_labels: int
    max_pos: int = 8192
    ln_eps: float = 1e-5
    local_window: int = 128
    global_every: int = 3
    theta_global: float = 160000.0
    theta_local: float = 10000.0

    @property
    def head_dim(self) -> int:
        return self.hidden // self.n_heads

    @property
    def n_types(self) -> int:
        return (self.n_labels - 1) // 2

    def is_global(self, layer: int) -> bool:
        return layer % self.global_every == 0


TINY = ModelConfig(n_layers=2, hidden=128, n_heads=2, ffn=512, vocab=8192, n_labels=9)
BASE = ModelConfig(n_layers=12, hidden=768, n_heads=12, ffn=3072, vocab=30522, n_labels=17)
LARGE = ModelConfig(n_layers=24, hidden=1024, n_heads=16, ffn=4096, vocab=30522, n_labels=17)
# ModernBERT-base shapes (22 layers, h768, 12 heads, GeGLU 1152, vocab 50368)
# and a small one for the parity cases
MODERN_BASE = ModernConfig(n_layers=22, hidden=768, n_heads=12, intermediate=1152, vocab=50368, n_labels=17)
MODERN_TINY = ModernConfig(n_layers=4, hidden=128, n_heads=2, intermediate=192, vocab=5000, n_labels=9,
                           max_pos=1024)


@dataclass(frozen=True)
class Workload:
    name: str
    model: ModelConfig
    n_records: int
    # ("uniform", lo, hi) or ("lognormal", mu, sigma, lo, hi): tokens per record
    lengths: tuple
    precision: str
    seed: int = 0
    weight_seed: int = 0
    # bias added to the O logit so that roughly 92% of tokens predict O
    # (None: a plain random head)
    o_target: float | None = 0.92
    zipf_pool: int = 0          # distinct entities in the Zipf pool (0: fresh entities)
    zipf_s: float = 1.1
    window: int = 0             # 0: no windowing, else window length in tokens
    stride: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "tiny_fp32": Workload(
        "tiny_fp32", TINY, 64, ("uniform", 16, 128), "fp32", o_target=None,
        notes="2-layer post-LN encoder h128, 64 records of 16..128 tokens"),
    "base_bf16": Workload(
        "base_bf16", BASE, 4096, ("lognormal", 5.2, 0.6, 16, 512), "bf16",
        notes="12-layer h768 encoder, 4096 packed varlen records"),
    "base_fp32": Workload(
        "base_fp32", BASE, 4096, ("lognormal", 5.2, 0.6, 16, 512), "fp32",
        notes="same workload as base_bf16 on the plain FP32 path"),
    "stream_bf16": Workload(
        "stream_bf16", BASE, 70951, ("lognormal", 7.04, 0.6, 16, 16384), "bf16",
        zipf_pool=200_000, window=512, stride=448,
        notes="dataset-scale records windowed at 512 tokens with 64-token overlap"),
    "tiny_fp8": Workload(
        "tiny_fp8", TINY, 64, ("uniform", 16, 128), "fp8", o_target=None,
        notes="the tiny encoder with FP8-E4M3 GEMMs (parity cases)"),
    "large_bf16": Workload(
        "large_bf16", LARGE, 16384, ("lognormal", 5.5, 0.7, 16, 512), "bf16",
        notes="the 24-layer h1024 workload in BF16 (comparison for FP8)"),
    "large_fp8": Workload(
        "large_fp8", LARGE, 16384, ("lognormal", 5.5, 0.7, 16, 512), "fp8",
        notes="24-layer h1024 encoder with FP8-E4M3 GEMMs"),
    "modern_bf16": Workload(
        "modern_bf16", MODERN_BASE, 4096, ("lognormal", 5.2, 0.6, 16, 512), "bf16",
        notes="ModernBERT-style encoder (22 layers, h768, RoPE, local/global attention, GeGLU) on the base "
              "workload's 4096 records"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
