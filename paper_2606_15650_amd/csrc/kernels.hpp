// Host-side launchers of the gfx950 kernels (one translation unit each).
#pragma once

#include "common.hpp"

namespace anon {

// ---- GEMM: C[M,N] = A[M,K] * W[N,K]^T with a fused epilogue --------------
// EPI_ROPE: bias, rotary rotation of the pairs (c, c+32) of each 64-column
// head block below rope_cols by the row's position, Q scaling.  EPI_GEGLU:
// GELU(u) * g of the interleaved 32-column blocks u, g (output N/2 wide).
enum GemmEpi { EPI_BIAS = 0, EPI_GELU = 1, EPI_RESID = 2, EPI_ROPE = 3, EPI_GEGLU = 4 };
enum ElemType { ET_F32 = 0, ET_BF16 = 1, ET_FP8 = 2 };

struct GemmParams {
  const void* A;      // [M, K] row-major, element type `in`
  const void* W;      // [N, K] row-major (transposed weights), element type `in`
  const float* bias;  // [N]
  const void* resid;  // [M, N] (EPI_RESID), element type `res`
  void* C;            // [M, N], element type `out`
  int M, N, K;
  float qscale;       // EPI_BIAS: columns n < qcols are multiplied by qscale
  int qcols;
  float acc_scale;    // multiplies the accumulator (FP8: sa * sw), else 1
  float out_inv_scale;  // FP8 output: value / scale before rounding
  ElemType in, out, res;
  GemmEpi epi;
  int config;         // tile configuration index (-1: default choice)
  int group_m;        // row blocks per tile group (0: chosen by shape; 1: row-major)
  int ldc;            // output row stride (0: N, or N/2 for EPI_GEGLU)
  const int* pos;     // EPI_ROPE: [M] position of each row within its record
  const float* rope;  // EPI_ROPE: [positions][64] cos (first 32), sin (last 32)
  int rope_cols;      // EPI_ROPE: columns below this are rotated
  const int* m_dev;   // non-null: rows to compute, read on the device (M is then the grid's capacity)
};
// Returns false (and sets the error) if no kernel matches the shapes/types.
bool launch_gemm(const GemmParams& p, hipStream_t s);
int default_gemm_config(const GemmParams& p);
int gemm_num_configs(ElemType in);
const char* gemm_config_name(ElemType in, int config);
bool gemm_config_fits(ElemType in, int config, int N, int K);
// the configuration divides the shape and, for the paired epilogues, gives
// each wave whole 64-column blocks
bool gemm_config_serves(const GemmParams& p, int config);

// ---- attention ------------------------------------------------------------
// Work list of the attention kernel (validates cu_seqlens on the device).
// `config` picks the BF16 kernel's tile configuration (attn_num_configs();
// -1: default); the FP32 kernel has one.  `items` holds attn_plan_items()
// entries; `n_items` (one int, device) receives their count.
int attn_num_configs();
const char* attn_config_name(int config);
int attn_plan_items(ElemType t, int config, int T, int B);
// t_dev (nullable): the token total in device memory, at most T; cu_seqlens[B]
// must equal it.
void launch_attn_plan(const int* cu_seqlens, int B, int T, int max_len, ElemType t, int config, int4* items,
                      int max_items, int* n_items, uint32_t* err, hipStream_t s, const int* t_dev = nullptr);
// window > 0: query i sees only keys j with |i - j| <= window
void launch_attention(const void* qkv, void* out, const int4* items, int max_items, const int* n_items,
                      int n_heads, int hidden, ElemType t, ElemType out_t, float out_inv_scale, int config,
                      hipStream_t s, int window = 0);

// ---- row-wise kernels -----------------------------------------------------
// pos_emb may be null (no learned positions); pos_out (nullable) receives
// each token's position within its record.  The row kernels take T (rows)
// as the capacity their grid covers; a non-null t_dev (rows_dev) holds the
// count to compute, read on the device (see live_rows).
void launch_embed_ln(const int* ids, const int* cu_seqlens, int B, int T, const float* tok_emb, const float* pos_emb,
                     const float* g, const float* b, float eps, int vocab, int max_pos, int h, void* out,
                     ElemType out_t, fp8_t* out_q, float q_inv_scale, uint32_t* err, hipStream_t s,
                     int* pos_out = nullptr, const int* t_dev = nullptr);
void launch_f32_to_bf16(const float* x, bf16_t* out, int64_t n, hipStream_t s);
void launch_layernorm(const void* y, ElemType y_t, const float* g, const float* b, float eps, int rows, int h,
                      void* out, ElemType out_t, fp8_t* out_q, float q_inv_scale, hipStream_t s,
                      const int* rows_dev = nullptr);
void launch_classifier(const void* x, ElemType x_t, const float* wc_t, const float* bc, int T, int h, int C,
                       uint8_t* labels, float* logits, float* margin, hipStream_t s,
                       const int* t_dev = nullptr);
void launch_to_f32(const void* x, ElemType t, float* out, int64_t n, hipStream_t s);
void launch_transpose_convert(const float* src, int rows, int cols, void* dst, ElemType t, float inv_scale,
                              hipStream_t s);

// ---- windows --------------------------------------------------------------
void launch_window_gather(const int* ids, const int* cu_seqlens, const int4* windows, int n_windows,
                          int* w_ids, hipStream_t s);
void launch_window_merge(const int* cu_seqlens, int B, const int* rec_win0, const int4* windows, int window,
                         int stride, const uint8_t* w_labels, const float* w_logits, const float* w_margin, int C,
                         uint8_t* labels, float* logits, float* margin, int T, hipStream_t s);

// ---- scans ----------------------------------------------------------------
size_t scan_temp_bytes(int64_t n);
// out[i] = sum_{j<i} in[i], i in [0, n]; out has n+1 entries.
void launch_exclusive_scan_i32(const int* in, int* out, int64_t n, void* temp, hipStream_t s);
void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t s);

// ---- spans ----------------------------------------------------------------
void launch_bio_flags(const uint8_t* labels, const int* cu_seqlens, int B, int T, int n_types, int* flags,
                      uint32_t* err, hipStream_t s);
void launch_bio_write(const uint8_t* labels, const int* tok_off, const int* cu_seqlens, int B, int T, int n_types,
                      const int* flags, const int* excl, anon_span* spans, int span_cap, int* cu_spans,
                      uint32_t* err, hipStream_t s);

// ---- pseudonyms -----------------------------------------------------------
struct PcacheDev {
  uint8_t* table;         // capacity entries
  uint64_t mask;          // capacity - 1
  uint32_t ipad[8], opad[8];  // SHA-256 states after the key blocks
  int slug;
  int n_types;
  const uint8_t* names;   // concatenated type names
  const int* name_off;    // [n_types + 1]
  unsigned long long* counters;  // [0] lookups, [1] hits, [2] inserts
  int enabled;
  uint32_t preserve[4];   // bit t: spans of type t are left as they are
  uint32_t call;          // number of this pseudonymize call on the cache (1-based)
};
// Host view of the table entries (anon_pcache_export).
struct PcacheEntryView {
  uint32_t state, len;
  uint64_t fp;
  uint8_t bytes[96];
  uint32_t digest[8];
  int32_t type;
  uint32_t first, last, pad;
};
size_t pcache_entry_bytes();
bool hmac_selftest();
void sha256_hmac_midstates(const uint8_t* key, size_t key_len, uint32_t ipad[8], uint32_t opad[8]);
void launch_ps_layout(const PcacheDev& pc, const int64_t* cu_bytes, int B, const anon_span* spans,
                      const int* cu_spans, int span_cap, int64_t* out_len, int64_t* sp_out, int* sp_plen,
                      int64_t* sp_in_end, uint32_t* err, hipStream_t s);
void launch_ps_hash(const PcacheDev& pc, const uint8_t* text, const int64_t* cu_bytes, int B, const anon_span* spans,
                    const int* cu_spans, int span_cap, const int* sp_plen, uint8_t* digests, hipStream_t s);
void launch_ps_write(const PcacheDev& pc, const uint8_t* text, const int64_t* cu_bytes, int B,
                     const anon_span* spans, const int* cu_spans, int span_cap, const int64_t* sp_out,
                     const int* sp_plen, const int64_t* sp_in_end, const uint8_t* digests, const int64_t* cu_out,
                     uint8_t* out, int64_t out_cap, uint32_t* err, hipStream_t s);
void launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
// n elements of type t, uniform in [-1, 1) (benchmark and tuning operands)
void launch_fill_random(void* p, ElemType t, int64_t n, uint32_t seed, hipStream_t s);

// ---- pattern recognizers and overlap resolution ---------------------------
struct RecogBuffers {
  int *delta, *starts, *cover, *fstart, *fend, *sstart, *send;
  unsigned long long *key, *run_key;
  uint8_t* ner_type;
  int64_t *run_begin, *run_end;
  void* temp;
};
RecogBuffers recog_layout(int64_t n_bytes, Carver& k);
size_t recog_workspace_bytes(int64_t n_bytes);
// rec_types: type index of each of the 9 recognizers (0 = off).  ner/ner_cu
// may be null (no NER spans).
constexpr int kNumRecognizers = 9;  // URL, e-mail, IPv4, MAC, hash, CVE, hostname, IPv6, CPE
void launch_recognize(const uint8_t* text, const int64_t* cu_bytes, int B, int64_t n_bytes,
                      const int rec_types[kNumRecognizers],
                      const anon_span* ner, const int* ner_cu, int ner_cap, int n_types, const RecogBuffers& w,
                      anon_span* out, int cap, int* cu_spans, uint32_t* err, hipStream_t s);

// ---- schema-aware whole-field spans ----------------------------------------
constexpr int kFieldNameMax = 32;
constexpr int kFieldsMax = 64;
struct FieldTable {  // passed by value to the kernels
  uint8_t name[kFieldsMax][kFieldNameMax];
  uint8_t len[kFieldsMax];
  int type[kFieldsMax];
  int n;
};
struct FieldBuffers {
  uint8_t* rs;
  int *flags, *excl;
  void* temp;
};
FieldBuffers field_layout(int64_t n_bytes, Carver& k);
size_t field_workspace_bytes(int64_t n_bytes);
void launch_field_spans(const uint8_t* text, const int64_t* cu_bytes, int B, int64_t n_bytes, const FieldTable& ft,
                        const FieldBuffers& w, anon_span* out, int cap, int* cu_spans, uint32_t* err,
                        hipStream_t s);

// Shape of a created model (the struct itself is private to the runtime).
const anon_model_config* model_config(const anon_model* m);

}  // namespace anon
