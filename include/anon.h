/*
 * anon.h - C ABI of libanon.so, the MI355X (gfx950) NER + pseudonymize path.
 *
 * The library implements the data-parallel middle of the paper's pipeline
 * (Sec. II): stage 2, token-classification NER with a transformer encoder,
 * and stage 3, deterministic HMAC-SHA256 pseudonym substitution written as
 * [TYPE_slug].  Everything between the packed token ids and the substituted
 * bytes runs in HIP kernels on one GPU.
 *
 * Conventions
 *   - Pointers named d_* are device memory owned by the caller.  Pointers
 *     named h_* are host memory owned by the caller.  Opaque handles
 *     (anon_model, anon_pcache, anon_server) are owned by the library.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream only enqueue work and return; results are
 *     valid once the stream has been synchronised.
 *   - Argument errors are reported synchronously with a negative status;
 *     anon_last_error() then describes the problem (thread-local string).
 *   - Problems found in device data (token id outside the vocabulary,
 *     malformed cu_seqlens, labels outside [0, 2*n_types], malformed spans,
 *     exceeded capacities) never cause an out-of-bounds access: the kernels
 *     clamp or skip and raise a bit in the per-device error word read by
 *     anon_device_errors().
 *   - Packed varlen layout: B records, T tokens in total, record b owns
 *     tokens [cu_seqlens[b], cu_seqlens[b+1]); cu_seqlens[0] = 0,
 *     cu_seqlens[B] = T, no padding.
 */
#ifndef ANON_H
#define ANON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ANON_OK = 0,
  ANON_PENDING = 1,     /* anon_poll: request not finished yet            */
  ANON_EINVAL = -1,     /* invalid argument                               */
  ANON_ENOMEM = -2,     /* device or host allocation failed               */
  ANON_EDEVICE = -3,    /* HIP runtime error                              */
  ANON_ECAPACITY = -4,  /* a caller-provided buffer is too small          */
  ANON_EBUSY = -5,      /* server queue full / budget exhausted           */
  ANON_ENOTFOUND = -6,  /* unknown ticket                                 */
  ANON_EDATA = -7       /* malformed device data (see anon_device_errors) */
} anon_status;

typedef enum { ANON_FP32 = 0, ANON_BF16 = 1, ANON_FP8_E4M3 = 2 } anon_precision;

/* Bits of the per-device error word. */
enum {
  ANON_ERR_TOKEN_ID = 1,      /* token id >= vocab or < 0 (embedding row 0 used)   */
  ANON_ERR_SEQLENS = 2,       /* cu_seqlens not monotone / record longer than max_pos */
  ANON_ERR_LABEL = 4,         /* label > 2*n_types (token treated as O)             */
  ANON_ERR_SPAN = 8,          /* span outside its record / overlapping (skipped)     */
  ANON_ERR_SPAN_CAP = 16,     /* more spans than span_cap (extra spans dropped)      */
  ANON_ERR_OUT_CAP = 32,      /* output larger than out_cap (output truncated)       */
  ANON_ERR_TEXT = 64          /* cu_bytes malformed (recognize_spans, field_spans) or a record of >= 16 MiB (recognize_spans) */
};

/* Encoder shape.  head_dim = hidden / n_heads must be 64; n_labels = 2*types+1. */
typedef struct {
  int32_t n_layers, hidden, n_heads, ffn, vocab, n_labels, max_pos;
  float ln_eps;
} anon_model_config;

/* One entity span: bytes [begin, end) of record `record`, type in 1..n_types. */
typedef struct {
  int32_t record;
  int32_t type;
  int64_t begin;
  int64_t end;
} anon_span;

typedef struct anon_model anon_model;
typedef struct anon_pcache anon_pcache;
typedef struct anon_server anon_server;

/* Last error message of the calling thread ("" if none). */
const char* anon_last_error(void);

/* Library ABI version (increments on incompatible changes). */
int32_t anon_version(void);

/* Read (and if `clear`, reset) the error word of `device`.  Synchronises
 * the device. */
anon_status anon_device_errors(int32_t device, uint32_t* flags, int32_t clear);

/* ------------------------------------------------------------------------
 * Model (Sec. II stage 2: transformer token-classification NER)
 * ------------------------------------------------------------------------
 * anon_model_create uploads an encoder to `device`.
 *   h_weights: n_floats FP32 values, the tensors back to back in this order
 *     (matrices in "x @ W" orientation, i.e. [in, out], row-major):
 *       tok_emb [vocab,h], pos_emb [max_pos,h], emb_ln_g [h], emb_ln_b [h],
 *       per layer: wqkv [h,3h], bqkv [3h], wo [h,h], bo [h], ln1_g [h],
 *                  ln1_b [h], w1 [h,ffn], b1 [ffn], w2 [ffn,h], b2 [h],
 *                  ln2_g [h], ln2_b [h],
 *       wc [h,n_labels], bc [n_labels].
 *     Columns of wqkv are [Q | K | V]; head j owns columns j*64..j*64+63 of
 *     each block.  The host array is only read during the call.
 *   precision: FP32 (plain path), BF16, or FP8_E4M3 GEMMs.
 *   h_act_scales: FP8 only: 4*n_layers static per-tensor scales of the GEMM
 *     inputs (qkv, attention-out, ffn1, ffn2 per layer), each a power of two;
 *     NULL otherwise.
 * The returned model is used from one host thread at a time.
 */
anon_status anon_model_create(const anon_model_config* cfg, const float* h_weights, size_t n_floats,
                              anon_precision precision, const float* h_act_scales, int32_t device,
                              anon_model** out);
void anon_model_free(anon_model* model);

/* Versioned weights file.  Layout (little-endian): a 64-byte header --
 * "ANONWTS1", uint32 format version (1), uint32 kind (0: this BERT-style
 * encoder), anon_model_config (32 bytes), uint64 float count, uint64
 * FNV-1a-64 hash of the float bytes -- then the FP32 weights in
 * anon_model_create's order.
 *   anon_weights_write: writes `h_weights` (n_floats, checked against the
 *     config) to `path`; ANON_EINVAL if the file cannot be written.
 *   anon_weights_info: reads and checks a file (magic, version, kind,
 *     config, float count, file size, hash) without touching a device; the
 *     config and float count are returned through the non-NULL pointers.
 *   anon_model_load: anon_weights_info's checks, then anon_model_create with
 *     the file's config and weights.
 * A malformed, truncated or corrupt file is ANON_EINVAL (the message says
 * which check failed); the file is only read during the call. */
anon_status anon_weights_write(const char* path, const anon_model_config* cfg, const float* h_weights,
                               size_t n_floats);
anon_status anon_weights_info(const char* path, anon_model_config* cfg, size_t* n_floats);
anon_status anon_model_load(const char* path, anon_precision precision, const float* h_act_scales, int32_t device,
                            anon_model** out);

/* Device workspace bytes that ner_forward needs for a batch of T tokens in
 * B records (an upper bound, valid for any batch with at most T tokens and B
 * records). */
anon_status anon_ner_workspace_size(const anon_model* model, int32_t T, int32_t B, size_t* bytes);

/* NER forward pass over a packed batch (Sec. II stage 2).
 *   d_ids        int32 [T]   token ids in [0, vocab)
 *   d_cu_seqlens int32 [B+1] record boundaries; each record <= max_pos tokens
 *   d_labels     uint8 [T]   out: argmax label per token (lowest index on ties)
 *   d_logits     float [T, n_labels] out, or NULL
 *   d_margin     float [T]   out: top-1 minus top-2 logit, or NULL
 *   d_workspace  >= anon_ner_workspace_size(T, B) bytes, 256-byte aligned
 * Positions restart at 0 for every record; attention never crosses records.
 * Results do not depend on the other records of the batch. */
anon_status ner_forward(anon_model* model, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                        int32_t T, uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                        size_t ws_bytes, void* stream);

/* The NER forward pass (Sec. II stage 2) recorded as one HIP graph.
 * ner_forward_capture records ner_forward with exactly these arguments (same
 * meaning, layout and checks as ner_forward) on a private stream and
 * instantiates the result; nothing is computed by the call itself.
 * anon_graph_launch then runs the whole layer stack and the classifier on
 * `stream` as one launch.  The graph holds the device pointers, B, T and the
 * model's tile configuration as they were at capture: between launches the
 * caller may rewrite the contents of d_ids and d_cu_seqlens (a new batch of
 * exactly B records and T tokens), and every launch gives the same results
 * as ner_forward on the buffers' contents at that time.  The model, the
 * workspace and the buffers must outlive the graph; launches that overlap
 * share the workspace and race.  Kernel timing (anon_prof_enable) must be
 * off during the capture (ANON_EINVAL otherwise); T == 0 is ANON_EINVAL. */
typedef struct anon_graph anon_graph;
anon_status ner_forward_capture(anon_model* model, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                                int32_t T, uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                                size_t ws_bytes, anon_graph** out);
/* The same graph for a token bucket: any batch of at most B_cap records and
 * T_cap tokens.  Every kernel of the graph reads the batch's token count
 * from d_n_tokens (int32, device) when it runs; its grid covers T_cap rows
 * and the rows at or past the count are neither computed nor written.  To
 * run a batch of B <= B_cap records and T <= T_cap tokens, write its ids to
 * d_ids[0 .. T), its boundaries to d_cu_seqlens[0 .. B] and
 * d_cu_seqlens[b] = T for b in (B, B_cap] (empty records), T to
 * *d_n_tokens, then launch; labels, logits and margins of tokens 0 .. T-1
 * equal ner_forward's on that batch bit for bit.  A count outside
 * [0, T_cap] or a d_cu_seqlens[B_cap] that differs from it raises the
 * sequence-length bit of the device error word (the count is clamped, the
 * outputs are then unspecified).  d_workspace >=
 * anon_ner_workspace_size(T_cap, B_cap) bytes; ownership and races as for
 * ner_forward_capture.  Serving replays one such graph per bucket
 * (anon_server_config.graph_buckets). */
anon_status ner_forward_capture_bucket(anon_model* model, const int32_t* d_ids, const int32_t* d_cu_seqlens,
                                       const int32_t* d_n_tokens, int32_t B_cap, int32_t T_cap, uint8_t* d_labels,
                                       float* d_logits, float* d_margin, void* d_workspace, size_t ws_bytes,
                                       anon_graph** out);
anon_status anon_graph_launch(anon_graph* graph, void* stream);
void anon_graph_free(anon_graph* graph);

/* GEMM tile autotuner.  Times every tile configuration that fits each of the
 * four encoder GEMMs (0 QKV, 1 output projection, 2 FFN1, 3 FFN2) on T rows,
 * using d_workspace (>= anon_ner_workspace_size(T, 1) bytes; overwritten) as
 * operand memory, and keeps the fastest for this model's later calls; then,
 * with that tile, it times the tile orders (groups of 2, 4, 6, 8 or 12 row
 * blocks against the order by shape, see anon_model_set_tile_groups) and
 * keeps one that is at least 1% faster than the order by shape.  All
 * configurations and orders of a precision form every output element with
 * the same MFMA sequence in the same K order, so tuning never changes
 * results.
 *   chosen:   [4] picked configuration per GEMM, or NULL
 *   times_ms: [4 * max_configs] mean time per configuration (-1: does not
 *             fit the shape), or NULL
 * Synchronises the stream. */
anon_status anon_autotune(anon_model* model, int32_t T, void* d_workspace, size_t ws_bytes, void* stream,
                          int32_t* chosen, float* times_ms, int32_t max_configs);
/* Set the tile configuration of each encoder GEMM (-1 = built-in default). */
anon_status anon_model_set_tiles(anon_model* model, const int32_t tiles[4]);
/* Set the tile order of each encoder GEMM: output tiles are visited in
 * groups of groups[i] row blocks, column block by column block (1 = plain
 * row-major order; 0 = by shape, the default: 8 when a row block spans 8 or
 * more column blocks, else 1).  Only the order in which workgroups take
 * tiles changes (L2 reuse of the weight panels), never a result.  Range
 * [0, 1024]. */
anon_status anon_model_set_tile_groups(anon_model* model, const int32_t groups[4]);
/* Current tile configuration and tile group of each encoder GEMM (either
 * pointer may be NULL). */
anon_status anon_model_get_tiles(const anon_model* model, int32_t tiles[4], int32_t groups[4]);
/* Number of tile configurations of a precision and the name of one. */
int32_t anon_tile_config_count(anon_precision precision);
const char* anon_tile_config_name(anon_precision precision, int32_t config);

/* ------------------------------------------------------------------------
 * ModernBERT-style encoder (the paper's SecureModernBERT-NER model of Sec. II
 * stage 2, used for its accuracy run, Sec. IV-B): pre-LayerNorm layers with
 * no biases (LayerNorms without shift), rotary position embeddings (base
 * theta_global on layers 0, global_every, 2*global_every, ..., theta_local
 * elsewhere), full attention on those global layers and a sliding window on
 * the others (a token sees the keys at most local_window/2 positions away),
 * a gated MLP (x += (GELU(u) * g) Wo2 with [u | g] = LN(x) Wi), a final
 * LayerNorm, a dense + GELU + LayerNorm head and the token classifier.  The
 * residual stream is kept in FP32; FP32 or BF16 GEMM operands.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_layers, hidden, n_heads, intermediate, vocab, n_labels, max_pos;
  float ln_eps;
  int32_t local_window; /* total window width; a token sees local_window/2 keys on each side */
  int32_t global_every;
  float theta_global, theta_local;
} anon_modern_config;
typedef struct anon_modern anon_modern;

/* h_weights: host FP32 tensors back to back, matrices in x @ W orientation
 * ([in][out]):  tok_emb [vocab][h], emb_ln_g [h]; per layer l:
 * (l > 0) attn_ln_g [h], wqkv [h][3h] (columns Q | K | V, head j owns
 * columns 64j .. 64j+63 of each), wo [h][h], mlp_ln_g [h], wi [h][2I]
 * (columns: the input half u, then the gate half g), wo2 [I][h]; then
 * final_ln_g [h], head_w [h][h], head_ln_g [h], wc [h][C], bc [C].  Copied
 * before return.  Head dimension 64; h = 64 * {1,2,4,8,12,16}; I a multiple
 * of 32; at most 32 labels.  precision: ANON_FP32 or ANON_BF16. */
anon_status anon_modern_create(const anon_modern_config* cfg, const float* h_weights, size_t n_floats,
                               anon_precision precision, int32_t device, anon_modern** out);
void anon_modern_free(anon_modern* model);
anon_status anon_modern_workspace_size(const anon_modern* model, int32_t T, int32_t B, size_t* bytes);
/* As ner_forward, for the ModernBERT-style encoder (positions restart in
 * every record; a record may be up to max_pos tokens long). */
anon_status modern_ner_forward(anon_modern* model, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                               int32_t T, uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                               size_t ws_bytes, void* stream);
/* The FP32 residual stream after the first n_layers layers (0 = after the
 * embedding LayerNorm), [T, hidden], for layer-by-layer checking. */
anon_status anon_modern_hidden(anon_modern* model, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                               int32_t T, int32_t n_layers, float* d_hidden, void* d_workspace, size_t ws_bytes,
                               void* stream);
/* Tile configurations of the five GEMMs (QKV, output projection, gated MLP
 * input, MLP output, head; -1 = default, names as anon_tile_config_name) and
 * of the attention (-1 = default, names as anon_attn_config_name). */
anon_status anon_modern_set_tiles(anon_modern* model, const int32_t tiles[5], int32_t attn_config);
anon_status anon_modern_get_tiles(const anon_modern* model, int32_t tiles[5], int32_t* attn_config);

/* Attention tile autotuner: times every attention tile configuration of a
 * BF16/FP8 model (query rows per work item, keys per LDS tile, ring stages)
 * (and, for BF16 outputs, the form of the output stores: 16-byte stores
 * after a half-wave exchange or 8-byte stores of the accumulator quads)
 * on the given packed batch's record lengths (random Q, K, V of T rows in
 * the workspace, which must hold anon_ner_workspace_size(T, B) bytes) and
 * keeps the fastest for later calls.  Every configuration gives the same
 * bits (each query row sees the same keys in the same order), so the choice
 * only changes speed.  chosen: out (may be NULL); times_ms: out, mean time
 * of each configuration, max_configs entries (may be NULL).  FP32 models
 * have one attention kernel: ANON_OK, nothing timed.  Synchronises the
 * stream. */
anon_status anon_autotune_attention(anon_model* model, const int32_t* d_cu_seqlens, int32_t B, int32_t T,
                                    void* d_workspace, size_t ws_bytes, void* stream, int32_t* chosen,
                                    float* times_ms, int32_t max_configs);
/* Set (-1 = default) or read the attention tile configuration; the number
 * of configurations and the name of one. */
anon_status anon_model_set_attn_config(anon_model* model, int32_t config);
int32_t anon_model_get_attn_config(const anon_model* model);
int32_t anon_attn_config_count(void);
const char* anon_attn_config_name(int32_t config);

/* Hidden state after the first n_layers layers (0 = after the embedding
 * LayerNorm) as FP32 [T, hidden] in d_hidden: the activations ner_forward
 * computes, exposed for layer-by-layer checking.  Same workspace rule. */
anon_status anon_encoder_hidden(anon_model* model, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                                int32_t T, int32_t n_layers, float* d_hidden, void* d_workspace, size_t ws_bytes,
                                void* stream);

/* Windowed NER for records longer than one window (the paper names
 * truncation of long inputs as a limitation, Sec. VI).  A record of n tokens
 * is covered by windows of `window` tokens starting every `stride` tokens
 * (the last may be shorter); each token takes its logits from its owner
 * window: in the overlap of windows k and k+1, the first (window-stride)/2
 * tokens belong to k, the rest to k+1.  Positions restart in every window.
 *   h_cu_seqlens: host copy of d_cu_seqlens (used to plan the windows).
 * Outputs are per record token, as in ner_forward. */
anon_status anon_ner_windowed_workspace_size(const anon_model* model, const int32_t* h_cu_seqlens, int32_t B,
                                             int32_t window, int32_t stride, size_t* bytes);
anon_status ner_forward_windowed(anon_model* model, const int32_t* d_ids, const int32_t* d_cu_seqlens,
                                 const int32_t* h_cu_seqlens, int32_t B, int32_t T, int32_t window, int32_t stride,
                                 uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                                 size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * BIO span decoding (labels to entity byte ranges, input of Sec. II stage 3)
 * ------------------------------------------------------------------------
 * Label 0 = O; type t in 1..n_types has B-t = 2t-1, I-t = 2t.  O closes the
 * open span; B-t opens a new one; I-t extends an open span of type t and
 * otherwise opens a new one.  A span covers [begin of its first token, end of
 * its last token).
 *   d_tok_off    int32 [T, 2] byte range of each token inside its record
 *   d_spans      out: up to span_cap spans, record-major, in token order
 *   d_cu_spans   int32 [B+1] out: record b owns spans [cu_spans[b], cu_spans[b+1]);
 *                cu_spans[B] is the total even when it exceeds span_cap.
 *   d_workspace  >= anon_decode_workspace_size(T, B) bytes. */
anon_status anon_decode_workspace_size(int32_t T, int32_t B, size_t* bytes);
anon_status decode_spans(const uint8_t* d_labels, const int32_t* d_tok_off, const int32_t* d_cu_seqlens, int32_t B,
                         int32_t T, int32_t n_types, anon_span* d_spans, int32_t span_cap, int32_t* d_cu_spans,
                         void* d_workspace, size_t ws_bytes, void* stream);

/* decode_spans without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Its flag, offset and scan buffers are a device
 * array of the library of about 8.4 MB, one copy per GPU held until the
 * process ends; nothing is allocated.  T must be at most
 * ANON_NOALLOC_MAX_TOKENS (ANON_ECAPACITY otherwise, before any launch); the
 * other arguments and the outputs are those of decode_spans.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (two streams,
 * two threads) race and must be ordered by the caller. */
#define ANON_NOALLOC_MAX_TOKENS (1 << 20)
anon_status decode_spans_noalloc(const uint8_t* d_labels, const int32_t* d_tok_off, const int32_t* d_cu_seqlens,
                                 int32_t B, int32_t T, int32_t n_types, anon_span* d_spans, int32_t span_cap,
                                 int32_t* d_cu_spans, void* stream);

/* ------------------------------------------------------------------------
 * Pattern recognizers and overlap resolution (Sec. II stage 2 pairs the NER
 * model with regular-expression recognizers; Sec. IV-B and App. D show the cost of
 * overlapping detections that are not merged: truncated entities and extra
 * pseudonyms)
 * ------------------------------------------------------------------------
 * Nine recognizers run over every byte of every record (W = [A-Za-z0-9_],
 * LABEL = [A-Za-z0-9-], LOCAL = [A-Za-z0-9._%+-]), in this order:
 *   0 URL        "http://" or "https://" at a word start, then >= 1 non-space bytes
 *   1 EMAIL      maximal LOCAL run, '@', >= 1 "label." groups, then an all-letter
 *                top label of >= 2 bytes not followed by LABEL (longest domain)
 *   2 IPV4       four dot-separated octets 0..255, no leading zeros, word-bounded
 *   3 MAC        six hex pairs separated by ':', word-bounded
 *   4 HASH       a hex run of exactly 32, 40 or 64 bytes, word-bounded
 *   5 CVE        "CVE-" + 4 digits + '-' + 4..7 digits, word-bounded
 *   6 HOSTNAME   a dotted LABEL run not preceded by LABEL or '.', ending at a label
 *                equal to corp, lan, intra, net, org, local, example or internal
 *                and not followed by LABEL (longest)
 *   7 IPV6       an IPv6 address in an RFC 4291 section 2.2 text form (eight
 *                groups of 1-4 hex digits, one "::" for one or more zero groups,
 *                an optional dotted-quad last 32 bits): the maximal run of hex
 *                digits, ':' and '.' from a hex digit or ':' not preceded by a
 *                word byte, ':' or '.', without its trailing dots, not followed
 *                by a word byte
 *   8 CPE        "cpe:/" + a part in [aho] or "cpe:2.3:" + a part in [aho*-] at a
 *                word start, the part not followed by a component byte
 *                [A-Za-z0-9._~%*?!\-], then the maximal run of component bytes
 *                and ':'
 * Every start byte where a rule matches gives a candidate span.  The NER spans
 * and the candidates that share a byte are merged into their union
 * (transitively; spans that only touch stay apart); the union takes the type
 * of its longest member, then NER before recognizers (in the order above),
 * then the leftmost member.  The output feeds pseudonymize().
 *   d_text, d_cu_bytes  record bytes back to back, int64 offsets [B+1]
 *                       (cu_bytes[0] = 0, cu_bytes[B] = n_bytes, records below
 *                       16 MiB; otherwise ANON_ERR_TEXT is raised)
 *   n_bytes      host copy of cu_bytes[B] (sizes the launch), below 2^31 - 2
 *   h_rec_types  int32 [9] host: type index (1..n_types) each recognizer emits,
 *                0 switches it off
 *   d_ner_spans, d_ner_cu, ner_cap  decode_spans() output and its capacity
 *                (ner_cap = 0: recognizers alone; spans outside their record
 *                raise ANON_ERR_SPAN and are ignored)
 *   d_spans      out: up to span_cap merged spans, record-major, in byte order
 *   d_cu_spans   int32 [B+1] out: record b owns [cu_spans[b], cu_spans[b+1]);
 *                cu_spans[B] is the total even when it exceeds span_cap
 *                (then ANON_ERR_SPAN_CAP is raised)
 *   d_workspace  >= anon_recognize_workspace_size(n_bytes, B) bytes. */
anon_status anon_recognize_workspace_size(int64_t n_bytes, int32_t B, size_t* bytes);
anon_status recognize_spans(const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B, int64_t n_bytes,
                            const int32_t* h_rec_types, int32_t n_types, const anon_span* d_ner_spans,
                            const int32_t* d_ner_cu, int32_t ner_cap, anon_span* d_spans, int32_t span_cap,
                            int32_t* d_cu_spans, void* d_workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Schema-aware whole-field spans, no NER (the paper's configuration that maps
 * named fields straight to pseudonyms, bypassing inference: Sec. II; Sec. IV-A;
 * App. C, Table VI with and without it)
 * ------------------------------------------------------------------------
 * A line is a maximal run of bytes without '\n' inside one record.  It holds
 * a field if its first ':' is directly followed by ' '; the name is the bytes
 * before the ':', the value the bytes after ": " up to the end of the line.
 * Each line whose name equals (byte for byte) a configured name and whose
 * value is not empty gives one span of that name's type over the value.
 *   d_text, d_cu_bytes, n_bytes  as in recognize_spans (ANON_ERR_TEXT if
 *                                cu_bytes does not rise from 0 to n_bytes)
 *   h_field_names  host, n_fields (0..64) names of 1..32 bytes, no ':' or '\n'
 *   h_field_types  host int32 [n_fields], type index 1..n_types of each name
 *   d_spans, span_cap, d_cu_spans  output as in decode_spans (record-major,
 *                                  byte order; ANON_ERR_SPAN_CAP on overflow)
 *   d_workspace  >= anon_field_workspace_size(n_bytes, B) bytes.
 * The output feeds pseudonymize(). */
anon_status anon_field_workspace_size(int64_t n_bytes, int32_t B, size_t* bytes);
anon_status field_spans(const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B, int64_t n_bytes,
                        const char* const* h_field_names, const int32_t* h_field_types, int32_t n_fields,
                        int32_t n_types, anon_span* d_spans, int32_t span_cap, int32_t* d_cu_spans,
                        void* d_workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Pseudonyms (Sec. II stage 3)
 * ------------------------------------------------------------------------
 * A pseudonym cache holds the HMAC key, the slug length (0..64 lowercase hex
 * characters; 0 gives "[TYPE]"), the type names (type t is type_names[t-1],
 * characters A-Z, 0-9 and '_', at most 32 bytes) and a device hash table
 * mapping entity bytes to their HMAC-SHA256 digest (`capacity` slots, rounded
 * up to a power of two; entities longer than 96 bytes bypass the table).  The
 * table only changes how often HMAC is computed, never the output.  The
 * pseudonym of an entity depends only on (key, entity bytes, type, slug
 * length): the same entity gets the same pseudonym in every record and call. */
anon_status anon_pcache_create(const uint8_t* h_key, size_t key_len, int32_t slug_hex,
                               const char* const* type_names, int32_t n_types, int64_t capacity, int32_t device,
                               anon_pcache** out);
void anon_pcache_free(anon_pcache* cache);
/* Empty the table and zero the counters (stream-ordered). */
anon_status anon_pcache_clear(anon_pcache* cache, void* stream);
/* Enable (1) or bypass (0) the table for later calls. */
anon_status anon_pcache_set_enabled(anon_pcache* cache, int32_t enabled);
/* Probes, probes that found a ready entry, and inserted entries since the
 * last clear.  Synchronises the device. */
anon_status anon_pcache_stats(anon_pcache* cache, int64_t* lookups, int64_t* hits, int64_t* entries);

/* Types to preserve (the paper's per-type control, Sec. II): spans of these
 * types are left as they are by later pseudonymize() calls (their bytes are
 * copied, no pseudonym, no table entry).  The list replaces the previous one;
 * n = 0 preserves nothing.  Types outside 1..n_types are rejected. */
anon_status anon_pcache_set_preserve(anon_pcache* cache, const int32_t* h_types, int32_t n);

/* The entity <-> pseudonym mapping held by the table (the paper's persisted
 * mapping: type, original, slug, full hash, first and last seen; Sec. II
 * stage 4).  One row per distinct entity of at most 96 bytes met by
 * pseudonymize() with the table enabled since creation or the last clear
 * (all of them while the table has room): the smallest type index it was
 * pseudonymized under, its bytes, the full HMAC-SHA256 digest (the slug is
 * its first slug_hex lowercase hex digits) and the first and last call that
 * met it (calls are numbered from 1 per cache; a clear restarts the count).
 * Rows are ordered by first call, then by bytes.  Writes min(cap, total)
 * rows to h_out (host) and the total to *n_entries; synchronises the device. */
typedef struct {
  int32_t type;
  int32_t len;
  uint8_t bytes[96];
  uint8_t digest[32];
  uint32_t first_call;
  uint32_t last_call;
} anon_mapping;
anon_status anon_pcache_export(anon_pcache* cache, anon_mapping* h_out, int64_t cap, int64_t* n_entries);

/* Substitute every span of every record.
 *   d_text      uint8 record bytes back to back; record b is
 *               d_text[cu_bytes[b] .. cu_bytes[b+1])
 *   d_cu_bytes  int64 [B+1]
 *   d_spans, d_cu_spans, span_cap: as written by decode_spans (spans of a
 *               record must be sorted, disjoint and inside the record;
 *               others are skipped and flagged)
 *   d_out       uint8 [out_cap] out: record b is d_out[cu_out[b] .. cu_out[b+1])
 *   d_cu_out    int64 [B+1] out; cu_out[B] is the total length even when it
 *               exceeds out_cap (then the output is truncated and flagged)
 *   d_workspace >= anon_pseudonymize_workspace_size(B, span_cap) bytes. */
anon_status anon_pseudonymize_workspace_size(int32_t B, int32_t span_cap, size_t* bytes);
anon_status pseudonymize(anon_pcache* cache, const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B,
                         const anon_span* d_spans, const int32_t* d_cu_spans, int32_t span_cap, uint8_t* d_out,
                         int64_t out_cap, int64_t* d_cu_out, void* d_workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of record batches (submit / poll)
 * ------------------------------------------------------------------------
 * anon_submit checks a request (record lengths in [1, max_pos], token ids in
 * the vocabulary, token byte ranges ordered, disjoint and inside their record,
 * at most max_request_tokens tokens and 64 text bytes per token: ANON_EINVAL
 * otherwise), copies it and queues it.  A server thread takes queued requests
 * in arrival order into micro-batches of at most `max_batch_tokens` tokens and
 * runs NER, span decoding and substitution on one of `n_streams` streams.
 * Device memory is one activation arena of min(hbm_budget_bytes, what
 * n_streams full micro-batches use) bytes, allocated at start; each
 * micro-batch takes exactly its own footprint (inputs, outputs and the three
 * stages' workspaces) from it, so requests are admitted while their footprint
 * fits the budget left and a slot is free.  Requests that arrive while others
 * run are admitted as soon as budget and a slot free up.  A request's result
 * does not depend on the requests it was batched with.  Results come back
 * through events the thread only queries (it never waits on a stream).
 * Start fails (ANON_ENOMEM) when the budget cannot hold the largest request
 * anon_submit accepts, so every accepted request can run; the scheduler
 * still refuses (ANON_ECAPACITY) any request whose footprint alone exceeds
 * the arena.  A finished request's status is ANON_EDATA when its
 * micro-batch raised a device-data error bit (each micro-batch has its own
 * error word; requests that pass anon_submit's checks do not raise any).
 * With graph_buckets > 0 each slot also holds fixed forward buffers for a
 * full micro-batch (ids, boundaries, token count, labels, error word, NER
 * workspace), taken from the budget before the arena, and runs the NER
 * forward as one graph launch of the smallest bucket that holds the
 * micro-batch; the graphs are captured at start with the model's tile
 * configuration of that moment.  Results are the same in both modes. */
typedef struct {
  int64_t hbm_budget_bytes;   /* activation budget (e.g. 64 GiB)           */
  int32_t max_batch_tokens;   /* tokens per micro-batch                    */
  int32_t n_streams;          /* micro-batches in flight (1..8)            */
  int32_t max_queue;          /* queued requests before anon_submit EBUSY  */
  int32_t max_request_tokens; /* larger requests are rejected (EINVAL)     */
  int32_t graph_buckets;      /* 0: the NER forward is launched kernel by
                               * kernel; n in 1..16: each slot replays a HIP
                               * graph of it per token bucket (n buckets:
                               * max_batch_tokens, then halving; see
                               * ner_forward_capture_bucket) */
} anon_server_config;

/* One request: n_records records with host arrays (copied before return). */
typedef struct {
  int32_t n_records;
  const int32_t* ids;         /* [T]          */
  const int32_t* cu_seqlens;  /* [n_records+1] */
  const int32_t* tok_off;     /* [T, 2]       */
  const uint8_t* text;        /* [cu_bytes[n_records]] */
  const int64_t* cu_bytes;    /* [n_records+1] */
} anon_request;

/* Result of a finished request; buffers stay valid until anon_release. */
typedef struct {
  int32_t status;             /* ANON_OK or a negative anon_status        */
  int32_t n_records;
  int32_t n_tokens;
  int32_t n_spans;
  const uint8_t* out;         /* substituted bytes                         */
  const int64_t* cu_out;      /* [n_records+1]                             */
  const uint8_t* labels;      /* [n_tokens]                                */
  const anon_span* spans;     /* [n_spans], record index local to request  */
  double t_submit, t_start, t_done;  /* seconds, steady clock             */
} anon_result;

anon_status anon_server_start(anon_model* model, anon_pcache* cache, const anon_server_config* cfg,
                              anon_server** out);
anon_status anon_submit(anon_server* server, const anon_request* req, uint64_t* ticket);
/* ANON_PENDING while running; ANON_OK once `out` is filled. */
anon_status anon_poll(anon_server* server, uint64_t ticket, anon_result* out);
anon_status anon_release(anon_server* server, uint64_t ticket);
/* Counters since start: the arena size, the most arena bytes in use at once,
 * micro-batches launched, the most micro-batches in flight at once and the
 * forward passes run as graph replays. */
typedef struct {
  int64_t arena_bytes;
  int64_t peak_arena_bytes;
  int64_t micro_batches;
  int32_t max_concurrent;
  int64_t graph_launches;
} anon_server_counters;
anon_status anon_server_stats(anon_server* server, anon_server_counters* out);
/* Finishes in-flight work, fails queued requests, joins the thread. */
anon_status anon_server_stop(anon_server* server);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support)
 * ------------------------------------------------------------------------
 * While enabled, the library brackets every launch of the kernel class
 * `kclass` with HIP events on the launch stream and accumulates the elapsed
 * time; anon_prof_read synchronises and returns launches, total milliseconds
 * and the algorithmic FLOPs of those launches.  Classes: 0 QKV GEMM,
 * 1 attention, 2 output-projection GEMM, 3 FFN1 GEMM, 4 FFN2 GEMM,
 * 5 LayerNorm, 6 embedding, 7 classifier. */
anon_status anon_prof_enable(int32_t kclass, int32_t enabled);
anon_status anon_prof_read(int32_t kclass, int64_t* launches, double* total_ms, double* flops);

#ifdef __cplusplus
}
#endif
#endif /* ANON_H */
