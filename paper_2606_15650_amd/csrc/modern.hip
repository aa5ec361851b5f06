// The ModernBERT-style encoder (the paper's SecureModernBERT-NER, Sec. II
// stage 2; its accuracy run, Sec. IV-B): model upload, workspace and the
// forward pass, on the same kernels as the BERT-style encoder.
//
//   x = LN_e(E[id])                                FP32 residual stream
//   per layer: h = l ? LN_a(x) : x
//              qkv = h Wqkv, Q/K rotated by position   (EPI_ROPE epilogue)
//              A = attention (global, or |i-j| <= w)     (windowed kernels)
//              x += A Wo                                 (EPI_RESID, FP32 x)
//              x += (GELU(u) * g) Wo2, [u|g] = LN_m(x) Wi (EPI_GEGLU, EPI_RESID)
//   z = LN_h(GELU(LN_f(x) Wd)) Wc + bc                   (EPI_GELU, classifier)
//
// Weights arrive in the x @ W orientation; the GEMMs take them transposed.
// Wi's input and gate halves are interleaved in 32-column blocks on upload,
// so that one wave's 64-column accumulator block holds matching u and g
// columns.  The rotary tables cos/sin(pos * theta^(-2i/64)) of both bases are
// formed on the host in double precision.  LayerNorms have no shift (a zero
// vector), the GEMMs no bias (a zero vector).
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace anon;

namespace {

struct ModernLayerW {
  void *wqkv, *wo, *wi, *wo2;  // [N][K] in the GEMM operand type
  float *attn_g, *mlp_g;       // attn_g is null for layer 0
};

enum { MG_QKV = 0, MG_O, MG_WI, MG_WO2, MG_HEAD, MG_COUNT };

}  // namespace

struct anon_modern {
  anon_modern_config cfg;
  anon_precision prec;
  int device;
  void* mem = nullptr;
  float *tok_emb, *emb_g, *zeros, *final_g, *head_g, *wc_t, *bc, *rope_g, *rope_l;
  void* head_w;
  std::vector<ModernLayerW> layers;
  ElemType gemm_t;  // GEMM operands, Q/K/V, attention and MLP activations
  int gemm_cfg[MG_COUNT] = {-1, -1, -1, -1, -1};
  int attn_cfg = -1;
};

namespace {

size_t esize(ElemType t) { return t == ET_F32 ? 4 : 2; }

anon_status check_modern_cfg(const anon_modern_config* c) {
  if (!c) return set_error(ANON_EINVAL, "config is NULL");
  if (c->n_layers < 1 || c->hidden < 64 || c->n_heads < 1 || c->intermediate < 32 || c->vocab < 1 ||
      c->max_pos < 1 || c->n_labels < 1)
    return set_error(ANON_EINVAL, "config has a non-positive dimension");
  if (c->hidden % c->n_heads != 0 || c->hidden / c->n_heads != 64)
    return set_error(ANON_EINVAL, "head dimension must be 64");
  const int npl = c->hidden / 64;
  if (c->hidden % 64 != 0 || !(npl == 1 || npl == 2 || npl == 4 || npl == 8 || npl == 12 || npl == 16))
    return set_error(ANON_EINVAL, "hidden must be 64 times 1, 2, 4, 8, 12 or 16");
  if (c->intermediate % 32 != 0) return set_error(ANON_EINVAL, "intermediate must be a multiple of 32");
  if (c->n_labels > 32) return set_error(ANON_EINVAL, "at most 32 labels");
  if (c->local_window < 2 || c->global_every < 1) return set_error(ANON_EINVAL, "bad attention pattern");
  if (!(c->theta_global > 1.f) || !(c->theta_local > 1.f)) return set_error(ANON_EINVAL, "bad rotary base");
  if (!(c->ln_eps > 0.f)) return set_error(ANON_EINVAL, "ln_eps must be positive");
  return ANON_OK;
}

size_t n_modern_floats(const anon_modern_config& c) {
  const size_t h = c.hidden, I = c.intermediate, C = c.n_labels;
  size_t n = (size_t)c.vocab * h + h;
  n += (size_t)c.n_layers * (3 * h * h + h * h + h + 2 * I * h + I * h) + (size_t)(c.n_layers - 1) * h;
  n += h + h * h + h + h * C + C;
  return n;
}

bool is_global(const anon_modern_config& c, int l) { return l % c.global_every == 0; }

struct ModernWs {
  float* x;    // residual stream [T, h] FP32
  void* hn;    // GEMM inputs: LayerNorm outputs [T, h]
  void* qkv;   // [T, 3h]
  void* attn;  // attention output, then the head's GELU output [T, h]
  void* mid;   // gated MLP output [T, I]
  int* pos;    // [T]
  int4* items;
  int* n_items;
  int max_items;
};

void modern_layout(const anon_modern* m, int T, int B, Carver& k, ModernWs& w) {
  const size_t h = m->cfg.hidden, I = m->cfg.intermediate, e = esize(m->gemm_t);
  w.x = k.take<float>((size_t)T * h);
  w.hn = k.take<uint8_t>((size_t)T * h * e);
  w.qkv = k.take<uint8_t>((size_t)T * 3 * h * e);
  w.attn = k.take<uint8_t>((size_t)T * h * e);
  w.mid = k.take<uint8_t>((size_t)T * I * e);
  w.pos = k.take<int>(std::max(T, 1));
  w.max_items = 0;
  for (int c = 0; c < attn_num_configs(); ++c) w.max_items = std::max(w.max_items, attn_plan_items(m->gemm_t, c, T, B));
  w.items = k.take<int4>(w.max_items);
  w.n_items = k.take<int>(1);
}

size_t modern_ws_bytes(const anon_modern* m, int T, int B) {
  Carver k(nullptr, SIZE_MAX);
  ModernWs w;
  modern_layout(m, T, B, k, w);
  return k.used + 256;
}

anon_status check_modern_batch(const anon_modern* m, const void* ids, const void* cu, int B, int T) {
  if (!m) return set_error(ANON_EINVAL, "model is NULL");
  if (B < 0 || T < 0) return set_error(ANON_EINVAL, "negative batch size");
  if (B == 0 && T != 0) return set_error(ANON_EINVAL, "T > 0 with no records");
  if ((int64_t)T > (int64_t)B * m->cfg.max_pos) return set_error(ANON_EINVAL, "T exceeds B * max_pos");
  if (B > 0 && !cu) return set_error(ANON_EINVAL, "cu_seqlens is NULL");
  if (T > 0 && !ids) return set_error(ANON_EINVAL, "ids is NULL");
  return ANON_OK;
}

GemmParams base_gemm(const anon_modern* m, int T, int which) {
  GemmParams g{};
  g.M = T;
  g.in = m->gemm_t;
  g.acc_scale = 1.f;
  g.out_inv_scale = 1.f;
  g.qscale = 1.f;
  g.bias = m->zeros;
  g.config = m->gemm_cfg[which];
  return g;
}

// Embedding and the first n_layers layers into w.x (the residual stream).
anon_status run_layers(anon_modern* m, const int* ids, const int* cu, int B, int T, int n_layers, ModernWs& w,
                       hipStream_t s) {
  const anon_modern_config& c = m->cfg;
  const int h = c.hidden, I = c.intermediate;
  const bool bf = m->gemm_t == ET_BF16;
  uint32_t* err = error_word_ptr();
  launch_attn_plan(cu, B, T, c.max_pos, m->gemm_t, m->attn_cfg, w.items, w.max_items, w.n_items, err, s);
  {
    ProfScope ps(KC_EMBED, s, 0.0);
    launch_embed_ln(ids, cu, B, T, m->tok_emb, nullptr, m->emb_g, m->zeros, c.ln_eps, c.vocab, c.max_pos, h, w.x,
                    ET_F32, nullptr, 1.f, err, s, w.pos);
  }
  for (int l = 0; l < n_layers; ++l) {
    const ModernLayerW& L = m->layers[l];
    const bool glob = is_global(c, l);
    // attention input: the stream itself on layer 0, else its LayerNorm
    const void* hin = w.hn;
    {
      ProfScope ps(KC_LN, s, 0.0);
      if (l == 0) {
        if (bf) launch_f32_to_bf16(w.x, (bf16_t*)w.hn, (int64_t)T * h, s);
        else hin = w.x;
      } else {
        launch_layernorm(w.x, ET_F32, L.attn_g, m->zeros, c.ln_eps, T, h, w.hn, m->gemm_t, nullptr, 1.f, s);
      }
    }
    GemmParams g = base_gemm(m, T, MG_QKV);
    g.A = hin;
    g.W = L.wqkv;
    g.C = w.qkv;
    g.N = 3 * h;
    g.K = h;
    g.epi = EPI_ROPE;
    g.out = m->gemm_t;
    g.qscale = 0.125f;  // 1/sqrt(64), exact
    g.qcols = h;
    g.pos = w.pos;
    g.rope = glob ? m->rope_g : m->rope_l;
    g.rope_cols = 2 * h;
    {
      ProfScope ps(KC_QKV, s, 2.0 * T * 3 * h * h);
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    {
      ProfScope ps(KC_ATTN, s, 0.0);
      launch_attention(w.qkv, w.attn, w.items, w.max_items, w.n_items, c.n_heads, h, m->gemm_t, m->gemm_t, 1.f,
                       m->attn_cfg, s, glob ? 0 : c.local_window / 2);
    }
    g = base_gemm(m, T, MG_O);
    g.A = w.attn;
    g.W = L.wo;
    g.resid = w.x;
    g.res = ET_F32;
    g.C = w.x;
    g.out = ET_F32;
    g.N = h;
    g.K = h;
    g.epi = EPI_RESID;
    {
      ProfScope ps(KC_OPROJ, s, 2.0 * T * h * h);
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    {
      ProfScope ps(KC_LN, s, 0.0);
      launch_layernorm(w.x, ET_F32, L.mlp_g, m->zeros, c.ln_eps, T, h, w.hn, m->gemm_t, nullptr, 1.f, s);
    }
    g = base_gemm(m, T, MG_WI);
    g.A = w.hn;
    g.W = L.wi;
    g.C = w.mid;
    g.out = m->gemm_t;
    g.N = 2 * I;
    g.K = h;
    g.epi = EPI_GEGLU;
    {
      ProfScope ps(KC_FFN1, s, 2.0 * T * 2 * I * h);
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    g = base_gemm(m, T, MG_WO2);
    g.A = w.mid;
    g.W = L.wo2;
    g.resid = w.x;
    g.res = ET_F32;
    g.C = w.x;
    g.out = ET_F32;
    g.N = h;
    g.K = I;
    g.epi = EPI_RESID;
    {
      ProfScope ps(KC_FFN2, s, 2.0 * T * I * h);
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
  }
  return ANON_OK;
}

// The host's rotary table of one base: [max_pos][64], cos in the first 32
// entries of a row, sin in the last 32.
std::vector<float> rope_table(int max_pos, double theta) {
  std::vector<float> t((size_t)max_pos * 64);
  for (int p = 0; p < max_pos; ++p)
    for (int i = 0; i < 32; ++i) {
      const double a = (double)p * pow(theta, -2.0 * i / 64.0);
      t[(size_t)p * 64 + i] = (float)cos(a);
      t[(size_t)p * 64 + 32 + i] = (float)sin(a);
    }
  return t;
}

}  // namespace

extern "C" {

anon_status anon_modern_create(const anon_modern_config* cfg, const float* h_weights, size_t n_floats,
                               anon_precision precision, int32_t device, anon_modern** out) {
  clear_error();
  if (!out) return set_error(ANON_EINVAL, "out is NULL");
  *out = nullptr;
  anon_status st = check_modern_cfg(cfg);
  if (st != ANON_OK) return st;
  if (!h_weights) return set_error(ANON_EINVAL, "weights are NULL");
  if (n_floats != n_modern_floats(*cfg))
    return set_error(ANON_EINVAL, "weights hold " + std::to_string(n_floats) + " floats, the config needs " +
                                      std::to_string(n_modern_floats(*cfg)));
  if (precision != ANON_FP32 && precision != ANON_BF16)
    return set_error(ANON_EINVAL, "the ModernBERT-style encoder runs in FP32 or BF16");
  int ndev = 0;
  ANON_HIP_CHECK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(ANON_EINVAL, "no such device");
  ANON_HIP_CHECK(hipSetDevice(device));
  anon_modern* m = new anon_modern();
  m->cfg = *cfg;
  m->prec = precision;
  m->device = device;
  m->gemm_t = precision == ANON_FP32 ? ET_F32 : ET_BF16;
  const anon_modern_config& c = *cfg;
  const size_t h = c.hidden, I = c.intermediate, C = c.n_labels, e = esize(m->gemm_t);
  const size_t nz = std::max<size_t>(3 * h, 2 * I);
  auto plan = [&](Carver& k) {
    m->tok_emb = k.take<float>((size_t)c.vocab * h);
    m->emb_g = k.take<float>(h);
    m->zeros = k.take<float>(nz);
    m->layers.resize(c.n_layers);
    for (int l = 0; l < c.n_layers; ++l) {
      ModernLayerW& L = m->layers[l];
      L.attn_g = l ? k.take<float>(h) : nullptr;
      L.wqkv = k.take<uint8_t>(3 * h * h * e);
      L.wo = k.take<uint8_t>(h * h * e);
      L.mlp_g = k.take<float>(h);
      L.wi = k.take<uint8_t>(2 * I * h * e);
      L.wo2 = k.take<uint8_t>(I * h * e);
    }
    m->final_g = k.take<float>(h);
    m->head_w = k.take<uint8_t>(h * h * e);
    m->head_g = k.take<float>(h);
    m->wc_t = k.take<float>(C * h);
    m->bc = k.take<float>(C);
    m->rope_g = k.take<float>((size_t)c.max_pos * 64);
    m->rope_l = k.take<float>((size_t)c.max_pos * 64);
  };
  Carver cv(nullptr, SIZE_MAX);
  plan(cv);
  if (hipMalloc(&m->mem, cv.used) != hipSuccess) {
    delete m;
    return set_error(ANON_ENOMEM, "cannot allocate " + std::to_string(cv.used) + " bytes of weights");
  }
  Carver real(m->mem, cv.used);
  plan(real);
  // staging: the largest matrix (or the embedding table), FP32
  size_t stage_n = std::max<size_t>({(size_t)c.vocab * h, 3 * h * h, 2 * I * h, (size_t)c.max_pos * 64});
  float* staging = nullptr;
  if (hipMalloc(&staging, stage_n * sizeof(float)) != hipSuccess) {
    hipFree(m->mem);
    delete m;
    return set_error(ANON_ENOMEM, "cannot allocate the weight staging buffer");
  }
  hipStream_t s = nullptr;
  hipError_t err = hipMemsetAsync(m->zeros, 0, nz * sizeof(float), s);
  size_t off = 0;
  auto put = [&](float* dst, size_t n) {  // FP32 vector or table, as given
    if (err == hipSuccess) err = hipMemcpy(dst, h_weights + off, n * sizeof(float), hipMemcpyHostToDevice);
    off += n;
  };
  // [K][N] (x @ W) -> [N][K] in the operand type; `src` defaults to the blob
  auto gemm_w = [&](void* dst, size_t K, size_t N, const float* src) {
    if (err == hipSuccess) err = hipMemcpy(staging, src ? src : h_weights + off, K * N * sizeof(float),
                                           hipMemcpyHostToDevice);
    if (err == hipSuccess) {
      launch_transpose_convert(staging, (int)K, (int)N, dst, m->gemm_t, 1.f, s);
      err = hipDeviceSynchronize();
    }
    off += K * N;
  };
  put(m->tok_emb, (size_t)c.vocab * h);
  put(m->emb_g, h);
  std::vector<float> inter(2 * I * h);
  for (int l = 0; l < c.n_layers; ++l) {
    ModernLayerW& L = m->layers[l];
    if (l) put(L.attn_g, h);
    gemm_w(L.wqkv, h, 3 * h, nullptr);
    gemm_w(L.wo, h, h, nullptr);
    put(L.mlp_g, h);
    // Wi [h][2I]: column blocks of 32 alternate between the input half and
    // the gate half
    const float* wi = h_weights + off;
    for (size_t r = 0; r < h; ++r)
      for (size_t b = 0; b < I / 32; ++b)
        for (size_t j = 0; j < 32; ++j) {
          inter[r * 2 * I + b * 64 + j] = wi[r * 2 * I + b * 32 + j];
          inter[r * 2 * I + b * 64 + 32 + j] = wi[r * 2 * I + I + b * 32 + j];
        }
    gemm_w(L.wi, h, 2 * I, inter.data());
    gemm_w(L.wo2, I, h, nullptr);
  }
  put(m->final_g, h);
  gemm_w(m->head_w, h, h, nullptr);
  put(m->head_g, h);
  if (err == hipSuccess) err = hipMemcpy(staging, h_weights + off, h * C * sizeof(float), hipMemcpyHostToDevice);
  if (err == hipSuccess) {
    launch_transpose_convert(staging, (int)h, (int)C, m->wc_t, ET_F32, 1.f, s);
    err = hipDeviceSynchronize();
  }
  off += h * C;
  put(m->bc, C);
  const std::vector<float> tg = rope_table(c.max_pos, c.theta_global), tl = rope_table(c.max_pos, c.theta_local);
  if (err == hipSuccess) err = hipMemcpy(m->rope_g, tg.data(), tg.size() * sizeof(float), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(m->rope_l, tl.data(), tl.size() * sizeof(float), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipDeviceSynchronize();
  hipFree(staging);
  if (err != hipSuccess || off != n_floats) {
    hipFree(m->mem);
    delete m;
    return set_error(ANON_EDEVICE, std::string("weight upload: ") + hipGetErrorString(err));
  }
  *out = m;
  return ANON_OK;
}

void anon_modern_free(anon_modern* m) {
  if (!m) return;
  hipSetDevice(m->device);
  hipFree(m->mem);
  delete m;
}

anon_status anon_modern_workspace_size(const anon_modern* m, int32_t T, int32_t B, size_t* bytes) {
  if (!m || !bytes || T < 0 || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  *bytes = modern_ws_bytes(m, T, B);
  return ANON_OK;
}

anon_status modern_ner_forward(anon_modern* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                               int32_t T, uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                               size_t ws_bytes, void* stream) {
  clear_error();
  anon_status st = check_modern_batch(m, d_ids, d_cu_seqlens, B, T);
  if (st != ANON_OK) return st;
  if (T == 0) return ANON_OK;
  if (!d_labels) return set_error(ANON_EINVAL, "labels is NULL");
  if (!d_workspace || ws_bytes < modern_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  Carver k(d_workspace, ws_bytes);
  ModernWs w;
  modern_layout(m, T, B, k, w);
  const anon_modern_config& c = m->cfg;
  const int h = c.hidden;
  st = run_layers(m, d_ids, d_cu_seqlens, B, T, c.n_layers, w, s);
  if (st != ANON_OK) return st;
  {
    ProfScope ps(KC_LN, s, 0.0);
    launch_layernorm(w.x, ET_F32, m->final_g, m->zeros, c.ln_eps, T, h, w.hn, m->gemm_t, nullptr, 1.f, s);
  }
  GemmParams g = base_gemm(m, T, MG_HEAD);
  g.A = w.hn;
  g.W = m->head_w;
  g.C = w.attn;
  g.out = m->gemm_t;
  g.N = h;
  g.K = h;
  g.epi = EPI_GELU;
  {
    ProfScope ps(KC_CLS, s, 2.0 * T * h * h);
    if (!launch_gemm(g, s)) return ANON_EINVAL;
    launch_layernorm(w.attn, m->gemm_t, m->head_g, m->zeros, c.ln_eps, T, h, w.hn, m->gemm_t, nullptr, 1.f, s);
    launch_classifier(w.hn, m->gemm_t, m->wc_t, m->bc, T, h, c.n_labels, d_labels, d_logits, d_margin, s);
  }
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

anon_status anon_modern_hidden(anon_modern* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                               int32_t T, int32_t n_layers, float* d_hidden, void* d_workspace, size_t ws_bytes,
                               void* stream) {
  clear_error();
  anon_status st = check_modern_batch(m, d_ids, d_cu_seqlens, B, T);
  if (st != ANON_OK) return st;
  if (n_layers < 0 || n_layers > m->cfg.n_layers) return set_error(ANON_EINVAL, "n_layers out of range");
  if (T == 0) return ANON_OK;
  if (!d_hidden) return set_error(ANON_EINVAL, "hidden is NULL");
  if (!d_workspace || ws_bytes < modern_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  Carver k(d_workspace, ws_bytes);
  ModernWs w;
  modern_layout(m, T, B, k, w);
  st = run_layers(m, d_ids, d_cu_seqlens, B, T, n_layers, w, s);
  if (st != ANON_OK) return st;
  ANON_HIP_CHECK(hipMemcpyAsync(d_hidden, w.x, (size_t)T * m->cfg.hidden * sizeof(float), hipMemcpyDeviceToDevice,
                                s));
  return ANON_OK;
}

anon_status anon_modern_set_tiles(anon_modern* m, const int32_t tiles[5], int32_t attn_config) {
  if (!m || !tiles) return set_error(ANON_EINVAL, "NULL argument");
  const int h = m->cfg.hidden, I = m->cfg.intermediate;
  const int NK[MG_COUNT][2] = {{3 * h, h}, {h, h}, {2 * I, h}, {h, I}, {h, h}};
  const int epi[MG_COUNT] = {EPI_ROPE, EPI_RESID, EPI_GEGLU, EPI_RESID, EPI_GELU};
  const ElemType out[MG_COUNT] = {m->gemm_t, ET_F32, m->gemm_t, ET_F32, m->gemm_t};
  for (int i = 0; i < MG_COUNT; ++i) {
    if (tiles[i] < 0) continue;
    GemmParams g{};
    g.in = m->gemm_t;
    g.out = out[i];
    g.epi = (GemmEpi)epi[i];
    g.N = NK[i][0];
    g.K = NK[i][1];
    if (tiles[i] >= gemm_num_configs(m->gemm_t) || !gemm_config_serves(g, tiles[i]))
      return set_error(ANON_EINVAL, "tile configuration does not serve GEMM " + std::to_string(i));
  }
  if (attn_config < -1 || attn_config >= attn_num_configs())
    return set_error(ANON_EINVAL, "no such attention configuration");
  for (int i = 0; i < MG_COUNT; ++i) m->gemm_cfg[i] = tiles[i];
  m->attn_cfg = attn_config;
  return ANON_OK;
}

anon_status anon_modern_get_tiles(const anon_modern* m, int32_t tiles[5], int32_t* attn_config) {
  if (!m) return set_error(ANON_EINVAL, "model is NULL");
  for (int i = 0; i < MG_COUNT; ++i) {
    if (!tiles) break;
    tiles[i] = m->gemm_cfg[i];
  }
  if (attn_config) *attn_config = m->attn_cfg;
  return ANON_OK;
}

}  // extern "C"
