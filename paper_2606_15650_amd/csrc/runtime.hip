// Host runtime of libanon: the model (weights in HBM, per-precision layouts),
// workspace carving, the encoder driver, span decoding, pseudonym caches,
// kernel timing, and the C ABI entry points of include/anon.h.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace anon {

// ---------------------------------------------------------------- errors --
static thread_local std::string t_last_error;

anon_status set_error(anon_status st, const std::string& msg) {
  t_last_error = msg;
  return st;
}
void clear_error() { t_last_error.clear(); }

static std::mutex g_err_mu;
static uint32_t* g_err_words[64] = {nullptr};

// A caller that wants the errors of its own launches apart (the server, per
// micro-batch) points this thread's launches at another word for a while.
static thread_local uint32_t* t_err_override = nullptr;
void set_thread_error_word(uint32_t* w) { t_err_override = w; }

// The per-device error word is a device array of the library (zero when the
// code object loads, one copy per GPU), so that no call allocates for it.
static __device__ __align__(256) uint32_t g_err_dev[64];

uint32_t* error_word_ptr() {
  if (t_err_override) return t_err_override;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_err_mu);
  if (!g_err_words[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_err_dev)) != hipSuccess) return nullptr;
    g_err_words[dev] = (uint32_t*)p;
  }
  return g_err_words[dev];
}

// ---------------------------------------------------------------- timing --
struct ProfState {
  bool enabled[KC_COUNT] = {false};
  int64_t launches[KC_COUNT] = {0};
  double ms[KC_COUNT] = {0};
  double flops[KC_COUNT] = {0};
  struct Pending {
    int kc;
    hipEvent_t a, b;
    double flops;
  };
  std::vector<Pending> pending;
  std::mutex mu;
};
static ProfState g_prof;

ProfScope::ProfScope(int kc_, hipStream_t s_, double fl) : kc(kc_), s(s_), flops(fl) {
  if (kc < 0 || kc >= KC_COUNT || !g_prof.enabled[kc]) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

ProfScope::~ProfScope() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.pending.push_back({kc, e0, e1, flops});
}

static void prof_drain() {
  std::vector<ProfState::Pending> p;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    p.swap(g_prof.pending);
  }
  for (auto& e : p) {
    (void)hipEventSynchronize(e.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e.a, e.b);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.launches[e.kc] += 1;
    g_prof.ms[e.kc] += ms;
    g_prof.flops[e.kc] += e.flops;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
}

}  // namespace anon

using namespace anon;

// ----------------------------------------------------------------- model --
struct LayerW {
  void *wqkv, *wo, *w1, *w2;  // [N][K] in the GEMM operand type
  float *bqkv, *bo, *b1, *b2, *ln1_g, *ln1_b, *ln2_g, *ln2_b;
  float sw[4];  // FP8 weight scales (qkv, o, ffn1, ffn2)
  float sa[4];  // FP8 activation scales of the GEMM inputs
};

struct anon_model {
  anon_model_config cfg;
  anon_precision prec;
  int device;
  void* mem = nullptr;
  float *tok_emb, *pos_emb, *emb_g, *emb_b, *wc_t, *bc;
  std::vector<LayerW> layers;
  ElemType gemm_t;  // operand type of the big GEMMs
  ElemType act_t;   // stored hidden state / residual
  ElemType qkv_t;   // Q, K, V and attention operands
  int gemm_cfg[4] = {-1, -1, -1, -1};
  int gemm_gm[4] = {0, 0, 0, 0};  // row blocks per tile group (0: by shape)
  int attn_cfg = -1;               // attention tile configuration (-1: default)
};

const anon_model_config* anon::model_config(const anon_model* m) { return &m->cfg; }

static bool is_pow2_scale(float s) {
  if (!(s > 0.f) || !isfinite(s)) return false;
  int e;
  const float m = frexpf(s, &e);
  return m == 0.5f;
}

// Smallest power of two s with amax / s <= 448 (the E4M3 maximum).  log2 of
// the rounded quotient can land one binade off near amax = 448 * 2^k, so the
// estimate is corrected against the definition.
static float pow2_scale_for(float amax) {
  if (!(amax > 0.f)) return 1.f;
  int e = (int)ceil(log2((double)amax / 448.0));
  while ((double)amax / ldexp(1.0, e) > 448.0) ++e;
  while ((double)amax / ldexp(1.0, e - 1) <= 448.0) --e;
  return ldexpf(1.f, e);
}

static size_t elem_size(ElemType t) { return t == ET_F32 ? 4 : (t == ET_BF16 ? 2 : 1); }

static anon_status check_cfg(const anon_model_config* c) {
  if (!c) return set_error(ANON_EINVAL, "config is NULL");
  if (c->n_layers < 1 || c->hidden < 64 || c->n_heads < 1 || c->ffn < 64 || c->vocab < 1 || c->max_pos < 1)
    return set_error(ANON_EINVAL, "config has a non-positive dimension");
  if (c->hidden % c->n_heads != 0 || c->hidden / c->n_heads != 64)
    return set_error(ANON_EINVAL, "head dimension hidden/n_heads must be 64");
  const int npl = c->hidden / 64;
  if (c->hidden % 64 || !(npl == 1 || npl == 2 || npl == 4 || npl == 8 || npl == 12 || npl == 16))
    return set_error(ANON_EINVAL, "hidden must be 64 * {1,2,4,8,12,16}");
  if (c->ffn % 128) return set_error(ANON_EINVAL, "ffn must be a multiple of 128");
  if (c->n_labels < 1 || c->n_labels > 63 || c->n_labels % 2 == 0)
    return set_error(ANON_EINVAL, "n_labels must be odd (2*types+1) and <= 63");
  if (!(c->ln_eps > 0.f)) return set_error(ANON_EINVAL, "ln_eps must be positive");
  return ANON_OK;
}

static size_t n_weight_floats(const anon_model_config& c) {
  const size_t h = c.hidden, f = c.ffn, C = c.n_labels;
  size_t n = (size_t)c.vocab * h + (size_t)c.max_pos * h + 2 * h;
  n += (size_t)c.n_layers * (h * 3 * h + 3 * h + h * h + h + 2 * h + h * f + f + f * h + h + 2 * h);
  n += h * C + C;
  return n;
}

extern "C" {

const char* anon_last_error(void) { return t_last_error.c_str(); }

int32_t anon_version(void) { return 4; }

anon_status anon_device_errors(int32_t device, uint32_t* flags, int32_t clear) {
  if (!flags) return set_error(ANON_EINVAL, "flags is NULL");
  ANON_HIP_CHECK(hipSetDevice(device));
  uint32_t* w = error_word_ptr();
  if (!w) return set_error(ANON_EDEVICE, "cannot allocate the device error word");
  ANON_HIP_CHECK(hipDeviceSynchronize());
  ANON_HIP_CHECK(hipMemcpy(flags, w, 4, hipMemcpyDeviceToHost));
  if (clear) ANON_HIP_CHECK(hipMemset(w, 0, 4));
  return ANON_OK;
}

anon_status anon_model_create(const anon_model_config* cfg, const float* h_weights, size_t n_floats,
                              anon_precision precision, const float* h_act_scales, int32_t device,
                              anon_model** out) {
  clear_error();
  if (!out) return set_error(ANON_EINVAL, "out is NULL");
  *out = nullptr;
  anon_status st = check_cfg(cfg);
  if (st != ANON_OK) return st;
  if (!h_weights) return set_error(ANON_EINVAL, "weights are NULL");
  if (n_floats != n_weight_floats(*cfg))
    return set_error(ANON_EINVAL, "weights hold " + std::to_string(n_floats) + " floats, the config needs " +
                                      std::to_string(n_weight_floats(*cfg)));
  if (precision != ANON_FP32 && precision != ANON_BF16 && precision != ANON_FP8_E4M3)
    return set_error(ANON_EINVAL, "unknown precision");
  if (precision == ANON_FP8_E4M3) {
    if (!h_act_scales) return set_error(ANON_EINVAL, "FP8 needs 4*n_layers activation scales");
    for (int i = 0; i < 4 * cfg->n_layers; ++i)
      if (!is_pow2_scale(h_act_scales[i])) return set_error(ANON_EINVAL, "activation scales must be powers of two");
  }
  int ndev = 0;
  ANON_HIP_CHECK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(ANON_EINVAL, "no such device");
  ANON_HIP_CHECK(hipSetDevice(device));

  anon_model* m = new anon_model();
  m->cfg = *cfg;
  m->prec = precision;
  m->device = device;
  m->gemm_t = precision == ANON_FP32 ? ET_F32 : (precision == ANON_BF16 ? ET_BF16 : ET_FP8);
  m->act_t = precision == ANON_FP32 ? ET_F32 : ET_BF16;
  m->qkv_t = m->act_t;
  const anon_model_config& c = *cfg;
  const size_t h = c.hidden, f = c.ffn, C = c.n_labels;
  const size_t es = elem_size(m->gemm_t);

  // one device allocation for all weights
  Carver cv(nullptr, SIZE_MAX);
  auto plan = [&](Carver& k) {
    m->tok_emb = k.take<float>((size_t)c.vocab * h);
    m->pos_emb = k.take<float>((size_t)c.max_pos * h);
    m->emb_g = k.take<float>(h);
    m->emb_b = k.take<float>(h);
    m->layers.resize(c.n_layers);
    for (auto& L : m->layers) {
      L.wqkv = k.take<uint8_t>(3 * h * h * es);
      L.wo = k.take<uint8_t>(h * h * es);
      L.w1 = k.take<uint8_t>(f * h * es);
      L.w2 = k.take<uint8_t>(h * f * es);
      L.bqkv = k.take<float>(3 * h);
      L.bo = k.take<float>(h);
      L.b1 = k.take<float>(f);
      L.b2 = k.take<float>(h);
      L.ln1_g = k.take<float>(h);
      L.ln1_b = k.take<float>(h);
      L.ln2_g = k.take<float>(h);
      L.ln2_b = k.take<float>(h);
    }
    m->wc_t = k.take<float>(C * h);
    m->bc = k.take<float>(C);
  };
  plan(cv);
  const size_t total = cv.used;
  if (hipMalloc(&m->mem, total) != hipSuccess) {
    delete m;
    return set_error(ANON_ENOMEM, "cannot allocate " + std::to_string(total) + " bytes of weights");
  }
  Carver real(m->mem, total);
  plan(real);

  float* staging = nullptr;
  if (hipMalloc(&staging, n_floats * sizeof(float)) != hipSuccess) {
    hipFree(m->mem);
    delete m;
    return set_error(ANON_ENOMEM, "cannot allocate the weight staging buffer");
  }
  hipStream_t s = nullptr;
  hipError_t e = hipMemcpy(staging, h_weights, n_floats * sizeof(float), hipMemcpyHostToDevice);
  size_t off = 0;
  auto copy_f32 = [&](float* dst, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, staging + off, n * sizeof(float), hipMemcpyDeviceToDevice, s);
    off += n;
  };
  // GEMM weight [K][N] (x @ W orientation) -> [N][K] operand layout
  auto gemm_w = [&](void* dst, size_t K, size_t N, float* scale_out) {
    float sc = 1.f;
    if (m->gemm_t == ET_FP8) {
      float amax = 0.f;
      for (size_t i = 0; i < K * N; ++i) amax = fmaxf(amax, fabsf(h_weights[off + i]));
      sc = pow2_scale_for(amax);
    }
    if (scale_out) *scale_out = sc;
    if (e == hipSuccess) {
      launch_transpose_convert(staging + off, (int)K, (int)N, dst, m->gemm_t, 1.f / sc, s);
      e = hipGetLastError();
    }
    off += K * N;
  };
  copy_f32(m->tok_emb, (size_t)c.vocab * h);
  copy_f32(m->pos_emb, (size_t)c.max_pos * h);
  copy_f32(m->emb_g, h);
  copy_f32(m->emb_b, h);
  for (int l = 0; l < c.n_layers; ++l) {
    LayerW& L = m->layers[l];
    gemm_w(L.wqkv, h, 3 * h, &L.sw[0]);
    copy_f32(L.bqkv, 3 * h);
    gemm_w(L.wo, h, h, &L.sw[1]);
    copy_f32(L.bo, h);
    copy_f32(L.ln1_g, h);
    copy_f32(L.ln1_b, h);
    gemm_w(L.w1, h, f, &L.sw[2]);
    copy_f32(L.b1, f);
    gemm_w(L.w2, f, h, &L.sw[3]);
    copy_f32(L.b2, h);
    copy_f32(L.ln2_g, h);
    copy_f32(L.ln2_b, h);
    for (int i = 0; i < 4; ++i) L.sa[i] = precision == ANON_FP8_E4M3 ? h_act_scales[4 * l + i] : 1.f;
  }
  if (e == hipSuccess) {
    launch_transpose_convert(staging + off, (int)h, (int)C, m->wc_t, ET_F32, 1.f, s);
    e = hipGetLastError();
  }
  off += h * C;
  copy_f32(m->bc, C);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  hipFree(staging);
  if (e != hipSuccess) {
    hipFree(m->mem);
    delete m;
    return set_error(ANON_EDEVICE, std::string("weight upload: ") + hipGetErrorString(e));
  }
  *out = m;
  return ANON_OK;
}

void anon_model_free(anon_model* m) {
  if (!m) return;
  hipSetDevice(m->device);
  hipFree(m->mem);
  delete m;
}

}  // extern "C"

// ------------------------------------------------------------ weights file --
// A 64-byte header -- "ANONWTS1", format version, kind (0: the BERT-style
// encoder), the model config, the float count, the FNV-1a-64 hash of the
// float bytes -- then the FP32 weights in anon_model_create's order, all
// little-endian.
namespace {
struct WeightsHeader {
  char magic[8];
  uint32_t version, kind;
  anon_model_config cfg;
  uint64_t n_floats, fnv;
};
static_assert(sizeof(WeightsHeader) == 64 && offsetof(WeightsHeader, cfg) == 16 &&
                  offsetof(WeightsHeader, n_floats) == 48,
              "weights header layout");
constexpr char kWeightsMagic[8] = {'A', 'N', 'O', 'N', 'W', 'T', 'S', '1'};
constexpr uint32_t kWeightsVersion = 1;

uint64_t fnv1a64(const void* data, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
  const uint8_t* p = (const uint8_t*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 0x100000001b3ull;
  return h;
}

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

// Reads and checks the header and, if `w` is given, the weights (hash
// included); touches no device.
anon_status read_weights(const char* path, WeightsHeader& h, std::vector<float>* w) {
  if (!path) return set_error(ANON_EINVAL, "path is NULL");
  File f;
  f.f = fopen(path, "rb");
  if (!f.f) return set_error(ANON_EINVAL, std::string("cannot open ") + path);
  if (fread(&h, sizeof h, 1, f.f) != 1) return set_error(ANON_EINVAL, "weights file shorter than its header");
  if (memcmp(h.magic, kWeightsMagic, 8) != 0) return set_error(ANON_EINVAL, "not a weights file (magic)");
  if (h.version != kWeightsVersion)
    return set_error(ANON_EINVAL, "weights file version " + std::to_string(h.version) + ", this library reads " +
                                      std::to_string(kWeightsVersion));
  if (h.kind != 0) return set_error(ANON_EINVAL, "weights file holds another encoder kind");
  anon_status st = check_cfg(&h.cfg);
  if (st != ANON_OK) return st;
  if (h.n_floats != n_weight_floats(h.cfg))
    return set_error(ANON_EINVAL, "weights file holds " + std::to_string(h.n_floats) + " floats, its config needs " +
                                      std::to_string(n_weight_floats(h.cfg)));
  if (fseek(f.f, 0, SEEK_END) != 0) return set_error(ANON_EINVAL, "cannot size the weights file");
  const long size = ftell(f.f);
  if (size < 0 || (uint64_t)size != sizeof h + h.n_floats * sizeof(float))
    return set_error(ANON_EINVAL, "weights file size does not match its header");
  if (!w) return ANON_OK;
  if (fseek(f.f, (long)sizeof h, SEEK_SET) != 0) return set_error(ANON_EINVAL, "cannot read the weights");
  try {
    w->resize(h.n_floats);
  } catch (...) {
    return set_error(ANON_ENOMEM, "no host memory for the weights");
  }
  if (fread(w->data(), sizeof(float), h.n_floats, f.f) != h.n_floats)
    return set_error(ANON_EINVAL, "cannot read the weights");
  if (fnv1a64(w->data(), h.n_floats * sizeof(float)) != h.fnv)
    return set_error(ANON_EINVAL, "weights file hash mismatch (corrupt file)");
  return ANON_OK;
}
}  // namespace

extern "C" {

anon_status anon_weights_write(const char* path, const anon_model_config* cfg, const float* h_weights,
                               size_t n_floats) {
  clear_error();
  if (!path || !h_weights) return set_error(ANON_EINVAL, "NULL argument");
  anon_status st = check_cfg(cfg);
  if (st != ANON_OK) return st;
  if (n_floats != n_weight_floats(*cfg))
    return set_error(ANON_EINVAL, "weights hold " + std::to_string(n_floats) + " floats, the config needs " +
                                      std::to_string(n_weight_floats(*cfg)));
  WeightsHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kWeightsMagic, 8);
  h.version = kWeightsVersion;
  h.kind = 0;
  h.cfg = *cfg;
  h.n_floats = n_floats;
  h.fnv = fnv1a64(h_weights, n_floats * sizeof(float));
  File f;
  f.f = fopen(path, "wb");
  if (!f.f) return set_error(ANON_EINVAL, std::string("cannot create ") + path);
  if (fwrite(&h, sizeof h, 1, f.f) != 1 || fwrite(h_weights, sizeof(float), n_floats, f.f) != n_floats)
    return set_error(ANON_EINVAL, std::string("cannot write ") + path);
  const int rc = fclose(f.f);
  f.f = nullptr;
  if (rc != 0) return set_error(ANON_EINVAL, std::string("cannot write ") + path);
  return ANON_OK;
}

anon_status anon_weights_info(const char* path, anon_model_config* cfg, size_t* n_floats) {
  clear_error();
  WeightsHeader h;
  std::vector<float> w;
  const anon_status st = read_weights(path, h, &w);
  if (st != ANON_OK) return st;
  if (cfg) *cfg = h.cfg;
  if (n_floats) *n_floats = h.n_floats;
  return ANON_OK;
}

anon_status anon_model_load(const char* path, anon_precision precision, const float* h_act_scales, int32_t device,
                            anon_model** out) {
  clear_error();
  if (!out) return set_error(ANON_EINVAL, "out is NULL");
  *out = nullptr;
  WeightsHeader h;
  std::vector<float> w;
  const anon_status st = read_weights(path, h, &w);
  if (st != ANON_OK) return st;
  return anon_model_create(&h.cfg, w.data(), w.size(), precision, h_act_scales, device, out);
}

}  // extern "C"

// ------------------------------------------------------------- encoder ----
struct EncWs {
  void *x, *x2, *qkv, *attn, *ffn;
  fp8_t* xq;
  void* y;  // pre-LayerNorm residual sum (act type)
  int4* qblocks;
  int* nq;
  int max_q;
};

static void enc_layout(const anon_model* m, int T, int B, Carver& k, EncWs& w) {
  const size_t h = m->cfg.hidden, f = m->cfg.ffn;
  const size_t a = elem_size(m->act_t), g = elem_size(m->gemm_t), q = elem_size(m->qkv_t);
  w.x = k.take<uint8_t>(T * h * a);
  w.x2 = k.take<uint8_t>(T * h * a);
  w.xq = m->gemm_t == ET_FP8 ? k.take<fp8_t>(T * h) : nullptr;
  w.qkv = k.take<uint8_t>(T * 3 * h * q);
  w.attn = k.take<uint8_t>(T * h * g);
  w.y = k.take<uint8_t>(T * h * a);
  w.ffn = k.take<uint8_t>(T * f * g);
  // room for the work list of any attention configuration
  w.max_q = 0;
  for (int c = 0; c < attn_num_configs(); ++c) w.max_q = std::max(w.max_q, attn_plan_items(m->qkv_t, c, T, B));
  w.qblocks = k.take<int4>(w.max_q);
  w.nq = k.take<int>(1);
}

static anon_status check_batch(const anon_model* m, const void* d_ids, const void* d_cu, int B, int T) {
  if (!m) return set_error(ANON_EINVAL, "model is NULL");
  if (B < 0 || T < 0) return set_error(ANON_EINVAL, "negative batch size");
  if (B == 0 && T != 0) return set_error(ANON_EINVAL, "T > 0 with no records");
  if ((int64_t)T > (int64_t)B * m->cfg.max_pos) return set_error(ANON_EINVAL, "T exceeds B * max_pos");
  if (B > 0 && !d_cu) return set_error(ANON_EINVAL, "cu_seqlens is NULL");
  if (T > 0 && !d_ids) return set_error(ANON_EINVAL, "ids is NULL");
  return ANON_OK;
}

static double gemm_flops(double M, double N, double K) { return 2.0 * M * N * K; }

// Runs the embedding and the first n_layers layers; returns the hidden state.
// t_dev (nullable): the token count in device memory, at most T (the
// capacity every grid is sized for).
static anon_status run_encoder(anon_model* m, const int* ids, const int* cu, int B, int T, int n_layers, EncWs& w,
                               hipStream_t s, const int* t_dev = nullptr) {
  const anon_model_config& c = m->cfg;
  const int h = c.hidden, f = c.ffn;
  uint32_t* err = error_word_ptr();
  const bool fp8 = m->gemm_t == ET_FP8;
  launch_attn_plan(cu, B, T, c.max_pos, m->qkv_t, m->attn_cfg, w.qblocks, w.max_q, w.nq, err, s, t_dev);
  {
    ProfScope ps(KC_EMBED, s, 0.0);
    launch_embed_ln(ids, cu, B, T, m->tok_emb, m->pos_emb, m->emb_g, m->emb_b, c.ln_eps, c.vocab, c.max_pos, h, w.x,
                    m->act_t, w.xq, fp8 ? 1.f / m->layers[0].sa[0] : 1.f, err, s, nullptr, t_dev);
  }
  // attention FLOPs are counted from token-weighted lengths by the caller
  for (int l = 0; l < n_layers; ++l) {
    const LayerW& L = m->layers[l];
    GemmParams g{};
    g.M = T;
    g.m_dev = t_dev;
    g.in = m->gemm_t;
    g.acc_scale = 1.f;
    g.out_inv_scale = 1.f;
    g.qscale = 1.f;
    // QKV projection; Q columns scaled by 1/sqrt(64) = 1/8 (exact)
    g.A = fp8 ? (const void*)w.xq : w.x;
    g.W = L.wqkv;
    g.bias = L.bqkv;
    g.C = w.qkv;
    g.N = 3 * h;
    g.K = h;
    g.epi = EPI_BIAS;
    g.out = m->qkv_t;
    g.qscale = 0.125f;
    g.qcols = h;
    g.acc_scale = fp8 ? L.sa[0] * L.sw[0] : 1.f;
    g.config = m->gemm_cfg[0];
    g.group_m = m->gemm_gm[0];
    {
      ProfScope ps(KC_QKV, s, gemm_flops(T, 3 * h, h));
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    {
      ProfScope ps(KC_ATTN, s, 0.0);
      launch_attention(w.qkv, w.attn, w.qblocks, w.max_q, w.nq, c.n_heads, h, m->qkv_t, m->gemm_t,
                       fp8 ? 1.f / L.sa[1] : 1.f, m->attn_cfg, s);
    }
    // output projection + bias + residual -> FP32, then LayerNorm 1
    g.A = w.attn;
    g.W = L.wo;
    g.bias = L.bo;
    g.resid = w.x;
    g.res = m->act_t;
    g.C = w.y;
    g.out = m->act_t;
    g.N = h;
    g.K = h;
    g.epi = EPI_RESID;
    g.qscale = 1.f;
    g.qcols = 0;
    g.acc_scale = fp8 ? L.sa[1] * L.sw[1] : 1.f;
    g.config = m->gemm_cfg[1];
    g.group_m = m->gemm_gm[1];
    {
      ProfScope ps(KC_OPROJ, s, gemm_flops(T, h, h));
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    {
      ProfScope ps(KC_LN, s, 0.0);
      launch_layernorm(w.y, m->act_t, L.ln1_g, L.ln1_b, c.ln_eps, T, h, w.x2, m->act_t, w.xq, fp8 ? 1.f / L.sa[2] : 1.f, s,
                       t_dev);
    }
    // FFN1 + bias + GELU
    g.A = fp8 ? (const void*)w.xq : w.x2;
    g.W = L.w1;
    g.bias = L.b1;
    g.resid = nullptr;
    g.C = w.ffn;
    g.out = m->gemm_t;
    g.N = f;
    g.K = h;
    g.epi = EPI_GELU;
    g.acc_scale = fp8 ? L.sa[2] * L.sw[2] : 1.f;
    g.out_inv_scale = fp8 ? 1.f / L.sa[3] : 1.f;
    g.config = m->gemm_cfg[2];
    g.group_m = m->gemm_gm[2];
    {
      ProfScope ps(KC_FFN1, s, gemm_flops(T, f, h));
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    // FFN2 + bias + residual -> FP32, then LayerNorm 2
    g.A = w.ffn;
    g.W = L.w2;
    g.bias = L.b2;
    g.resid = w.x2;
    g.res = m->act_t;
    g.C = w.y;
    g.out = m->act_t;
    g.N = h;
    g.K = f;
    g.epi = EPI_RESID;
    g.acc_scale = fp8 ? L.sa[3] * L.sw[3] : 1.f;
    g.out_inv_scale = 1.f;
    g.config = m->gemm_cfg[3];
    g.group_m = m->gemm_gm[3];
    {
      ProfScope ps(KC_FFN2, s, gemm_flops(T, h, f));
      if (!launch_gemm(g, s)) return ANON_EINVAL;
    }
    {
      ProfScope ps(KC_LN, s, 0.0);
      const float nxt = (fp8 && l + 1 < c.n_layers) ? 1.f / m->layers[l + 1].sa[0] : 1.f;
      launch_layernorm(w.y, m->act_t, L.ln2_g, L.ln2_b, c.ln_eps, T, h, w.x, m->act_t, fp8 ? w.xq : nullptr, nxt, s,
                       t_dev);
    }
  }
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

static size_t enc_ws_bytes(const anon_model* m, int T, int B) {
  Carver k(nullptr, SIZE_MAX);
  EncWs w;
  enc_layout(m, T, B, k, w);
  return k.used + 256;
}

extern "C" {

anon_status anon_ner_workspace_size(const anon_model* m, int32_t T, int32_t B, size_t* bytes) {
  if (!m || !bytes || T < 0 || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  *bytes = enc_ws_bytes(m, T, B);
  return ANON_OK;
}

}  // extern "C"

// The forward for B records and T tokens; with t_dev, B and T are capacities
// and the kernels compute the *t_dev tokens that cu_seqlens lays out.
static anon_status forward(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B, int32_t T,
                           const int32_t* t_dev, uint8_t* d_labels, float* d_logits, float* d_margin,
                           void* d_workspace, size_t ws_bytes, hipStream_t s) {
  anon_status st = check_batch(m, d_ids, d_cu_seqlens, B, T);
  if (st != ANON_OK) return st;
  if (T == 0) return ANON_OK;
  if (!d_labels) return set_error(ANON_EINVAL, "labels is NULL");
  if (!d_workspace || ws_bytes < enc_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  Carver k(d_workspace, ws_bytes);
  EncWs w;
  enc_layout(m, T, B, k, w);
  st = run_encoder(m, d_ids, d_cu_seqlens, B, T, m->cfg.n_layers, w, s, t_dev);
  if (st != ANON_OK) return st;
  {
    ProfScope ps(KC_CLS, s, gemm_flops(T, m->cfg.n_labels, m->cfg.hidden));
    launch_classifier(w.x, m->act_t, m->wc_t, m->bc, T, m->cfg.hidden, m->cfg.n_labels, d_labels, d_logits,
                      d_margin, s, t_dev);
  }
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

extern "C" {

anon_status ner_forward(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B, int32_t T,
                        uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace, size_t ws_bytes,
                        void* stream) {
  clear_error();
  return forward(m, d_ids, d_cu_seqlens, B, T, nullptr, d_labels, d_logits, d_margin, d_workspace, ws_bytes,
                 (hipStream_t)stream);
}

// The layer stack as one HIP graph: ner_forward recorded on a private
// stream and instantiated once, so that a batch shape seen again costs one
// launch instead of one per kernel.  The forward makes no host round trip
// and allocates nothing once the device error word exists, and every
// clear is a kernel, so the recording holds kernel nodes only.
struct anon_graph {
  int device;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

}  // extern "C"

// Records the forward on a private stream and instantiates it.
static anon_status capture_forward(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                                   int32_t T, const int32_t* t_dev, uint8_t* d_labels, float* d_logits,
                                   float* d_margin, void* d_workspace, size_t ws_bytes, anon_graph** out) {
  if (!out) return set_error(ANON_EINVAL, "out is NULL");
  *out = nullptr;
  anon_status st = check_batch(m, d_ids, d_cu_seqlens, B, T);
  if (st != ANON_OK) return st;
  if (T == 0) return set_error(ANON_EINVAL, "nothing to capture: the batch has no tokens");
  if (!d_labels) return set_error(ANON_EINVAL, "labels is NULL");
  if (!d_workspace || ws_bytes < enc_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  for (int kc = 0; kc < KC_COUNT; ++kc)
    if (g_prof.enabled[kc]) return set_error(ANON_EINVAL, "kernel timing is enabled; disable it to capture");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  if (!error_word_ptr()) return set_error(ANON_EDEVICE, "cannot allocate the device error word");
  hipStream_t cs;
  ANON_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return set_error(ANON_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  st = forward(m, d_ids, d_cu_seqlens, B, T, t_dev, d_labels, d_logits, d_margin, d_workspace, ws_bytes, cs);
  const std::string fwd_err = anon_last_error();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (st != ANON_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (st != ANON_OK) return set_error(st, "capture: " + fwd_err);
    return set_error(ANON_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(ANON_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *out = new anon_graph{m->device, g, x};
  return ANON_OK;
}

extern "C" {

anon_status ner_forward_capture(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                                int32_t T, uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                                size_t ws_bytes, anon_graph** out) {
  clear_error();
  return capture_forward(m, d_ids, d_cu_seqlens, B, T, nullptr, d_labels, d_logits, d_margin, d_workspace,
                         ws_bytes, out);
}

anon_status ner_forward_capture_bucket(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens,
                                       const int32_t* d_n_tokens, int32_t B_cap, int32_t T_cap, uint8_t* d_labels,
                                       float* d_logits, float* d_margin, void* d_workspace, size_t ws_bytes,
                                       anon_graph** out) {
  clear_error();
  if (!d_n_tokens) return set_error(ANON_EINVAL, "n_tokens is NULL");
  if (B_cap < 1 || T_cap < 1) return set_error(ANON_EINVAL, "bucket capacities must be positive");
  return capture_forward(m, d_ids, d_cu_seqlens, B_cap, T_cap, d_n_tokens, d_labels, d_logits, d_margin,
                         d_workspace, ws_bytes, out);
}

anon_status anon_graph_launch(anon_graph* g, void* stream) {
  clear_error();
  if (!g) return set_error(ANON_EINVAL, "graph is NULL");
  ANON_HIP_CHECK(hipSetDevice(g->device));
  ANON_HIP_CHECK(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return ANON_OK;
}

void anon_graph_free(anon_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
}

static ElemType prec_type(anon_precision p) {
  return p == ANON_FP32 ? ET_F32 : (p == ANON_BF16 ? ET_BF16 : ET_FP8);
}

int32_t anon_tile_config_count(anon_precision precision) { return gemm_num_configs(prec_type(precision)); }

const char* anon_tile_config_name(anon_precision precision, int32_t config) {
  return gemm_config_name(prec_type(precision), config);
}

anon_status anon_model_set_tiles(anon_model* m, const int32_t tiles[4]) {
  if (!m || !tiles) return set_error(ANON_EINVAL, "NULL argument");
  const int h = m->cfg.hidden, f = m->cfg.ffn;
  const int NK[4][2] = {{3 * h, h}, {h, h}, {f, h}, {h, f}};
  for (int i = 0; i < 4; ++i)
    if (tiles[i] >= 0 && !gemm_config_fits(m->gemm_t, tiles[i], NK[i][0], NK[i][1]))
      return set_error(ANON_EINVAL, "tile configuration does not fit GEMM " + std::to_string(i));
  for (int i = 0; i < 4; ++i) m->gemm_cfg[i] = tiles[i];
  return ANON_OK;
}

anon_status anon_model_set_tile_groups(anon_model* m, const int32_t groups[4]) {
  if (!m || !groups) return set_error(ANON_EINVAL, "NULL argument");
  for (int i = 0; i < 4; ++i)
    if (groups[i] < 0 || groups[i] > 1024) return set_error(ANON_EINVAL, "tile group must be in [0, 1024]");
  for (int i = 0; i < 4; ++i) m->gemm_gm[i] = groups[i];
  return ANON_OK;
}

anon_status anon_model_get_tiles(const anon_model* m, int32_t tiles[4], int32_t groups[4]) {
  if (!m) return set_error(ANON_EINVAL, "NULL argument");
  for (int i = 0; i < 4; ++i) {
    if (tiles) tiles[i] = m->gemm_cfg[i];
    if (groups) groups[i] = m->gemm_gm[i];
  }
  return ANON_OK;
}

anon_status anon_autotune(anon_model* m, int32_t T, void* d_workspace, size_t ws_bytes, void* stream,
                          int32_t* chosen, float* times_ms, int32_t max_configs) {
  clear_error();
  if (!m || T < 1) return set_error(ANON_EINVAL, "bad arguments");
  if (!d_workspace || ws_bytes < enc_ws_bytes(m, T, 1)) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  Carver k(d_workspace, ws_bytes);
  EncWs w;
  enc_layout(m, T, 1, k, w);
  launch_fill_u8((uint8_t*)d_workspace, 0, (int64_t)k.used, s);  // finite operands
  const anon_model_config& c = m->cfg;
  const int h = c.hidden, f = c.ffn;
  const bool fp8 = m->gemm_t == ET_FP8;
  const LayerW& L = m->layers[0];
  hipEvent_t e0, e1;
  ANON_HIP_CHECK(hipEventCreate(&e0));
  ANON_HIP_CHECK(hipEventCreate(&e1));
  const int ncfg = gemm_num_configs(m->gemm_t);
  anon_status st = ANON_OK;
  for (int gi = 0; gi < 4 && st == ANON_OK; ++gi) {
    GemmParams g{};
    g.M = T;
    g.in = m->gemm_t;
    g.acc_scale = 1.f;
    g.out_inv_scale = 1.f;
    g.qscale = 1.f;
    if (gi == 0) {
      g.A = fp8 ? (const void*)w.xq : w.x;
      g.W = L.wqkv, g.bias = L.bqkv, g.C = w.qkv, g.N = 3 * h, g.K = h, g.epi = EPI_BIAS, g.out = m->qkv_t;
    } else if (gi == 1) {
      g.A = w.attn, g.W = L.wo, g.bias = L.bo, g.resid = w.x, g.res = m->act_t, g.C = w.y, g.N = h, g.K = h;
      g.epi = EPI_RESID, g.out = m->act_t;
    } else if (gi == 2) {
      g.A = fp8 ? (const void*)w.xq : w.x2;
      g.W = L.w1, g.bias = L.b1, g.C = w.ffn, g.N = f, g.K = h, g.epi = EPI_GELU, g.out = m->gemm_t;
    } else {
      g.A = w.ffn, g.W = L.w2, g.bias = L.b2, g.resid = w.x2, g.res = m->act_t, g.C = w.y, g.N = h, g.K = f;
      g.epi = EPI_RESID, g.out = m->act_t;
    }
    // random operands: zeros would time the tiles at a lower power draw
    // (and higher clock) than real activations allow
    launch_fill_random(const_cast<void*>(g.A), g.in, (int64_t)T * g.K, 0x1234u + gi, s);
    if (g.epi == EPI_RESID) launch_fill_random(const_cast<void*>(g.resid), g.res, (int64_t)T * g.N, 0x5678u + gi, s);
    // two rounds over all configurations (5 timed launches each), keeping
    // each configuration's best mean; near-ties go to the default tile
    std::vector<float> best_ms(ncfg, 1e30f);
    for (int round = 0; round < 2 && st == ANON_OK; ++round) {
      for (int ci = 0; ci < ncfg; ++ci) {
        if (!gemm_config_fits(m->gemm_t, ci, g.N, g.K)) continue;
        g.config = ci;
        if (!launch_gemm(g, s)) {
          st = ANON_EINVAL;
          break;
        }
        const int reps = 5;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) launch_gemm(g, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          st = set_error(ANON_EDEVICE, "autotune: kernel failed");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best_ms[ci] = std::min(best_ms[ci], ms / reps);
      }
    }
    g.config = -1;
    const int def = default_gemm_config(g);
    int best_c = def;
    for (int ci = 0; ci < ncfg; ++ci) {
      const bool fits = gemm_config_fits(m->gemm_t, ci, g.N, g.K);
      if (times_ms && ci < max_configs) times_ms[gi * max_configs + ci] = fits ? best_ms[ci] : -1.f;
      if (!fits) continue;
      const float ref = best_c >= 0 ? best_ms[best_c] : 1e30f;
      const float margin = best_c == def ? 0.97f : 1.0f;
      if (best_ms[ci] < ref * margin) best_c = ci;
    }
    m->gemm_cfg[gi] = best_c;
    if (chosen) chosen[gi] = best_c;
    // then the tile order of that tile: groups of 2..12 row blocks against
    // the order by shape (kept unless another is at least 1% faster)
    if (st != ANON_OK) break;
    g.config = best_c;
    const int kGroups[] = {0, 2, 4, 6, 8, 12};
    constexpr int NG = (int)(sizeof(kGroups) / sizeof(int));
    float gbest[NG];
    for (int j = 0; j < NG; ++j) gbest[j] = 1e30f;
    for (int round = 0; round < 2 && st == ANON_OK; ++round) {
      for (int j = 0; j < NG; ++j) {
        g.group_m = kGroups[j];
        const int reps = 5;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) launch_gemm(g, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          st = set_error(ANON_EDEVICE, "autotune: kernel failed");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        gbest[j] = std::min(gbest[j], ms / reps);
      }
    }
    int gsel = 0;
    for (int j = 1; j < NG; ++j)
      if (gbest[j] < gbest[gsel] * (gsel == 0 ? 0.99f : 1.0f)) gsel = j;
    m->gemm_gm[gi] = kGroups[gsel];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ANON_HIP_CHECK(hipGetLastError());
  return st;
}

anon_status anon_autotune_attention(anon_model* m, const int32_t* d_cu_seqlens, int32_t B, int32_t T,
                                    void* d_workspace, size_t ws_bytes, void* stream, int32_t* chosen,
                                    float* times_ms, int32_t max_configs) {
  clear_error();
  if (!m || B < 1 || T < 1 || !d_cu_seqlens) return set_error(ANON_EINVAL, "bad arguments");
  if ((int64_t)T > (int64_t)B * m->cfg.max_pos) return set_error(ANON_EINVAL, "T exceeds B * max_pos");
  if (!d_workspace || ws_bytes < enc_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  const int ncfg = attn_num_configs();
  if (times_ms)
    for (int c = 0; c < max_configs; ++c) times_ms[c] = -1.f;
  if (m->qkv_t != ET_BF16) {
    if (chosen) *chosen = -1;
    return ANON_OK;
  }
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  Carver k(d_workspace, ws_bytes);
  EncWs w;
  enc_layout(m, T, B, k, w);
  const anon_model_config& c = m->cfg;
  launch_fill_random(w.qkv, ET_BF16, (int64_t)T * 3 * c.hidden, 0x9e37u, s);
  uint32_t* err = error_word_ptr();
  const bool fp8 = m->gemm_t == ET_FP8;
  hipEvent_t e0, e1;
  ANON_HIP_CHECK(hipEventCreate(&e0));
  ANON_HIP_CHECK(hipEventCreate(&e1));
  std::vector<float> best(ncfg, 1e30f);
  anon_status st = ANON_OK;
  for (int round = 0; round < 2 && st == ANON_OK; ++round) {
    for (int ci = 0; ci < ncfg; ++ci) {
      launch_attn_plan(d_cu_seqlens, B, T, c.max_pos, ET_BF16, ci, w.qblocks, w.max_q, w.nq, err, s);
      launch_attention(w.qkv, w.attn, w.qblocks, w.max_q, w.nq, c.n_heads, c.hidden, ET_BF16, m->gemm_t,
                       fp8 ? 1.f / m->layers[0].sa[1] : 1.f, ci, s);
      const int reps = 3;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r)
        launch_attention(w.qkv, w.attn, w.qblocks, w.max_q, w.nq, c.n_heads, c.hidden, ET_BF16, m->gemm_t,
                         fp8 ? 1.f / m->layers[0].sa[1] : 1.f, ci, s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = set_error(ANON_EDEVICE, "autotune: attention kernel failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best[ci] = std::min(best[ci], ms / reps);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ANON_OK) return st;
  // near-ties go to the default configuration
  int pick = 0;
  for (int ci = 1; ci < ncfg; ++ci)
    if (best[ci] < best[pick] * (pick == 0 ? 0.99f : 1.0f)) pick = ci;
  m->attn_cfg = pick;
  if (chosen) *chosen = pick;
  if (times_ms)
    for (int ci = 0; ci < std::min(ncfg, (int)max_configs); ++ci) times_ms[ci] = best[ci];
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

anon_status anon_model_set_attn_config(anon_model* m, int32_t config) {
  if (!m) return set_error(ANON_EINVAL, "model is NULL");
  if (config < -1 || config >= attn_num_configs()) return set_error(ANON_EINVAL, "no such attention configuration");
  m->attn_cfg = config;
  return ANON_OK;
}

int32_t anon_model_get_attn_config(const anon_model* m) { return m ? m->attn_cfg : -1; }
int32_t anon_attn_config_count(void) { return attn_num_configs(); }
const char* anon_attn_config_name(int32_t config) { return attn_config_name(config); }

anon_status anon_encoder_hidden(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens, int32_t B,
                                int32_t T, int32_t n_layers, float* d_hidden, void* d_workspace, size_t ws_bytes,
                                void* stream) {
  clear_error();
  anon_status st = check_batch(m, d_ids, d_cu_seqlens, B, T);
  if (st != ANON_OK) return st;
  if (n_layers < 0 || n_layers > m->cfg.n_layers) return set_error(ANON_EINVAL, "n_layers out of range");
  if (T == 0) return ANON_OK;
  if (!d_hidden) return set_error(ANON_EINVAL, "hidden is NULL");
  if (!d_workspace || ws_bytes < enc_ws_bytes(m, T, B)) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  Carver k(d_workspace, ws_bytes);
  EncWs w;
  enc_layout(m, T, B, k, w);
  st = run_encoder(m, d_ids, d_cu_seqlens, B, T, n_layers, w, s);
  if (st != ANON_OK) return st;
  launch_to_f32(w.x, m->act_t, d_hidden, (int64_t)T * m->cfg.hidden, s);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

// ------------------------------------------------------------- windows ----
struct WinPlan {
  std::vector<int4> win;  // (record, start, length, first window token)
  std::vector<int> rec0;  // [B+1] first window of each record
  std::vector<int> wcu;   // [n_windows+1]
  int n_tok = 0;
};

static anon_status plan_windows(const int32_t* h_cu, int B, int window, int stride, int max_pos, WinPlan& p) {
  if (!h_cu && B > 0) return set_error(ANON_EINVAL, "host cu_seqlens is NULL");
  if (window < 1 || window > max_pos) return set_error(ANON_EINVAL, "window must be in [1, max_pos]");
  if (stride < 1 || stride > window) return set_error(ANON_EINVAL, "stride must be in [1, window]");
  p.rec0.assign(B + 1, 0);
  p.wcu.assign(1, 0);
  if (B > 0 && h_cu[0] != 0) return set_error(ANON_EINVAL, "cu_seqlens[0] must be 0");
  for (int b = 0; b < B; ++b) {
    const int n = h_cu[b + 1] - h_cu[b];
    if (n < 0) return set_error(ANON_EINVAL, "cu_seqlens must be non-decreasing");
    p.rec0[b] = (int)p.win.size();
    int nw = 1;
    if (n > window) nw = 1 + (n - window + stride - 1) / stride;
    for (int k = 0; k < nw; ++k) {
      const int st = k * stride, len = std::min(window, n - st);
      p.win.push_back(int4{b, st, len, p.n_tok});
      p.n_tok += len;
      p.wcu.push_back(p.n_tok);
    }
  }
  p.rec0[B] = (int)p.win.size();
  return ANON_OK;
}

struct WinWs {
  int *w_ids, *w_cu, *rec0, *cu;  // cu: validated copy of the host cu_seqlens
  int4* win;
  uint8_t* w_labels;
  float *w_logits, *w_margin;
};

static void win_layout(const anon_model* m, const WinPlan& p, bool logits, Carver& k, WinWs& w, EncWs& e) {
  const int nw = (int)p.win.size();
  w.w_ids = k.take<int>(p.n_tok);
  w.cu = k.take<int>(p.rec0.size());
  w.w_cu = k.take<int>(nw + 1);
  w.rec0 = k.take<int>(p.rec0.size());
  w.win = k.take<int4>(nw);
  w.w_labels = k.take<uint8_t>(p.n_tok);
  w.w_logits = logits ? k.take<float>((size_t)p.n_tok * m->cfg.n_labels) : nullptr;
  w.w_margin = k.take<float>(p.n_tok);
  enc_layout(m, p.n_tok, nw, k, e);
}

anon_status anon_ner_windowed_workspace_size(const anon_model* m, const int32_t* h_cu_seqlens, int32_t B,
                                             int32_t window, int32_t stride, size_t* bytes) {
  if (!m || !bytes || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  WinPlan p;
  anon_status st = plan_windows(h_cu_seqlens, B, window, stride, m->cfg.max_pos, p);
  if (st != ANON_OK) return st;
  Carver k(nullptr, SIZE_MAX);
  WinWs w;
  EncWs e;
  win_layout(m, p, true, k, w, e);
  *bytes = k.used + 256;
  return ANON_OK;
}

anon_status ner_forward_windowed(anon_model* m, const int32_t* d_ids, const int32_t* d_cu_seqlens,
                                 const int32_t* h_cu_seqlens, int32_t B, int32_t T, int32_t window, int32_t stride,
                                 uint8_t* d_labels, float* d_logits, float* d_margin, void* d_workspace,
                                 size_t ws_bytes, void* stream) {
  clear_error();
  if (!m) return set_error(ANON_EINVAL, "model is NULL");
  if (B < 0 || T < 0 || (B > 0 && (!d_cu_seqlens || !h_cu_seqlens))) return set_error(ANON_EINVAL, "bad batch");
  if (B > 0 && h_cu_seqlens[B] != T) return set_error(ANON_EINVAL, "cu_seqlens[B] != T");
  if (T == 0) return ANON_OK;
  if (!d_ids || !d_labels) return set_error(ANON_EINVAL, "ids/labels is NULL");
  WinPlan p;
  anon_status st = plan_windows(h_cu_seqlens, B, window, stride, m->cfg.max_pos, p);
  if (st != ANON_OK) return st;
  Carver k(d_workspace, ws_bytes);
  WinWs w;
  EncWs e;
  win_layout(m, p, d_logits != nullptr, k, w, e);
  if (!d_workspace || !k.ok()) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  const int nw = (int)p.win.size();
  ANON_HIP_CHECK(hipMemcpyAsync(w.w_cu, p.wcu.data(), p.wcu.size() * 4, hipMemcpyHostToDevice, s));
  ANON_HIP_CHECK(hipMemcpyAsync(w.cu, h_cu_seqlens, (size_t)(B + 1) * 4, hipMemcpyHostToDevice, s));
  ANON_HIP_CHECK(hipMemcpyAsync(w.rec0, p.rec0.data(), p.rec0.size() * 4, hipMemcpyHostToDevice, s));
  ANON_HIP_CHECK(hipMemcpyAsync(w.win, p.win.data(), p.win.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  // the host vectors die with this call: make sure the copies have landed
  ANON_HIP_CHECK(hipStreamSynchronize(s));
  // gather and merge index with the validated host plan, never with device data
  launch_window_gather(d_ids, w.cu, w.win, nw, w.w_ids, s);
  st = run_encoder(m, w.w_ids, w.w_cu, nw, p.n_tok, m->cfg.n_layers, e, s);
  if (st != ANON_OK) return st;
  launch_classifier(e.x, m->act_t, m->wc_t, m->bc, p.n_tok, m->cfg.hidden, m->cfg.n_labels, w.w_labels, w.w_logits,
                    w.w_margin, s);
  launch_window_merge(w.cu, B, w.rec0, w.win, window, stride, w.w_labels, w.w_logits, w.w_margin,
                      m->cfg.n_labels, d_labels, d_logits, d_margin, T, s);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

// --------------------------------------------------------------- spans ----
static void dec_layout(int T, Carver& k, int** flags, int** excl, void** temp) {
  *flags = k.take<int>(std::max(T, 1));
  *excl = k.take<int>(T + 1);
  *temp = k.take<uint8_t>(scan_temp_bytes(T));
}

anon_status anon_decode_workspace_size(int32_t T, int32_t B, size_t* bytes) {
  if (!bytes || T < 0 || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  Carver k(nullptr, SIZE_MAX);
  int *f, *e;
  void* t;
  dec_layout(T, k, &f, &e, &t);
  *bytes = k.used + 256;
  return ANON_OK;
}

anon_status decode_spans(const uint8_t* d_labels, const int32_t* d_tok_off, const int32_t* d_cu_seqlens, int32_t B,
                         int32_t T, int32_t n_types, anon_span* d_spans, int32_t span_cap, int32_t* d_cu_spans,
                         void* d_workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (B < 0 || T < 0 || span_cap < 0) return set_error(ANON_EINVAL, "negative size");
  if (B == 0 && T != 0) return set_error(ANON_EINVAL, "T > 0 with no records");
  if (n_types < 1 || n_types > 127) return set_error(ANON_EINVAL, "n_types must be in [1, 127]");
  if (!d_cu_spans || (B > 0 && !d_cu_seqlens)) return set_error(ANON_EINVAL, "cu arrays are NULL");
  if (T > 0 && (!d_labels || !d_tok_off)) return set_error(ANON_EINVAL, "labels/tok_off is NULL");
  if (span_cap > 0 && !d_spans) return set_error(ANON_EINVAL, "spans is NULL");
  Carver k(d_workspace, ws_bytes);
  int *flags, *excl;
  void* temp;
  dec_layout(T, k, &flags, &excl, &temp);
  if (!d_workspace || !k.ok()) return set_error(ANON_ECAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* err = error_word_ptr();
  if (B == 0) {
    launch_fill_u8((uint8_t*)d_cu_spans, 0, 4, s);
    ANON_HIP_CHECK(hipGetLastError());
    return ANON_OK;
  }
  launch_bio_flags(d_labels, d_cu_seqlens, B, T, n_types, flags, err, s);
  launch_exclusive_scan_i32(flags, excl, T, temp, s);
  launch_bio_write(d_labels, d_tok_off, d_cu_seqlens, B, T, n_types, flags, excl, d_spans, span_cap, d_cu_spans,
                   err, s);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

// decode_spans_noalloc: the same kernels with their flag, offset and scan
// buffers in `scratch`, a device array sized for ANON_NOALLOC_MAX_TOKENS
// tokens.  Host code never passes the array's name to a kernel (that is a
// host-side stand-in): each device's own address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static constexpr size_t kNoAllocScratchBytes =
    (size_t)ANON_NOALLOC_MAX_TOKENS * 4 * 2 + ((size_t)ANON_NOALLOC_MAX_TOKENS / 256 + 64) * 8 + 4 * 256;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {nullptr};

static anon_status scratch_for_current_device(void** out) {
  int dev = 0;
  ANON_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return set_error(ANON_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(ANON_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ANON_OK;
}

anon_status decode_spans_noalloc(const uint8_t* d_labels, const int32_t* d_tok_off, const int32_t* d_cu_seqlens,
                                 int32_t B, int32_t T, int32_t n_types, anon_span* d_spans, int32_t span_cap,
                                 int32_t* d_cu_spans, void* stream) {
  clear_error();
  if (T > ANON_NOALLOC_MAX_TOKENS)
    return set_error(ANON_ECAPACITY, "decode_spans_noalloc: T = " + std::to_string(T) + " exceeds " +
                                         std::to_string(ANON_NOALLOC_MAX_TOKENS) + " tokens");
  if (T < 0) return set_error(ANON_EINVAL, "negative size");
  void* ws = nullptr;
  anon_status st = scratch_for_current_device(&ws);
  if (st != ANON_OK) return st;
  // the flags and offsets are fully rewritten by every call (no state to clear)
  return decode_spans(d_labels, d_tok_off, d_cu_seqlens, B, T, n_types, d_spans, span_cap, d_cu_spans, ws,
                      kNoAllocScratchBytes, stream);
}

anon_status anon_recognize_workspace_size(int64_t n_bytes, int32_t B, size_t* bytes) {
  if (!bytes || n_bytes < 0 || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  *bytes = recog_workspace_bytes(n_bytes);
  return ANON_OK;
}

anon_status recognize_spans(const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B, int64_t n_bytes,
                            const int32_t* h_rec_types, int32_t n_types, const anon_span* d_ner_spans,
                            const int32_t* d_ner_cu, int32_t ner_cap, anon_span* d_spans, int32_t span_cap,
                            int32_t* d_cu_spans, void* d_workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (B < 0 || n_bytes < 0 || span_cap < 0 || ner_cap < 0) return set_error(ANON_EINVAL, "negative size");
  if (B == 0 && n_bytes != 0) return set_error(ANON_EINVAL, "n_bytes > 0 with no records");
  if (n_bytes >= (int64_t(1) << 31) - 2) return set_error(ANON_EINVAL, "n_bytes must be below 2^31 - 2");
  if (n_types < 1 || n_types > 127) return set_error(ANON_EINVAL, "n_types must be in [1, 127]");
  if (!h_rec_types) return set_error(ANON_EINVAL, "rec_types is NULL");
  int rt[kNumRecognizers];
  for (int k = 0; k < kNumRecognizers; ++k) {
    rt[k] = h_rec_types[k];
    if (rt[k] < 0 || rt[k] > n_types) return set_error(ANON_EINVAL, "recognizer type outside [0, n_types]");
  }
  if (!d_cu_spans || !d_cu_bytes) return set_error(ANON_EINVAL, "cu arrays are NULL");
  if (n_bytes > 0 && !d_text) return set_error(ANON_EINVAL, "text is NULL");
  if (span_cap > 0 && !d_spans) return set_error(ANON_EINVAL, "spans is NULL");
  if (ner_cap > 0 && (!d_ner_spans || !d_ner_cu)) return set_error(ANON_EINVAL, "NER spans are NULL");
  Carver k(d_workspace, ws_bytes);
  const RecogBuffers w = recog_layout(n_bytes, k);
  if (!d_workspace || !k.ok()) return set_error(ANON_ECAPACITY, "workspace too small");
  launch_recognize(d_text, d_cu_bytes, B, n_bytes, rt, d_ner_spans, d_ner_cu, ner_cap, n_types, w, d_spans,
                   span_cap, d_cu_spans, error_word_ptr(), (hipStream_t)stream);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

anon_status anon_field_workspace_size(int64_t n_bytes, int32_t B, size_t* bytes) {
  if (!bytes || n_bytes < 0 || B < 0) return set_error(ANON_EINVAL, "bad arguments");
  *bytes = field_workspace_bytes(n_bytes);
  return ANON_OK;
}

anon_status field_spans(const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B, int64_t n_bytes,
                        const char* const* h_field_names, const int32_t* h_field_types, int32_t n_fields,
                        int32_t n_types, anon_span* d_spans, int32_t span_cap, int32_t* d_cu_spans,
                        void* d_workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (B < 0 || n_bytes < 0 || span_cap < 0) return set_error(ANON_EINVAL, "negative size");
  if (B == 0 && n_bytes != 0) return set_error(ANON_EINVAL, "n_bytes > 0 with no records");
  if (n_bytes >= (int64_t(1) << 31) - 2) return set_error(ANON_EINVAL, "n_bytes must be below 2^31 - 2");
  if (n_types < 1 || n_types > 127) return set_error(ANON_EINVAL, "n_types must be in [1, 127]");
  if (n_fields < 0 || n_fields > kFieldsMax) return set_error(ANON_EINVAL, "n_fields must be in [0, 64]");
  if (n_fields > 0 && (!h_field_names || !h_field_types)) return set_error(ANON_EINVAL, "field table is NULL");
  FieldTable ft{};
  ft.n = n_fields;
  for (int k = 0; k < n_fields; ++k) {
    const char* nm = h_field_names[k];
    if (!nm) return set_error(ANON_EINVAL, "field name is NULL");
    const size_t L = strlen(nm);
    if (L < 1 || L > (size_t)kFieldNameMax) return set_error(ANON_EINVAL, "field names must have 1..32 bytes");
    for (size_t i = 0; i < L; ++i)
      if (nm[i] == ':' || nm[i] == '\n') return set_error(ANON_EINVAL, "field names cannot hold ':' or newline");
    if (h_field_types[k] < 1 || h_field_types[k] > n_types) return set_error(ANON_EINVAL, "field type outside [1, n_types]");
    memcpy(ft.name[k], nm, L);
    ft.len[k] = (uint8_t)L;
    ft.type[k] = h_field_types[k];
  }
  if (!d_cu_spans || !d_cu_bytes) return set_error(ANON_EINVAL, "cu arrays are NULL");
  if (n_bytes > 0 && !d_text) return set_error(ANON_EINVAL, "text is NULL");
  if (span_cap > 0 && !d_spans) return set_error(ANON_EINVAL, "spans is NULL");
  Carver k(d_workspace, ws_bytes);
  const FieldBuffers w = field_layout(n_bytes, k);
  if (!d_workspace || !k.ok()) return set_error(ANON_ECAPACITY, "workspace too small");
  launch_field_spans(d_text, d_cu_bytes, B, n_bytes, ft, w, d_spans, span_cap, d_cu_spans, error_word_ptr(),
                     (hipStream_t)stream);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

}  // extern "C"

// ---------------------------------------------------------- pseudonyms ----
struct anon_pcache {
  int device;
  PcacheDev dev;
  int64_t capacity;
  void* mem = nullptr;
  std::atomic<uint32_t> calls{0};  // pseudonymize calls since creation or the last clear
};

extern "C" {

anon_status anon_pcache_create(const uint8_t* h_key, size_t key_len, int32_t slug_hex,
                               const char* const* type_names, int32_t n_types, int64_t capacity, int32_t device,
                               anon_pcache** out) {
  clear_error();
  if (!out) return set_error(ANON_EINVAL, "out is NULL");
  *out = nullptr;
  if (!h_key && key_len > 0) return set_error(ANON_EINVAL, "key is NULL");
  if (slug_hex < 0 || slug_hex > 64) return set_error(ANON_EINVAL, "slug length must be in [0, 64]");
  if (n_types < 1 || n_types > 127 || !type_names) return set_error(ANON_EINVAL, "n_types must be in [1, 127]");
  if (capacity < 0 || capacity > (int64_t(1) << 30)) return set_error(ANON_EINVAL, "capacity out of range");
  if (!hmac_selftest()) return set_error(ANON_EDEVICE, "SHA-256 known-answer test failed");
  std::vector<uint8_t> names;
  std::vector<int> offs(1, 0);
  for (int t = 0; t < n_types; ++t) {
    const char* nm = type_names[t];
    if (!nm) return set_error(ANON_EINVAL, "type name is NULL");
    const size_t L = strlen(nm);
    if (L == 0 || L > 32) return set_error(ANON_EINVAL, "type names must have 1..32 characters");
    for (size_t i = 0; i < L; ++i) {
      const char ch = nm[i];
      if (!((ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') || ch == '_'))
        return set_error(ANON_EINVAL, "type names may only hold A-Z, 0-9 and '_'");
      names.push_back((uint8_t)ch);
    }
    offs.push_back((int)names.size());
  }
  int ndev = 0;
  ANON_HIP_CHECK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(ANON_EINVAL, "no such device");
  ANON_HIP_CHECK(hipSetDevice(device));
  int64_t cap = 1024;
  while (cap < capacity) cap <<= 1;
  anon_pcache* p = new anon_pcache();
  p->device = device;
  p->capacity = cap;
  Carver lay(nullptr, SIZE_MAX);
  lay.take<uint8_t>(cap * pcache_entry_bytes());
  lay.take<uint8_t>(names.size());
  lay.take<int>(offs.size());
  lay.take<unsigned long long>(4);
  if (hipMalloc(&p->mem, lay.used) != hipSuccess) {
    delete p;
    return set_error(ANON_ENOMEM, "cannot allocate the pseudonym table");
  }
  Carver k(p->mem, lay.used);
  p->dev.table = k.take<uint8_t>(cap * pcache_entry_bytes());
  uint8_t* dn = k.take<uint8_t>(names.size());
  int* doff = k.take<int>(offs.size());
  p->dev.counters = k.take<unsigned long long>(4);
  p->dev.mask = (uint64_t)cap - 1;
  p->dev.slug = slug_hex;
  p->dev.n_types = n_types;
  p->dev.names = dn;
  p->dev.name_off = doff;
  p->dev.enabled = 1;
  sha256_hmac_midstates(h_key, key_len, p->dev.ipad, p->dev.opad);
  hipError_t e = hipMemset(p->mem, 0, lay.used);
  if (e == hipSuccess) e = hipMemcpy(dn, names.data(), names.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(doff, offs.data(), offs.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(p->mem);
    delete p;
    return set_error(ANON_EDEVICE, std::string("pcache upload: ") + hipGetErrorString(e));
  }
  *out = p;
  return ANON_OK;
}

void anon_pcache_free(anon_pcache* p) {
  if (!p) return;
  hipSetDevice(p->device);
  hipFree(p->mem);
  delete p;
}

anon_status anon_pcache_clear(anon_pcache* p, void* stream) {
  if (!p) return set_error(ANON_EINVAL, "cache is NULL");
  ANON_HIP_CHECK(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  launch_fill_u8(p->dev.table, 0, p->capacity * (int64_t)pcache_entry_bytes(), s);
  launch_fill_u8((uint8_t*)p->dev.counters, 0, 4 * sizeof(unsigned long long), s);
  ANON_HIP_CHECK(hipGetLastError());
  p->calls = 0;
  return ANON_OK;
}

anon_status anon_pcache_set_preserve(anon_pcache* p, const int32_t* h_types, int32_t n) {
  clear_error();
  if (!p) return set_error(ANON_EINVAL, "cache is NULL");
  if (n < 0 || (n > 0 && !h_types)) return set_error(ANON_EINVAL, "bad type list");
  uint32_t m[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const int t = h_types[i];
    if (t < 1 || t > p->dev.n_types) return set_error(ANON_EINVAL, "type outside [1, n_types]");
    m[t >> 5] |= 1u << (t & 31);
  }
  memcpy(p->dev.preserve, m, sizeof(m));
  return ANON_OK;
}

anon_status anon_pcache_export(anon_pcache* p, anon_mapping* h_out, int64_t cap, int64_t* n_entries) {
  clear_error();
  if (!p || !n_entries) return set_error(ANON_EINVAL, "NULL argument");
  if (cap < 0 || (cap > 0 && !h_out)) return set_error(ANON_EINVAL, "bad output buffer");
  ANON_HIP_CHECK(hipSetDevice(p->device));
  ANON_HIP_CHECK(hipDeviceSynchronize());
  // the table is read in chunks of 64 Ki entries (10 MiB), whatever its size;
  // an insert race can leave two entries for one entity: they are merged
  const int64_t chunk = 1 << 16;
  std::vector<PcacheEntryView> tab((size_t)std::min(chunk, std::max(p->capacity, (int64_t)1)));
  std::map<std::string, anon_mapping> merged;
  for (int64_t c0 = 0; c0 < p->capacity; c0 += chunk) {
    const int64_t cn = std::min(chunk, p->capacity - c0);
    ANON_HIP_CHECK(hipMemcpy(tab.data(), p->dev.table + c0 * (int64_t)sizeof(PcacheEntryView),
                             (size_t)cn * sizeof(PcacheEntryView), hipMemcpyDeviceToHost));
    for (int64_t ei = 0; ei < cn; ++ei) {
      const PcacheEntryView& e = tab[(size_t)ei];
      if (e.state != 2 || e.len > 96) continue;
      const std::string k((const char*)e.bytes, e.len);
      auto it = merged.find(k);
      if (it == merged.end()) {
        anon_mapping m{};
        m.type = e.type;
        m.len = (int32_t)e.len;
        memcpy(m.bytes, e.bytes, e.len);
        for (int w = 0; w < 8; ++w)
          for (int b = 0; b < 4; ++b) m.digest[4 * w + b] = (uint8_t)(e.digest[w] >> (24 - 8 * b));
        m.first_call = e.first;
        m.last_call = e.last;
        merged.emplace(k, m);
      } else {
        it->second.type = std::min(it->second.type, e.type);
        it->second.first_call = std::min(it->second.first_call, e.first);
        it->second.last_call = std::max(it->second.last_call, e.last);
      }
    }
  }
  std::vector<anon_mapping> out;
  out.reserve(merged.size());
  for (auto& kv : merged) out.push_back(kv.second);
  std::stable_sort(out.begin(), out.end(),
                   [](const anon_mapping& a, const anon_mapping& b) { return a.first_call < b.first_call; });
  *n_entries = (int64_t)out.size();
  for (int64_t i = 0; i < std::min(cap, (int64_t)out.size()); ++i) h_out[i] = out[(size_t)i];
  return ANON_OK;
}

anon_status anon_pcache_set_enabled(anon_pcache* p, int32_t enabled) {
  if (!p) return set_error(ANON_EINVAL, "cache is NULL");
  p->dev.enabled = enabled ? 1 : 0;
  return ANON_OK;
}

anon_status anon_pcache_stats(anon_pcache* p, int64_t* lookups, int64_t* hits, int64_t* entries) {
  if (!p) return set_error(ANON_EINVAL, "cache is NULL");
  ANON_HIP_CHECK(hipSetDevice(p->device));
  ANON_HIP_CHECK(hipDeviceSynchronize());
  unsigned long long c[4];
  ANON_HIP_CHECK(hipMemcpy(c, p->dev.counters, sizeof(c), hipMemcpyDeviceToHost));
  if (lookups) *lookups = (int64_t)c[0];
  if (hits) *hits = (int64_t)c[1];
  if (entries) *entries = (int64_t)c[2];
  return ANON_OK;
}

}  // extern "C"

static void ps_layout_ws(int B, int cap, Carver& k, int64_t** out_len, int64_t** sp_out, int** sp_plen,
                         int64_t** sp_in_end, uint8_t** dig, void** temp) {
  *out_len = k.take<int64_t>(std::max(B, 1));
  *sp_out = k.take<int64_t>(std::max(cap, 1));
  *sp_plen = k.take<int>(std::max(cap, 1));
  *sp_in_end = k.take<int64_t>(std::max(cap, 1));
  *dig = k.take<uint8_t>((size_t)std::max(cap, 1) * 32);
  *temp = k.take<uint8_t>(scan_temp_bytes(B));
}

extern "C" {

anon_status anon_pseudonymize_workspace_size(int32_t B, int32_t span_cap, size_t* bytes) {
  if (!bytes || B < 0 || span_cap < 0) return set_error(ANON_EINVAL, "bad arguments");
  Carver k(nullptr, SIZE_MAX);
  int64_t *a, *b, *d;
  int* c;
  uint8_t* g;
  void* t;
  ps_layout_ws(B, span_cap, k, &a, &b, &c, &d, &g, &t);
  *bytes = k.used + 256;
  return ANON_OK;
}

anon_status pseudonymize(anon_pcache* p, const uint8_t* d_text, const int64_t* d_cu_bytes, int32_t B,
                         const anon_span* d_spans, const int32_t* d_cu_spans, int32_t span_cap, uint8_t* d_out,
                         int64_t out_cap, int64_t* d_cu_out, void* d_workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return set_error(ANON_EINVAL, "cache is NULL");
  if (B < 0 || span_cap < 0 || out_cap < 0) return set_error(ANON_EINVAL, "negative size");
  if (!d_cu_out || (B > 0 && (!d_cu_bytes || !d_cu_spans || !d_text))) return set_error(ANON_EINVAL, "NULL array");
  if (span_cap > 0 && !d_spans) return set_error(ANON_EINVAL, "spans is NULL");
  if (out_cap > 0 && !d_out) return set_error(ANON_EINVAL, "out is NULL");
  Carver k(d_workspace, ws_bytes);
  int64_t *out_len, *sp_out, *sp_in_end;
  int* sp_plen;
  uint8_t* dig;
  void* temp;
  ps_layout_ws(B, span_cap, k, &out_len, &sp_out, &sp_plen, &sp_in_end, &dig, &temp);
  if (!d_workspace || !k.ok()) return set_error(ANON_ECAPACITY, "workspace too small");
  ANON_HIP_CHECK(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  uint32_t* err = error_word_ptr();
  PcacheDev dev = p->dev;
  dev.call = ++p->calls;
  launch_ps_layout(dev, d_cu_bytes, B, d_spans, d_cu_spans, span_cap, out_len, sp_out, sp_plen, sp_in_end, err, s);
  launch_exclusive_scan_i64(out_len, d_cu_out, B, temp, s);
  launch_ps_hash(dev, d_text, d_cu_bytes, B, d_spans, d_cu_spans, span_cap, sp_plen, dig, s);
  launch_ps_write(dev, d_text, d_cu_bytes, B, d_spans, d_cu_spans, span_cap, sp_out, sp_plen, sp_in_end, dig,
                  d_cu_out, d_out, out_cap, err, s);
  ANON_HIP_CHECK(hipGetLastError());
  return ANON_OK;
}

// -------------------------------------------------------------- timing ----
anon_status anon_prof_enable(int32_t kclass, int32_t enabled) {
  if (kclass < 0 || kclass >= KC_COUNT) return set_error(ANON_EINVAL, "unknown kernel class");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.enabled[kclass] = enabled != 0;
  g_prof.launches[kclass] = 0;
  g_prof.ms[kclass] = 0;
  g_prof.flops[kclass] = 0;
  return ANON_OK;
}

anon_status anon_prof_read(int32_t kclass, int64_t* launches, double* total_ms, double* flops) {
  if (kclass < 0 || kclass >= KC_COUNT) return set_error(ANON_EINVAL, "unknown kernel class");
  prof_drain();
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (launches) *launches = g_prof.launches[kclass];
  if (total_ms) *total_ms = g_prof.ms[kclass];
  if (flops) *flops = g_prof.flops[kclass];
  return ANON_OK;
}

}  // extern "C"
