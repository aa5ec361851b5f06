// Row-wise kernels of the encoder: embedding + LayerNorm, LayerNorm, the
// token-classification head (argmax and top-2 margin), type conversions and
// the window gather / owner-window merge for long records.
//
// A 64-lane wave owns a token row (LayerNorm: two rows); lane i holds VEC
// consecutive elements (4 where the row length allows) of each chunk of
// 64*VEC elements, so every load and store is a contiguous wave access (see
// RowMap).  LayerNorm statistics are
// FP32 and two-pass (mean, then mean of squared deviations) with a fixed
// butterfly reduction order, so a row's result never depends on the other
// rows of the batch.  The classifier runs on the FP32 matrix cores, 32
// tokens per wave.
#include <algorithm>

#include "kernels.hpp"

namespace anon {
namespace {

__device__ __forceinline__ float ldf(const float* p) { return *p; }
__device__ __forceinline__ float ldf(const bf16_t* p) { return static_cast<float>(*p); }

// Record containing packed token t (largest b with cu[b] <= t), robust to
// malformed cu_seqlens (the result is then only clamped, never out of range).
__device__ __forceinline__ int find_record(const int* cu, int B, int t) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cu[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A lane owns NPL elements of a row in chunks of VEC consecutive columns:
// element i sits at column (i / VEC) * 64 * VEC + lane * VEC + i % VEC, so
// every chunk is one 16-byte (fp32) or 8-byte (bf16) access and each wave
// access covers a contiguous span of the row.
template <int NPL>
struct RowMap {
  static constexpr int VEC = NPL % 4 == 0 ? 4 : NPL;
  __device__ static int col(int i, int lane) { return (i / VEC) * 64 * VEC + lane * VEC + i % VEC; }
};

template <int NPL>
__device__ __forceinline__ void load_row(const float* src, int lane, float (&v)[NPL]) {
  typedef RowMap<NPL> RM;
#pragma unroll
  for (int c = 0; c < NPL / RM::VEC; ++c) {
    if constexpr (RM::VEC == 4) {
      const floatx4 x = *(const floatx4*)(src + RM::col(c * 4, lane));
#pragma unroll
      for (int k = 0; k < 4; ++k) v[c * 4 + k] = x[k];
    } else {
#pragma unroll
      for (int k = 0; k < RM::VEC; ++k) v[c * RM::VEC + k] = src[RM::col(c * RM::VEC + k, lane)];
    }
  }
}

template <int NPL>
__device__ __forceinline__ void load_row(const bf16_t* src, int lane, float (&v)[NPL]) {
  typedef RowMap<NPL> RM;
#pragma unroll
  for (int c = 0; c < NPL / RM::VEC; ++c) {
    if constexpr (RM::VEC == 4) {
      const bf16x4 x = __builtin_nontemporal_load((const bf16x4*)(src + RM::col(c * 4, lane)));
#pragma unroll
      for (int k = 0; k < 4; ++k) v[c * 4 + k] = static_cast<float>(x[k]);
    } else {
#pragma unroll
      for (int k = 0; k < RM::VEC; ++k) v[c * RM::VEC + k] = static_cast<float>(src[RM::col(c * RM::VEC + k, lane)]);
    }
  }
}

// LayerNorm of the row in v (lane-owned elements, RowMap order) with gain gv
// and shift bv in the same order, written to row `row` of out (and out_q).
template <int NPL>
__device__ __forceinline__ void ln_store(float (&v)[NPL], const float (&gv)[NPL], const float (&bv)[NPL], float eps,
                                         int h, int lane, size_t row, void* out, ElemType out_t, fp8_t* out_q,
                                         float q_inv_scale) {
  typedef RowMap<NPL> RM;
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NPL; ++i) s += v[i];
  const float mean = wave_sum(s) / (float)h;
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const float d = v[i] - mean;
    q += d * d;
  }
  const float var = wave_sum(q) / (float)h;
  const float rstd = 1.0f / sqrtf(var + eps);
#pragma unroll
  for (int c = 0; c < NPL / RM::VEC; ++c) {
    float y[RM::VEC];
    const int c0 = RM::col(c * RM::VEC, lane);
#pragma unroll
    for (int k = 0; k < RM::VEC; ++k)
      y[k] = gv[c * RM::VEC + k] * ((v[c * RM::VEC + k] - mean) * rstd) + bv[c * RM::VEC + k];
    if (out_t == ET_F32) {
#pragma unroll
      for (int k = 0; k < RM::VEC; ++k) ((float*)out)[row * h + c0 + k] = y[k];
    } else {
      bf16_t yb[RM::VEC];
#pragma unroll
      for (int k = 0; k < RM::VEC; ++k) yb[k] = static_cast<bf16_t>(y[k]);
      if constexpr (RM::VEC == 4) {
        __builtin_nontemporal_store(bf16x4{yb[0], yb[1], yb[2], yb[3]}, (bf16x4*)((bf16_t*)out + row * h + c0));
      } else {
#pragma unroll
        for (int k = 0; k < RM::VEC; ++k) ((bf16_t*)out)[row * h + c0 + k] = yb[k];
      }
      if (out_q) {
#pragma unroll
        for (int k = 0; k < RM::VEC; ++k)
          out_q[row * h + c0 + k].v = f32_to_e4m3(static_cast<float>(yb[k]) * q_inv_scale);
      }
    }
  }
}

template <int NPL>
__global__ __launch_bounds__(256) void embed_ln_kernel(const int* __restrict__ ids, const int* __restrict__ cu,
                                                       int B, int T_cap, const float* __restrict__ tok,
                                                       const float* __restrict__ pos, const float* __restrict__ g,
                                                       const float* __restrict__ b, float eps, int vocab,
                                                       int max_pos, void* out, ElemType out_t, fp8_t* out_q,
                                                       float q_inv_scale, int* pos_out, uint32_t* err,
                                                       const int* t_dev) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= live_rows(T_cap, t_dev)) return;
  constexpr int h = NPL * 64;
  int id = ids[t];
  if (id < 0 || id >= vocab) {
    if (lane == 0) raise_error(err, ANON_ERR_TOKEN_ID);
    id = 0;
  }
  const int r = find_record(cu, B, t);
  const int p = min(max(t - cu[r], 0), max_pos - 1);
  if (pos_out && lane == 0) pos_out[t] = p;
  float v[NPL];
  load_row<NPL>(tok + (size_t)id * h, lane, v);
  if (pos) {  // learned absolute positions (no table: positions enter elsewhere)
    float w[NPL];
    load_row<NPL>(pos + (size_t)p * h, lane, w);
#pragma unroll
    for (int i = 0; i < NPL; ++i) v[i] += w[i];
  }
  float gv[NPL], bv[NPL];
  load_row<NPL>(g, lane, gv);
  load_row<NPL>(b, lane, bv);
  ln_store<NPL>(v, gv, bv, eps, h, lane, t, out, out_t, out_q, q_inv_scale);
}

// RPW rows per wave: every row's loads are issued before the first
// reduction, so more bytes are in flight per wave.
template <typename TY, int NPL, int RPW>
__global__ __launch_bounds__(256) void layernorm_kernel(const TY* __restrict__ y, const float* __restrict__ g,
                                                        const float* __restrict__ b, float eps, int rows_cap,
                                                        void* out, ElemType out_t, fp8_t* out_q, float q_inv_scale,
                                                        const int* rows_dev) {
  const int lane = threadIdx.x & 63;
  const int rows = live_rows(rows_cap, rows_dev);
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
  if (row0 >= rows) return;
  constexpr int h = NPL * 64;
  float v[RPW][NPL], gv[NPL], bv[NPL];
#pragma unroll
  for (int k = 0; k < RPW; ++k)
    if (row0 + k < rows) load_row<NPL>(y + (size_t)(row0 + k) * h, lane, v[k]);
  load_row<NPL>(g, lane, gv);
  load_row<NPL>(b, lane, bv);
#pragma unroll
  for (int k = 0; k < RPW; ++k)
    if (row0 + k < rows) ln_store<NPL>(v[k], gv, bv, eps, h, lane, row0 + k, out, out_t, out_q, q_inv_scale);
}

constexpr int kMaxLabels = 64;
#ifndef ANON_LN_RPW
#define ANON_LN_RPW 2
#endif

// Token classifier on the FP32 matrix cores (C <= 32 labels): one wave forms
// z^T = Wc x^T for 32 tokens with v_mfma_f32_32x32x2_f32, exact products of
// the FP32 head and the (bf16 or FP32) hidden state, FP32 sums.  Lane half hh
// feeds the k-index hh of every MFMA from its own 16-element slice of each
// 32-column chunk.  Then lane l holds the logits of token (l & 31) for
// classes (r/4)*8 + hh*4 + r%4 of register r; the two halves merge their
// top-2 with one exchange (ties to the lowest class index).
template <typename TX, int H>
__global__ __launch_bounds__(256) void classifier_mfma_kernel(const TX* __restrict__ x, const float* __restrict__ wc,
                                                              const float* __restrict__ bc, int T_cap, int C,
                                                              uint8_t* __restrict__ labels,
                                                              float* __restrict__ logits, float* __restrict__ margin,
                                                              const int* t_dev) {
  const int lane = threadIdx.x & 63;
  const int T = live_rows(T_cap, t_dev);
  const int t0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
  if (t0 >= T) return;
  const int hh = lane >> 5, r32 = lane & 31;
  const int tok = min(t0 + r32, T - 1);  // rows past T re-read row T-1, never stored
  const bool cvalid = r32 < C;
  const TX* xr = x + (size_t)tok * H + hh * 16;
  const float* wr = wc + (size_t)(cvalid ? r32 : 0) * H + hh * 16;
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int kc = 0; kc < H / 32; ++kc) {
    float xv[16], wv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) xv[e] = ldf(xr + kc * 32 + e);
#pragma unroll
    for (int e = 0; e < 16; e += 4) {
      const floatx4 w4 = *(const floatx4*)(wr + kc * 32 + e);
#pragma unroll
      for (int k = 0; k < 4; ++k) wv[e + k] = cvalid ? w4[k] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wv[e], xv[e], acc, 0, 0, 0);
  }
  float best = -INFINITY, second = -INFINITY;
  int arg = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int c = (r >> 2) * 8 + hh * 4 + (r & 3);  // increasing in r
    if (c < C) {
      const float z = acc[r] + bc[c];
      if (logits && t0 + r32 < T) logits[(size_t)(t0 + r32) * C + c] = z;
      if (z > best) {
        second = best;
        best = z;
        arg = c;
      } else if (z > second) {
        second = z;
      }
    }
  }
  const float ob = __shfl_xor(best, 32, 64), os = __shfl_xor(second, 32, 64);
  const int oa = __shfl_xor(arg, 32, 64);
  if (hh == 0 && t0 + r32 < T) {
    float b1, b2;
    int a1;
    if (best > ob) {
      b1 = best, a1 = arg, b2 = fmaxf(second, ob);
    } else if (ob > best) {
      b1 = ob, a1 = oa, b2 = fmaxf(os, best);
    } else {
      b1 = best, a1 = min(arg, oa), b2 = best;
    }
    labels[t0 + r32] = (uint8_t)a1;
    if (margin) margin[t0 + r32] = C > 1 ? b1 - b2 : INFINITY;
  }
}

template <typename TX, int NPL>
__global__ __launch_bounds__(256) void classifier_kernel(const TX* __restrict__ x, const float* __restrict__ wc,
                                                         const float* __restrict__ bc, int T_cap, int C,
                                                         uint8_t* __restrict__ labels, float* __restrict__ logits,
                                                         float* __restrict__ margin, const int* t_dev) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= live_rows(T_cap, t_dev)) return;
  constexpr int h = NPL * 64;
  float xv[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) xv[i] = ldf(x + (size_t)t * h + lane + 64 * i);
  float best = -INFINITY, second = -INFINITY, mine = 0.f;
  int arg = 0;
  for (int c = 0; c < C; ++c) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < NPL; ++i) s += xv[i] * wc[(size_t)c * h + lane + 64 * i];
    const float z = wave_sum(s) + bc[c];
    if (lane == c) mine = z;
    if (z > best) {
      second = best;
      best = z;
      arg = c;
    } else if (z > second) {
      second = z;
    }
  }
  if (logits && lane < C) logits[(size_t)t * C + lane] = mine;
  if (lane == 0) {
    labels[t] = (uint8_t)arg;
    if (margin) margin[t] = C > 1 ? best - second : INFINITY;
  }
}

template <typename TX>
__global__ void to_f32_kernel(const TX* __restrict__ x, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ldf(x + i);
}

// FP32 -> bf16, four elements per thread (n a multiple of 4)
__global__ void f32_to_bf16_kernel(const float* __restrict__ x, bf16_t* __restrict__ out, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const floatx4 v = *(const floatx4*)(x + 4 * i);
  *(bf16x4*)(out + 4 * i) = bf16x4{static_cast<bf16_t>(v[0]), static_cast<bf16_t>(v[1]), static_cast<bf16_t>(v[2]),
                                   static_cast<bf16_t>(v[3])};
}

// dst[c][r] = src[r][c] * inv_scale, converted to the storage type.
template <typename TD>
__global__ __launch_bounds__(256) void transpose_convert_kernel(const float* __restrict__ src, int rows, int cols,
                                                                TD* __restrict__ dst, float inv_scale) {
  __shared__ float tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < rows && c < cols) ? src[(size_t)r * cols + c] : 0.f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < cols && r < rows) {
      const float v = tile[tx][k] * inv_scale;
      if constexpr (sizeof(TD) == 4) dst[(size_t)c * rows + r] = v;
      else if constexpr (sizeof(TD) == 2) dst[(size_t)c * rows + r] = static_cast<bf16_t>(v);
      else dst[(size_t)c * rows + r].v = f32_to_e4m3(v);
    }
  }
}

__global__ void window_gather_kernel(const int* __restrict__ ids, const int* __restrict__ cu,
                                     const int4* __restrict__ win, int* __restrict__ w_ids) {
  const int4 w = win[blockIdx.x];  // (record, start in record, length, first window token)
  const int src = cu[w.x] + w.y;
  for (int i = threadIdx.x; i < w.z; i += blockDim.x) w_ids[w.w + i] = ids[src + i];
}

__global__ void window_merge_kernel(const int* __restrict__ cu, int B, const int* __restrict__ rec_win0,
                                    const int4* __restrict__ win, int window, int stride,
                                    const uint8_t* __restrict__ wl, const float* __restrict__ wz,
                                    const float* __restrict__ wm, int C, uint8_t* __restrict__ labels,
                                    float* __restrict__ logits, float* __restrict__ margin, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int b = find_record(cu, B, t);
  const int i = t - cu[b];
  const int nw = rec_win0[b + 1] - rec_win0[b];
  const int half = (window - stride) / 2;
  int k = i >= half ? (i - half) / stride : 0;
  k = min(k, nw - 1);
  const int4 w = win[rec_win0[b] + k];
  const int src = w.w + (i - w.y);
  labels[t] = wl[src];
  if (margin) margin[t] = wm[src];
  if (logits)
    for (int c = 0; c < C; ++c) logits[(size_t)t * C + c] = wz[(size_t)src * C + c];
}

__global__ void fill_u8_kernel(uint8_t* p, uint8_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Values uniform in [-1, 1) from a 32-bit integer hash of the element index
// (the "lowbias32" mixer of Chris Wellons' hash-prospector): operands with
// the bit statistics of real activations, so that timed kernels draw the
// power (and run at the clock) they do on real data.
__global__ void fill_random_kernel(void* p, ElemType t, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    const float v = (float)(x >> 8) * (1.0f / 8388608.0f) - 1.0f;
    if (t == ET_F32) ((float*)p)[i] = v;
    else if (t == ET_BF16) ((bf16_t*)p)[i] = static_cast<bf16_t>(v);
    else ((fp8_t*)p)[i].v = f32_to_e4m3(v);
  }
}

#define ANON_NPL_SWITCH(NPLV, ...)            \
  switch (NPLV) {                             \
    case 1: { constexpr int NPL = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int NPL = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int NPL = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int NPL = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int NPL = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int NPL = 16; __VA_ARGS__; } break; \
    default: break;                           \
  }

}  // namespace

void launch_embed_ln(const int* ids, const int* cu_seqlens, int B, int T, const float* tok_emb, const float* pos_emb,
                     const float* g, const float* b, float eps, int vocab, int max_pos, int h, void* out,
                     ElemType out_t, fp8_t* out_q, float q_inv_scale, uint32_t* err, hipStream_t s, int* pos_out,
                     const int* t_dev) {
  if (T <= 0) return;
  ANON_NPL_SWITCH(h / 64, hipLaunchKernelGGL((embed_ln_kernel<NPL>), dim3(ceil_div(T, 4)), dim3(256), 0, s, ids,
                                             cu_seqlens, B, T, tok_emb, pos_emb, g, b, eps, vocab, max_pos, out,
                                             out_t, out_q, q_inv_scale, pos_out, err, t_dev));
}

void launch_f32_to_bf16(const float* x, bf16_t* out, int64_t n, hipStream_t s) {
  const int64_t n4 = n / 4;
  if (n4 <= 0) return;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, x, out, n4);
}

void launch_layernorm(const void* y, ElemType y_t, const float* g, const float* b, float eps, int rows, int h,
                      void* out, ElemType out_t, fp8_t* out_q, float q_inv_scale, hipStream_t s,
                      const int* rows_dev) {
  if (rows <= 0) return;
  constexpr int RPW = ANON_LN_RPW;
  const int blocks = ceil_div(rows, 4 * RPW);
  if (y_t == ET_F32) {
    ANON_NPL_SWITCH(h / 64, hipLaunchKernelGGL((layernorm_kernel<float, NPL, RPW>), dim3(blocks), dim3(256), 0, s,
                                               (const float*)y, g, b, eps, rows, out, out_t, out_q, q_inv_scale,
                                               rows_dev));
  } else {
    ANON_NPL_SWITCH(h / 64, hipLaunchKernelGGL((layernorm_kernel<bf16_t, NPL, RPW>), dim3(blocks), dim3(256), 0, s,
                                               (const bf16_t*)y, g, b, eps, rows, out, out_t, out_q, q_inv_scale,
                                               rows_dev));
  }
}

void launch_classifier(const void* x, ElemType x_t, const float* wc_t, const float* bc, int T, int h, int C,
                       uint8_t* labels, float* logits, float* margin, hipStream_t s, const int* t_dev) {
  if (T <= 0) return;
  if (C <= 32) {
    const int blocks = ceil_div(ceil_div(T, 32), 4);
#define ANON_CLS_MFMA(HV)                                                                                        \
  case HV:                                                                                                       \
    if (x_t == ET_F32)                                                                                           \
      hipLaunchKernelGGL((classifier_mfma_kernel<float, HV>), dim3(blocks), dim3(256), 0, s, (const float*)x,    \
                         wc_t, bc, T, C, labels, logits, margin, t_dev);                                         \
    else                                                                                                         \
      hipLaunchKernelGGL((classifier_mfma_kernel<bf16_t, HV>), dim3(blocks), dim3(256), 0, s, (const bf16_t*)x,  \
                         wc_t, bc, T, C, labels, logits, margin, t_dev);                                         \
    return;
    switch (h) {
      ANON_CLS_MFMA(128)
      ANON_CLS_MFMA(256)
      ANON_CLS_MFMA(512)
      ANON_CLS_MFMA(768)
      ANON_CLS_MFMA(1024)
      default:
        break;
    }
#undef ANON_CLS_MFMA
  }
  if (x_t == ET_F32) {
    ANON_NPL_SWITCH(h / 64, hipLaunchKernelGGL((classifier_kernel<float, NPL>), dim3(ceil_div(T, 4)), dim3(256), 0,
                                               s, (const float*)x, wc_t, bc, T, C, labels, logits, margin, t_dev));
  } else {
    ANON_NPL_SWITCH(h / 64, hipLaunchKernelGGL((classifier_kernel<bf16_t, NPL>), dim3(ceil_div(T, 4)), dim3(256), 0,
                                               s, (const bf16_t*)x, wc_t, bc, T, C, labels, logits, margin, t_dev));
  }
}

void launch_to_f32(const void* x, ElemType t, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int grid = ceil_div(n, 256);
  if (t == ET_F32) hipLaunchKernelGGL(to_f32_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)x, out, n);
  else hipLaunchKernelGGL(to_f32_kernel<bf16_t>, dim3(grid), dim3(256), 0, s, (const bf16_t*)x, out, n);
}

void launch_transpose_convert(const float* src, int rows, int cols, void* dst, ElemType t, float inv_scale,
                              hipStream_t s) {
  dim3 grid(ceil_div(cols, 32), ceil_div(rows, 32));
  if (t == ET_F32)
    hipLaunchKernelGGL(transpose_convert_kernel<float>, grid, dim3(256), 0, s, src, rows, cols, (float*)dst,
                       inv_scale);
  else if (t == ET_BF16)
    hipLaunchKernelGGL(transpose_convert_kernel<bf16_t>, grid, dim3(256), 0, s, src, rows, cols, (bf16_t*)dst,
                       inv_scale);
  else
    hipLaunchKernelGGL(transpose_convert_kernel<fp8_t>, grid, dim3(256), 0, s, src, rows, cols, (fp8_t*)dst,
                       inv_scale);
}

void launch_window_gather(const int* ids, const int* cu_seqlens, const int4* windows, int n_windows, int* w_ids,
                          hipStream_t s) {
  if (n_windows <= 0) return;
  hipLaunchKernelGGL(window_gather_kernel, dim3(n_windows), dim3(256), 0, s, ids, cu_seqlens, windows, w_ids);
}

void launch_window_merge(const int* cu_seqlens, int B, const int* rec_win0, const int4* windows, int window,
                         int stride, const uint8_t* w_labels, const float* w_logits, const float* w_margin, int C,
                         uint8_t* labels, float* logits, float* margin, int T, hipStream_t s) {
  if (T <= 0) return;
  hipLaunchKernelGGL(window_merge_kernel, dim3(ceil_div(T, 256)), dim3(256), 0, s, cu_seqlens, B, rec_win0, windows,
                     window, stride, w_labels, w_logits, w_margin, C, labels, logits, margin, T);
}

void launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u8_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, v, n);
}

void launch_fill_random(void* p, ElemType t, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 65536);
  hipLaunchKernelGGL(fill_random_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, t, n, seed);
}

}  // namespace anon
