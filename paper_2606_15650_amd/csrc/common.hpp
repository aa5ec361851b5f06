// Shared definitions of the gfx950 kernels and the host runtime of libanon.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/anon.h"

typedef __bf16 bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx2 __attribute__((ext_vector_type(2)));

// One FP8-E4M3 (OCP "fn") value in a byte.
struct fp8_t {
  uint8_t v;
};

namespace anon {

// Thread-local last error string; set_error returns `st` for chaining.
anon_status set_error(anon_status st, const std::string& msg);
void clear_error();

#define ANON_HIP_CHECK(expr)                                                             \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return ::anon::set_error(ANON_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

// Per-device error word (bits ANON_ERR_*): kernels that check device data
// take its address and raise bits instead of reading or writing out of bounds.
__device__ __forceinline__ void raise_error(uint32_t* err, uint32_t bit) {
  if (err) atomicOr(err, bit);
}

// Address of the current device's error word (allocated once per device),
// or the word set for the calling thread by set_thread_error_word.
uint32_t* error_word_ptr();
// Route the error bits of this thread's later launches to `w` (device
// memory, the caller's); nullptr restores the per-device word.
void set_thread_error_word(uint32_t* w);

constexpr int kWave = 64;

// Rows a launch computes: its capacity `cap` (the grid is sized for it), or,
// when `dev` is given, the count held in device memory clamped to [0, cap].
// A graph captured for a token bucket reads the batch's count this way.
__device__ __forceinline__ int live_rows(int cap, const int* dev) {
  return dev ? max(0, min(*dev, cap)) : cap;
}

__device__ __forceinline__ float bf16_to_float(bf16_t x) { return static_cast<float>(x); }
__device__ __forceinline__ bf16_t float_to_bf16(float x) { return static_cast<bf16_t>(x); }

// FP32 -> OCP E4M3FN, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3(float v) {
  v = fminf(fmaxf(v, -448.0f), 448.0f);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, v, 0, false) & 0xff);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// 16 bytes per lane from global memory straight into LDS
// (global_load_lds_dwordx4): lane i's bytes land at l + 16 i, where l is
// the same for the whole wave.
__device__ __forceinline__ void dma16(const void* g, char* l) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                   (__attribute__((address_space(3))) void*)l, 16, 0, 0);
}

// s_waitcnt vmcnt(n) alone (expcnt and lgkmcnt left at their maxima)
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carving: consecutive 256-byte aligned sub-buffers.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base((char*)b), cap(c) {}
  template <typename T>
  T* take(size_t n) {
    size_t off = align_up(used, 256);
    used = off + n * sizeof(T);
    return base ? (T*)(base + off) : nullptr;
  }
  bool ok() const { return used <= cap; }
};

// Kernel-class timing (anon_prof_*).
enum KClass { KC_QKV = 0, KC_ATTN, KC_OPROJ, KC_FFN1, KC_FFN2, KC_LN, KC_EMBED, KC_CLS, KC_COUNT };
struct ProfScope {
  int kc;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double flops;
  ProfScope(int kc, hipStream_t s, double flops);
  ~ProfScope();
};

}  // namespace anon
