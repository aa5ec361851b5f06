// BIO span decoding on the GPU, plus the device-wide exclusive scans that
// compact variable-length outputs.
//
// Decoding is token-parallel.  A token opens a span iff its label is not O
// and it is B-t, or it is the first token of its record, or the previous
// token's type differs (so an I-t without an open span of type t opens one).
// An exclusive scan of these flags gives every span its index in record-major
// order; the opening token then walks forward over the following I-t tokens
// of its record to find the span's last token.  Every token is visited by at
// most one walk, so the work is O(T).
#include "kernels.hpp"

namespace anon {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const T x = tid >= o ? sh[tid - o] : T(0);
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  const T incl = sh[tid];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const T* __restrict__ in, int64_t n,
                                                                   T* __restrict__ part) {
  __shared__ T sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  T total;
  block_exclusive_scan<T>(s, sh, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the per-tile sums; writes the grand
// total to out[n].
template <typename T>
__global__ __launch_bounds__(1024) void scan_parts_kernel(T* __restrict__ part, int nparts, T* __restrict__ out,
                                                          int64_t n) {
  __shared__ T sh[1024];
  const int tid = threadIdx.x;
  const int per = (nparts + 1023) / 1024;
  const int a = min(nparts, tid * per), b = min(nparts, a + per);
  T s = 0;
  for (int i = a; i < b; ++i) s += part[i];
  sh[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const T x = tid >= o ? sh[tid - o] : T(0);
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  T run = sh[tid] - s;
  for (int i = a; i < b; ++i) {
    const T v = part[i];
    part[i] = run;
    run += v;
  }
  if (tid == 1023) out[n] = sh[1023];
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const T* __restrict__ in, int64_t n,
                                                                  const T* __restrict__ part, T* __restrict__ out) {
  __shared__ T sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : T(0);
    s += v[i];
  }
  T total;
  T run = block_exclusive_scan<T>(s, sh, &total) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

template <typename T>
void exclusive_scan(const T* in, T* out, int64_t n, void* temp, hipStream_t s) {
  const int nparts = (int)((n + kScanTile - 1) / kScanTile);
  T* part = (T*)temp;
  if (nparts > 0) hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3(nparts), dim3(kScanThreads), 0, s, in, n, part);
  hipLaunchKernelGGL(scan_parts_kernel<T>, dim3(1), dim3(1024), 0, s, part, nparts, out, n);
  if (nparts > 0)
    hipLaunchKernelGGL(scan_apply_kernel<T>, dim3(nparts), dim3(kScanThreads), 0, s, in, n, (const T*)part, out);
}

__device__ __forceinline__ int find_record(const int* cu, int B, int t) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cu[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int clean_label(int lab, int n_types, uint32_t* err) {
  if (lab > 2 * n_types) {
    raise_error(err, ANON_ERR_LABEL);
    return 0;
  }
  return lab;
}

__global__ void bio_flags_kernel(const uint8_t* __restrict__ labels, const int* __restrict__ cu, int B, int T,
                                 int n_types, int* __restrict__ flags, uint32_t* err) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int lab = clean_label(labels[t], n_types, err);
  int f = 0;
  if (lab != 0) {
    const int b = find_record(cu, B, t);
    const int typ = (lab + 1) >> 1;
    bool open = (lab & 1) || t == cu[b] || t == 0;
    if (!open) {
      const int pl = labels[t - 1];
      const int ptyp = pl > 2 * n_types ? 0 : (pl + 1) >> 1;
      open = ptyp != typ;
    }
    f = open ? 1 : 0;
  }
  flags[t] = f;
}

__global__ void bio_write_kernel(const uint8_t* __restrict__ labels, const int* __restrict__ tok_off,
                                 const int* __restrict__ cu, int B, int T, int n_types, const int* __restrict__ flags,
                                 const int* __restrict__ excl, anon_span* __restrict__ spans, int span_cap) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || !flags[t]) return;
  const int idx = excl[t];
  if (idx >= span_cap) return;
  const int b = find_record(cu, B, t);
  const int end_tok = min(cu[b + 1], T);
  const int lab = labels[t];
  const int typ = (lab + 1) >> 1;
  const int cont = 2 * typ;  // I-typ
  int e = t;
  while (e + 1 < end_tok && labels[e + 1] == cont) ++e;
  anon_span sp;
  sp.record = b;
  sp.type = typ;
  sp.begin = tok_off[2 * t];
  sp.end = tok_off[2 * e + 1];
  spans[idx] = sp;
}

__global__ void cu_spans_kernel(const int* __restrict__ cu, int B, int T, const int* __restrict__ excl,
                                int* __restrict__ cu_spans, int span_cap, uint32_t* err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > B) return;
  const int t = min(max(cu[b], 0), T);
  cu_spans[b] = excl[t];
  if (b == B && excl[T] > span_cap) raise_error(err, ANON_ERR_SPAN_CAP);
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t); }

void launch_exclusive_scan_i32(const int* in, int* out, int64_t n, void* temp, hipStream_t s) {
  exclusive_scan<int>(in, out, n, temp, s);
}
void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t s) {
  exclusive_scan<int64_t>(in, out, n, temp, s);
}

void launch_bio_flags(const uint8_t* labels, const int* cu_seqlens, int B, int T, int n_types, int* flags,
                      uint32_t* err, hipStream_t s) {
  if (T <= 0) return;
  hipLaunchKernelGGL(bio_flags_kernel, dim3(ceil_div(T, 256)), dim3(256), 0, s, labels, cu_seqlens, B, T, n_types,
                     flags, err);
}

void launch_bio_write(const uint8_t* labels, const int* tok_off, const int* cu_seqlens, int B, int T, int n_types,
                      const int* flags, const int* excl, anon_span* spans, int span_cap, int* cu_spans,
                      uint32_t* err, hipStream_t s) {
  if (T > 0)
    hipLaunchKernelGGL(bio_write_kernel, dim3(ceil_div(T, 256)), dim3(256), 0, s, labels, tok_off, cu_seqlens, B, T,
                       n_types, flags, excl, spans, span_cap);
  hipLaunchKernelGGL(cu_spans_kernel, dim3(ceil_div(B + 1, 256)), dim3(256), 0, s, cu_seqlens, B, T, excl, cu_spans,
                     span_cap, err);
}

}  // namespace anon
