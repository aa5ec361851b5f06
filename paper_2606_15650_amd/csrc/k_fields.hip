// Schema-aware whole-field spans without NER: the paper's configuration that
// maps named fields straight to pseudonyms and bypasses inference (Sec. II;
// Sec. IV-A; App. C, Table VI with and without the configuration).
//
// Records are "Field: value" lines.  A line (a maximal run of bytes without
// '\n', never crossing a record boundary) holds a field if its first ':' is
// directly followed by ' '; the name is the bytes before the ':', the value
// the bytes after ": " up to the end of the line.  A configured name with a
// non-empty value gives one span of the configured type over the value.
//
// Byte-parallel: a thread per byte tests whether a line starts there and, if
// so, whether it is a configured field (names are at most 32 bytes, so the
// colon is looked for in the first 33 bytes); a scan of the per-byte flags
// numbers the spans in byte order, which is record-major, and the count
// before a record's first byte is its cu_spans entry.
#include "kernels.hpp"

namespace anon {
namespace {

// rs[p] = 1 where a record begins (cu_bytes[b] < n)
__global__ __launch_bounds__(256) void fd_mark_kernel(const int64_t* __restrict__ cu, int B, int64_t n,
                                                      uint8_t* rs, uint32_t* err) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > B) return;
  const int64_t x = cu[b];
  if ((b == 0 && x != 0) || (b == B && x != n) || (b < B && cu[b + 1] < x)) raise_error(err, ANON_ERR_TEXT);
  if (b < B && x >= 0 && x < n) rs[x] = 1;
}

// The configured field whose line starts at p, if any: its type and value
// [vb, ve).  A line ends at '\n', at the next record's first byte or at n.
__device__ int field_at(const uint8_t* __restrict__ t, const uint8_t* __restrict__ rs, int64_t n, int64_t p,
                        const FieldTable& ft, int64_t& vb, int64_t& ve) {
  if (p > 0 && t[p - 1] != '\n' && !rs[p]) return 0;
  int64_t c = p;
  const int64_t lim = min(n, p + kFieldNameMax + 1);
  while (c < lim && t[c] != ':' && t[c] != '\n' && (c == p || !rs[c])) ++c;
  if (c >= lim || t[c] != ':' || (c > p && rs[c])) return 0;
  if (c + 1 >= n || t[c + 1] != ' ' || rs[c + 1]) return 0;
  const int len = (int)(c - p);
  int type = 0;
  for (int k = 0; k < ft.n && !type; ++k) {
    if (ft.len[k] != len) continue;
    bool eq = true;
    for (int i = 0; i < len && eq; ++i) eq = t[p + i] == ft.name[k][i];
    if (eq) type = ft.type[k];
  }
  if (!type) return 0;
  vb = c + 2;
  ve = vb;
  while (ve < n && t[ve] != '\n' && !rs[ve]) ++ve;
  return ve > vb ? type : 0;
}

__global__ __launch_bounds__(256) void fd_flags_kernel(const uint8_t* __restrict__ text,
                                                       const uint8_t* __restrict__ rs, int64_t n, FieldTable ft,
                                                       int* flags) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n; p += (int64_t)gridDim.x * 256) {
    int64_t vb, ve;
    flags[p] = (p < n && field_at(text, rs, n, p, ft, vb, ve)) ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void fd_emit_kernel(const uint8_t* __restrict__ text,
                                                      const uint8_t* __restrict__ rs, int64_t n, FieldTable ft,
                                                      const int* __restrict__ flags, const int* __restrict__ excl,
                                                      const int64_t* __restrict__ cu, int B, anon_span* out,
                                                      int cap) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
    if (!flags[p] || excl[p] >= cap) continue;
    int64_t vb, ve;
    const int type = field_at(text, rs, n, p, ft, vb, ve);
    int a = 0, c = B;  // cu[a] <= p < cu[c]
    while (c - a > 1) {
      const int m = (a + c) >> 1;
      if (cu[m] <= p) a = m;
      else c = m;
    }
    out[excl[p]] = anon_span{a, type, vb - cu[a], ve - cu[a]};
  }
}

__global__ __launch_bounds__(256) void fd_cu_kernel(const int* __restrict__ excl, const int64_t* __restrict__ cu,
                                                    int B, int64_t n, int cap, int* cu_spans, uint32_t* err) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > B) return;
  const int64_t x = min(max(cu[b], (int64_t)0), n);
  cu_spans[b] = excl[x];
  if (b == B && excl[n] > cap) raise_error(err, ANON_ERR_SPAN_CAP);
}

}  // namespace

FieldBuffers field_layout(int64_t n, Carver& k) {
  FieldBuffers w;
  w.rs = k.take<uint8_t>(n + 1);
  w.flags = k.take<int>(n + 1);
  w.excl = k.take<int>(n + 2);
  w.temp = k.take<uint8_t>(scan_temp_bytes(n + 1));
  return w;
}

size_t field_workspace_bytes(int64_t n) {
  Carver k(nullptr, SIZE_MAX);
  field_layout(n, k);
  return k.used + 256;
}

void launch_field_spans(const uint8_t* text, const int64_t* cu_bytes, int B, int64_t n, const FieldTable& ft,
                        const FieldBuffers& w, anon_span* out, int cap, int* cu_spans, uint32_t* err,
                        hipStream_t s) {
  const int g = std::max(1, std::min(ceil_div(n + 1, 256), 8192));
  launch_fill_u8(w.rs, 0, n + 1, s);
  hipLaunchKernelGGL(fd_mark_kernel, dim3(ceil_div(B + 1, 256)), dim3(256), 0, s, cu_bytes, B, n, w.rs, err);
  hipLaunchKernelGGL(fd_flags_kernel, dim3(g), dim3(256), 0, s, text, w.rs, n, ft, w.flags);
  launch_exclusive_scan_i32(w.flags, w.excl, n + 1, w.temp, s);
  if (n > 0 && cap > 0)
    hipLaunchKernelGGL(fd_emit_kernel, dim3(g), dim3(256), 0, s, text, w.rs, n, ft, w.flags, w.excl, cu_bytes, B,
                       out, cap);
  hipLaunchKernelGGL(fd_cu_kernel, dim3(ceil_div(B + 1, 256)), dim3(256), 0, s, w.excl, cu_bytes, B, n, cap,
                     cu_spans, err);
}

}  // namespace anon
