// Pseudonym substitution on the GPU (the paper's Sec. II stage 3).
//
// Every entity span is replaced by "[" TYPE "_" slug "]", slug = the first n
// lowercase hex digits of HMAC-SHA256(key, entity bytes).  HMAC (RFC 2104)
// is computed with the SHA-256 states after the key^ipad and key^opad blocks
// precomputed once per key, so a message of up to 55 bytes costs two
// compressions.  A device hash table (open addressing, insert-only) caches
// entity bytes -> digest across calls; because the digest is a pure function
// of the bytes, a lost insert race or a full table only costs a recompute and
// never changes the output.
//
// Substitution is two-pass: a per-record pass validates the spans and lays
// out each pseudonym's output offset and the record's output length, a scan
// turns lengths into output offsets, and a per-record block writes every
// output byte (copied text or pseudonym character) at its final position.
#include "kernels.hpp"

namespace anon {

// FIPS 180-4 Sec. 4.2.2 round constants and Sec. 5.3.3 initial hash value.
#define ANON_SHA256_K                                                                                         \
  {0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u, \
   0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u, \
   0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau, \
   0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u, \
   0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, \
   0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u, \
   0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u, \
   0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u}

namespace {

constexpr uint32_t kH0[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                             0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

__host__ __device__ __forceinline__ uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

// One SHA-256 compression of the 16 big-endian words w into state st.
__host__ __device__ inline void sha256_compress(uint32_t st[8], const uint32_t win[16]) {
  constexpr uint32_t K[64] = ANON_SHA256_K;
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = win[i];
  uint32_t a = st[0], b = st[1], c = st[2], d = st[3], e = st[4], f = st[5], g = st[6], h = st[7];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    uint32_t wi;
    if (i < 16) {
      wi = w[i];
    } else {
      const uint32_t x15 = w[(i + 1) & 15], x2 = w[(i + 14) & 15];
      const uint32_t s0 = rotr(x15, 7) ^ rotr(x15, 18) ^ (x15 >> 3);
      const uint32_t s1 = rotr(x2, 17) ^ rotr(x2, 19) ^ (x2 >> 10);
      wi = w[i & 15] = w[i & 15] + s0 + w[(i + 9) & 15] + s1;
    }
    const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = h + S1 + ch + K[i] + wi;
    const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    const uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
    const uint32_t t2 = S0 + mj;
    h = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + t2;
  }
  st[0] += a;
  st[1] += b;
  st[2] += c;
  st[3] += d;
  st[4] += e;
  st[5] += f;
  st[6] += g;
  st[7] += h;
}

// SHA-256 continued from `st` (which has already absorbed `prefix` bytes)
// over msg[0..len); the final state is left in st.
__host__ __device__ inline void sha256_tail(uint32_t st[8], uint64_t prefix, const uint8_t* msg, int64_t len) {
  uint32_t w[16];
  int64_t pos = 0;
  while (len - pos >= 64) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      w[i] = ((uint32_t)msg[pos + 4 * i] << 24) | ((uint32_t)msg[pos + 4 * i + 1] << 16) |
             ((uint32_t)msg[pos + 4 * i + 2] << 8) | (uint32_t)msg[pos + 4 * i + 3];
    sha256_compress(st, w);
    pos += 64;
  }
  const int rem = (int)(len - pos);
  const uint64_t bits = (prefix + (uint64_t)len) * 8u;
  // final one or two blocks: remaining bytes, 0x80, zeros, 64-bit length
  const int nblk = rem < 56 ? 1 : 2;
  for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = blk * 64 + 4 * i + j;
        uint32_t byte = 0;
        if (k < rem) byte = msg[pos + k];
        else if (k == rem) byte = 0x80;
        v = (v << 8) | byte;
      }
      w[i] = v;
    }
    if (blk == nblk - 1) {
      w[14] = (uint32_t)(bits >> 32);
      w[15] = (uint32_t)bits;
    }
    sha256_compress(st, w);
  }
}

__device__ inline void hmac_sha256(const PcacheDev& pc, const uint8_t* msg, int64_t len, uint32_t out[8]) {
  uint32_t st[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) st[i] = pc.ipad[i];
  sha256_tail(st, 64, msg, len);
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = st[i];
  w[8] = 0x80000000u;
#pragma unroll
  for (int i = 9; i < 15; ++i) w[i] = 0;
  w[15] = (64 + 32) * 8;
#pragma unroll
  for (int i = 0; i < 8; ++i) out[i] = pc.opad[i];
  sha256_compress(out, w);
}

// Table entry: state, length, fingerprint, entity bytes, digest, and for the
// mapping export the smallest type the entity was pseudonymized under and the
// first and last call that met it.
constexpr int kMaxEntity = 96;
struct __align__(16) Entry {
  uint32_t state;  // 0 empty, 1 being written, 2 ready
  uint32_t len;
  uint64_t fp;
  uint8_t bytes[kMaxEntity];
  uint32_t digest[8];
  int32_t type;
  uint32_t first, last, pad;
};
static_assert(sizeof(Entry) == 160 && sizeof(Entry) == sizeof(PcacheEntryView), "entry layout");

__device__ __forceinline__ bool preserved(const PcacheDev& pc, int type) {
  return (pc.preserve[(type >> 5) & 3] >> (type & 31)) & 1u;
}

// A later meeting of a ready entry: keep the smallest type and the last call.
__device__ __forceinline__ void touch(Entry* e, int type, uint32_t call) {
  atomicMin(&e->type, type);
  atomicMax(&e->last, call);
}
constexpr int kMaxProbe = 32;

__device__ inline uint64_t fingerprint(const uint8_t* p, int len) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a 64
  for (int i = 0; i < len; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h ^ ((uint64_t)len << 56);
}

__device__ inline bool same_bytes(const uint8_t* a, const uint8_t* b, int len) {
  for (int i = 0; i < len; ++i)
    if (a[i] != b[i]) return false;
  return true;
}

__global__ void ps_layout_kernel(PcacheDev pc, const int64_t* __restrict__ cu_bytes, int B,
                                 const anon_span* __restrict__ spans, const int* __restrict__ cu_spans, int span_cap,
                                 int64_t* __restrict__ out_len, int64_t* __restrict__ sp_out,
                                 int* __restrict__ sp_plen, int64_t* __restrict__ sp_in_end, uint32_t* err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int64_t in_len = cu_bytes[b + 1] - cu_bytes[b];
  if (in_len < 0) {
    raise_error(err, ANON_ERR_SPAN);
    in_len = 0;
  }
  int s0 = cu_spans[b], s1 = cu_spans[b + 1];
  if (s1 > span_cap) raise_error(err, ANON_ERR_SPAN_CAP);
  s0 = min(max(s0, 0), span_cap);
  s1 = min(max(s1, s0), span_cap);
  int64_t acc = 0, prev_end = 0;
  const int tail = pc.slug > 0 ? pc.slug + 1 : 0;
  for (int s = s0; s < s1; ++s) {
    const anon_span sp = spans[s];
    const bool ok = sp.record == b && sp.type >= 1 && sp.type <= pc.n_types && sp.begin >= prev_end &&
                    sp.end >= sp.begin && sp.end <= in_len;
    if (ok && preserved(pc, sp.type)) {
      // a preserved type: the span's bytes are copied like the text around it
      sp_out[s] = prev_end + acc;
      sp_plen[s] = 0;
      sp_in_end[s] = prev_end;
    } else if (ok) {
      const int plen = 2 + (pc.name_off[sp.type] - pc.name_off[sp.type - 1]) + tail;
      sp_out[s] = sp.begin + acc;
      sp_plen[s] = plen;
      sp_in_end[s] = sp.end;
      acc += plen - (sp.end - sp.begin);
      prev_end = sp.end;
    } else {
      raise_error(err, ANON_ERR_SPAN);
      sp_out[s] = prev_end + acc;
      sp_plen[s] = 0;
      sp_in_end[s] = prev_end;
    }
  }
  out_len[b] = in_len + acc;
}

__global__ void ps_hash_kernel(PcacheDev pc, const uint8_t* __restrict__ text, const int64_t* __restrict__ cu_bytes,
                               int B, const anon_span* __restrict__ spans, const int* __restrict__ cu_spans,
                               int span_cap, const int* __restrict__ sp_plen, uint32_t* __restrict__ digests) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = min(cu_spans[B], span_cap);
  if (s >= n || sp_plen[s] <= 0 || pc.slug == 0) return;
  const anon_span sp = spans[s];
  const uint8_t* msg = text + cu_bytes[sp.record] + sp.begin;
  const int64_t len = sp.end - sp.begin;
  uint32_t dg[8];
  bool have = false;
  Entry* table = (Entry*)pc.table;
  uint64_t fp = 0;
  const bool use_table = pc.enabled && len <= kMaxEntity;
  if (use_table) {
    fp = fingerprint(msg, (int)len);
    atomicAdd(&pc.counters[0], 1ull);
    uint64_t slot = fp & pc.mask;
    for (int i = 0; i < kMaxProbe; ++i, slot = (slot + 1) & pc.mask) {
      Entry* e = table + slot;
      const uint32_t stt = __hip_atomic_load(&e->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (stt == 0) break;
      if (stt != 2) continue;
      // a ready entry: this fence pairs with its writer's release fence, so
      // the entry's fields read below are the ones written before "ready"
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (e->fp == fp && e->len == (uint32_t)len && same_bytes(e->bytes, msg, (int)len)) {
#pragma unroll
        for (int k = 0; k < 8; ++k) dg[k] = e->digest[k];
        have = true;
        atomicAdd(&pc.counters[1], 1ull);
        touch(e, sp.type, pc.call);
        break;
      }
    }
  }
  if (!have) {
    hmac_sha256(pc, msg, len, dg);
    if (use_table) {
      uint64_t slot = fp & pc.mask;
      for (int i = 0; i < kMaxProbe; ++i, slot = (slot + 1) & pc.mask) {
        Entry* e = table + slot;
        // claiming an empty slot reads nothing of another writer's, so the
        // claim needs no ordering; the fields are published by one release
        // fence ahead of the "ready" store (a fence is a cache write-back on
        // this part: one per wave instead of one per atomic)
        uint32_t expected = 0;
        if (__hip_atomic_compare_exchange_strong(&e->state, &expected, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          e->len = (uint32_t)len;
          e->fp = fp;
          for (int k = 0; k < len; ++k) e->bytes[k] = msg[k];
#pragma unroll
          for (int k = 0; k < 8; ++k) e->digest[k] = dg[k];
          e->type = sp.type;
          e->first = e->last = pc.call;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(&e->state, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicAdd(&pc.counters[2], 1ull);
          break;
        }
        if (expected == 2) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (e->fp == fp && e->len == (uint32_t)len && same_bytes(e->bytes, msg, (int)len)) {
            touch(e, sp.type, pc.call);
            break;
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) digests[(size_t)s * 8 + k] = dg[k];
}

__global__ __launch_bounds__(256) void ps_write_kernel(PcacheDev pc, const uint8_t* __restrict__ text,
                                                       const int64_t* __restrict__ cu_bytes,
                                                       const anon_span* __restrict__ spans,
                                                       const int* __restrict__ cu_spans, int span_cap,
                                                       const int64_t* __restrict__ sp_out,
                                                       const int* __restrict__ sp_plen,
                                                       const int64_t* __restrict__ sp_in_end,
                                                       const uint32_t* __restrict__ digests,
                                                       const int64_t* __restrict__ cu_out, uint8_t* __restrict__ out,
                                                       int64_t out_cap, uint32_t* err) {
  const int b = blockIdx.x;
  const int s0 = min(max(cu_spans[b], 0), span_cap);
  const int s1 = min(max(cu_spans[b + 1], s0), span_cap);
  const int64_t o0 = cu_out[b], n_out = cu_out[b + 1] - o0;
  const uint8_t* in = text + cu_bytes[b];
  const int64_t in_len = max(cu_bytes[b + 1] - cu_bytes[b], (int64_t)0);
  const char* hex = "0123456789abcdef";
  bool over = false;
  for (int64_t j = threadIdx.x; j < n_out; j += blockDim.x) {
    if (o0 + j >= out_cap) {
      over = true;
      break;
    }
    // last span whose pseudonym starts at or before output position j
    int lo = s0, hi = s1 - 1, sel = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      if (sp_out[mid] <= j) {
        sel = mid;
        lo = mid + 1;
      } else {
        hi = mid - 1;
      }
    }
    uint8_t c;
    if (sel < 0) {
      c = j < in_len ? in[j] : 0;
    } else {
      const int64_t k = j - sp_out[sel];
      const int plen = sp_plen[sel];
      if (k < plen) {
        const int typ = spans[sel].type;
        const int tl = pc.name_off[typ] - pc.name_off[typ - 1];
        if (k == 0) c = '[';
        else if (k == plen - 1) c = ']';
        else if (k <= tl) c = pc.names[pc.name_off[typ - 1] + k - 1];
        else if (k == tl + 1) c = '_';
        else {
          const int q = (int)(k - tl - 2);
          const uint32_t word = digests[(size_t)sel * 8 + (q >> 3)];
          c = hex[(word >> (28 - 4 * (q & 7))) & 15];
        }
      } else {
        const int64_t i = sp_in_end[sel] + (k - plen);
        c = i < in_len ? in[i] : 0;
      }
    }
    out[o0 + j] = c;
  }
  if (over) raise_error(err, ANON_ERR_OUT_CAP);
}

}  // namespace

size_t pcache_entry_bytes() { return sizeof(Entry); }

// Known-answer check of the host SHA-256/HMAC code (RFC 4231 Sec. 4.3).
bool hmac_selftest() {
  const char* key = "Jefe";
  const char* msg = "what do ya want for nothing?";
  const uint32_t want[8] = {0x5bdcc146u, 0xbf60754eu, 0x6a042426u, 0x089575c7u,
                            0x5a003f08u, 0x9d273983u, 0x9dec58b9u, 0x64ec3843u};
  uint32_t ip[8], op[8];
  sha256_hmac_midstates((const uint8_t*)key, 4, ip, op);
  sha256_tail(ip, 64, (const uint8_t*)msg, 28);
  uint32_t w[16] = {0};
  for (int i = 0; i < 8; ++i) w[i] = ip[i];
  w[8] = 0x80000000u;
  w[15] = (64 + 32) * 8;
  sha256_compress(op, w);
  for (int i = 0; i < 8; ++i)
    if (op[i] != want[i]) return false;
  return true;
}

void sha256_hmac_midstates(const uint8_t* key, size_t key_len, uint32_t ipad[8], uint32_t opad[8]) {
  uint8_t k0[64] = {0};
  if (key_len > 64) {
    uint32_t st[8];
    for (int i = 0; i < 8; ++i) st[i] = kH0[i];
    sha256_tail(st, 0, key, (int64_t)key_len);
    for (int i = 0; i < 8; ++i) {
      k0[4 * i] = (uint8_t)(st[i] >> 24);
      k0[4 * i + 1] = (uint8_t)(st[i] >> 16);
      k0[4 * i + 2] = (uint8_t)(st[i] >> 8);
      k0[4 * i + 3] = (uint8_t)st[i];
    }
  } else {
    for (size_t i = 0; i < key_len; ++i) k0[i] = key[i];
  }
  uint32_t wi[16], wo[16];
  for (int i = 0; i < 16; ++i) {
    uint32_t a = 0, b = 0;
    for (int j = 0; j < 4; ++j) {
      a = (a << 8) | (uint8_t)(k0[4 * i + j] ^ 0x36);
      b = (b << 8) | (uint8_t)(k0[4 * i + j] ^ 0x5c);
    }
    wi[i] = a;
    wo[i] = b;
  }
  for (int i = 0; i < 8; ++i) ipad[i] = opad[i] = kH0[i];
  sha256_compress(ipad, wi);
  sha256_compress(opad, wo);
}

void launch_ps_layout(const PcacheDev& pc, const int64_t* cu_bytes, int B, const anon_span* spans,
                      const int* cu_spans, int span_cap, int64_t* out_len, int64_t* sp_out, int* sp_plen,
                      int64_t* sp_in_end, uint32_t* err, hipStream_t s) {
  if (B <= 0) return;
  hipLaunchKernelGGL(ps_layout_kernel, dim3(ceil_div(B, 128)), dim3(128), 0, s, pc, cu_bytes, B, spans, cu_spans,
                     span_cap, out_len, sp_out, sp_plen, sp_in_end, err);
}

void launch_ps_hash(const PcacheDev& pc, const uint8_t* text, const int64_t* cu_bytes, int B, const anon_span* spans,
                    const int* cu_spans, int span_cap, const int* sp_plen, uint8_t* digests, hipStream_t s) {
  if (span_cap <= 0) return;
  hipLaunchKernelGGL(ps_hash_kernel, dim3(ceil_div(span_cap, 128)), dim3(128), 0, s, pc, text, cu_bytes, B, spans,
                     cu_spans, span_cap, sp_plen, (uint32_t*)digests);
}

void launch_ps_write(const PcacheDev& pc, const uint8_t* text, const int64_t* cu_bytes, int B,
                     const anon_span* spans, const int* cu_spans, int span_cap, const int64_t* sp_out,
                     const int* sp_plen, const int64_t* sp_in_end, const uint8_t* digests, const int64_t* cu_out,
                     uint8_t* out, int64_t out_cap, uint32_t* err, hipStream_t s) {
  if (B <= 0) return;
  hipLaunchKernelGGL(ps_write_kernel, dim3(B), dim3(256), 0, s, pc, text, cu_bytes, spans, cu_spans, span_cap,
                     sp_out, sp_plen, sp_in_end, (const uint32_t*)digests, cu_out, out, out_cap, err);
}

}  // namespace anon
