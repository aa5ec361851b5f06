// Pattern recognizers beside the NER model (the paper's detector pairs the
// transformer with regular-expression recognizers, Sec. II stage 2) and the
// merge of overlapping detections into whole-entity spans.
//
// Nine recognizers, each a rule at one start byte of a record (W = word bytes
// [A-Za-z0-9_], LABEL = [A-Za-z0-9-], LOCAL = [A-Za-z0-9._%+-]):
//   0 URL       "http://" or "https://" at a word start, then >= 1 non-space bytes
//   1 EMAIL     maximal LOCAL run, '@', >= 1 "label." groups, then an all-letter
//               top label of >= 2 bytes not followed by a LABEL byte (longest)
//   2 IPV4      four dot-separated octets 0..255 without leading zeros, at word
//               boundaries
//   3 MAC       six hex pairs separated by ':', at word boundaries
//   4 HASH      a hex run of exactly 32, 40 or 64 bytes at word boundaries
//   5 CVE       "CVE-" + 4 digits + '-' + 4..7 digits at word boundaries
//   6 HOSTNAME  dotted LABEL run not preceded by LABEL or '.', ending at a label
//               equal to one of eight top labels, not followed by LABEL (longest)
//   7 IPV6      an address in an RFC 4291 (section 2.2) text form: the maximal
//               run of hex digits, ':' and '.' from a hex digit or ':' not
//               preceded by W, ':' or '.', without its trailing dots, not
//               followed by W
//   8 CPE       "cpe:/" + part [aho] or "cpe:2.3:" + part [aho*-] at a word
//               start, the part not followed by a component byte C =
//               [A-Za-z0-9._~%*?!\-], then the maximal run of C and ':'
// Every start byte where a rule matches gives one candidate span.
//
// Merge: NER spans and candidates sharing a byte form one span, their union
// (transitively; spans that only touch stay apart), typed by its longest
// member, then NER before recognizers (in the order above), then the leftmost.
//
// Byte-parallel throughout: one thread per text byte tries the rules; every
// span adds +1 at its begin and -1 at its end of a delta array and a 64-bit
// key (length, priority, begin) at its begin.  A scan of the deltas gives, per
// byte, how many spans cover it; a union starts at a byte where a span begins
// and no earlier-begun span still covers it, and ends at the first byte after
// it where again no earlier-begun span covers.  Scans of the start and end
// flags number the unions; the largest key among a union's begin bytes gives
// its type.
#include "kernels.hpp"

namespace anon {
namespace {

__device__ __forceinline__ bool is_digit(uint8_t c) { return c >= '0' && c <= '9'; }
__device__ __forceinline__ bool is_letter(uint8_t c) { return (c | 0x20) >= 'a' && (c | 0x20) <= 'z'; }
__device__ __forceinline__ bool is_word(uint8_t c) { return is_digit(c) || is_letter(c) || c == '_'; }
__device__ __forceinline__ bool is_label(uint8_t c) { return is_digit(c) || is_letter(c) || c == '-'; }
__device__ __forceinline__ bool is_local(uint8_t c) {
  return is_digit(c) || is_letter(c) || c == '.' || c == '_' || c == '%' || c == '+' || c == '-';
}
__device__ __forceinline__ bool is_hex(uint8_t c) {
  return is_digit(c) || ((c | 0x20) >= 'a' && (c | 0x20) <= 'f');
}
__device__ __forceinline__ bool is_space(uint8_t c) { return c == ' ' || (c >= '\t' && c <= '\r'); }

// One record's bytes [lo, hi) of the text; positions are absolute.  Bytes
// inside the workgroup's staged window [wlo, whi) are read from LDS, the rest
// (long runs past the window) from global memory.
struct Rec {
  const uint8_t* t;
  int64_t lo, hi;
  const uint8_t* win;
  int64_t wlo, whi;
  __device__ uint8_t at(int64_t i) const { return (i >= wlo && i < whi) ? win[i - wlo] : t[i]; }
  __device__ bool word_start(int64_t p) const { return is_word(at(p)) && (p == lo || !is_word(at(p - 1))); }
  __device__ bool word_end(int64_t q) const { return q == hi || !is_word(at(q)); }
  __device__ bool has(int64_t p, const char* s, int n) const {
    if (p + n > hi) return false;
    for (int i = 0; i < n; ++i)
      if (at(p + i) != (uint8_t)s[i]) return false;
    return true;
  }
};

__device__ int64_t match_url(const Rec& r, int64_t p) {
  if (!r.word_start(p)) return -1;
  int64_t q;
  if (r.has(p, "https://", 8)) q = p + 8;
  else if (r.has(p, "http://", 7)) q = p + 7;
  else return -1;
  int64_t e = q;
  while (e < r.hi && !is_space(r.at(e))) ++e;
  return e > q ? e : -1;
}

// An all-letter label of >= 2 bytes at s, not followed by a LABEL byte.
__device__ int64_t top_letters(const Rec& r, int64_t s) {
  int64_t e = s;
  while (e < r.hi && is_letter(r.at(e))) ++e;
  return (e - s >= 2 && (e == r.hi || !is_label(r.at(e)))) ? e : -1;
}

// One of the eight top labels at s, not followed by a LABEL byte.
__device__ int64_t top_listed(const Rec& r, int64_t s) {
  const char* const tops[8] = {"corp", "lan", "intra", "net", "org", "local", "example", "internal"};
  const int lens[8] = {4, 3, 5, 3, 3, 5, 7, 8};
  for (int k = 0; k < 8; ++k)
    if (r.has(s, tops[k], lens[k]) && (s + lens[k] == r.hi || !is_label(r.at(s + lens[k])))) return s + lens[k];
  return -1;
}

// Dotted LABEL groups from i on: the top label may start after any group but
// the first; the longest successful domain is the last success in order.
template <bool LISTED>
__device__ int64_t dotted_domain(const Rec& r, int64_t i) {
  int64_t best = -1;
  int groups = 0;
  while (true) {
    int64_t j = i;
    while (j < r.hi && is_label(r.at(j))) ++j;
    const bool group = j > i && j < r.hi && r.at(j) == '.';
    if (groups >= 1) {
      const int64_t e = LISTED ? top_listed(r, i) : top_letters(r, i);
      if (e >= 0) best = e;
    }
    if (!group) return best;
    ++groups;
    i = j + 1;
  }
}

__device__ int64_t match_email(const Rec& r, int64_t p) {
  if (!is_local(r.at(p)) || (p > r.lo && is_local(r.at(p - 1)))) return -1;
  int64_t q = p;
  while (q < r.hi && is_local(r.at(q))) ++q;
  if (q == r.hi || r.at(q) != '@') return -1;
  return dotted_domain<false>(r, q + 1);
}

__device__ int64_t match_hostname(const Rec& r, int64_t p) {
  if (!is_label(r.at(p)) || (p > r.lo && (is_label(r.at(p - 1)) || r.at(p - 1) == '.'))) return -1;
  return dotted_domain<true>(r, p);
}

// End of a valid octet spanning the whole digit run at i, else -1.
__device__ int64_t octet(const Rec& r, int64_t i) {
  int64_t e = i;
  int v = 0;
  while (e < r.hi && is_digit(r.at(e)) && e - i < 4) v = v * 10 + (r.at(e++) - '0');
  const int64_t c = e - i;
  if (c < 1 || c > 3 || (c > 1 && r.at(i) == '0') || v > 255) return -1;
  return e;
}

__device__ int64_t match_ipv4(const Rec& r, int64_t p) {
  if (!is_digit(r.at(p)) || !r.word_start(p)) return -1;
  int64_t i = p;
  for (int k = 0; k < 4; ++k) {
    const int64_t e = octet(r, i);
    if (e < 0) return -1;
    if (k == 3) return r.word_end(e) ? e : -1;
    if (e == r.hi || r.at(e) != '.') return -1;
    i = e + 1;
  }
  return -1;
}

__device__ int64_t match_mac(const Rec& r, int64_t p) {
  if (!r.word_start(p) || p + 17 > r.hi) return -1;
  for (int k = 0; k < 17; ++k) {
    const uint8_t c = r.at(p + k);
    if (k % 3 == 2 ? c != ':' : !is_hex(c)) return -1;
  }
  return r.word_end(p + 17) ? p + 17 : -1;
}

__device__ int64_t match_hash(const Rec& r, int64_t p) {
  if (!is_hex(r.at(p)) || !r.word_start(p)) return -1;
  int64_t e = p;
  while (e < r.hi && is_hex(r.at(e)) && e - p < 65) ++e;
  const int64_t c = e - p;
  return ((c == 32 || c == 40 || c == 64) && r.word_end(e)) ? e : -1;
}

__device__ int64_t match_cve(const Rec& r, int64_t p) {
  if (!r.word_start(p) || p + 9 > r.hi || !r.has(p, "CVE-", 4)) return -1;
  for (int k = 0; k < 4; ++k)
    if (!is_digit(r.at(p + 4 + k))) return -1;
  if (r.at(p + 8) != '-') return -1;
  int64_t e = p + 9;
  while (e < r.hi && is_digit(r.at(e)) && e - (p + 9) < 8) ++e;
  const int64_t c = e - (p + 9);
  return (c >= 4 && c <= 7 && r.word_end(e)) ? e : -1;
}

__device__ __forceinline__ bool is_cpe(uint8_t c) {
  return is_digit(c) || is_letter(c) || c == '.' || c == '_' || c == '~' || c == '%' || c == '*' || c == '?' ||
         c == '!' || c == '\\' || c == '-';
}

__device__ int64_t match_cpe(const Rec& r, int64_t p) {
  if (!r.word_start(p)) return -1;
  int64_t q;
  bool v23;
  if (r.has(p, "cpe:/", 5)) q = p + 5, v23 = false;
  else if (r.has(p, "cpe:2.3:", 8)) q = p + 8, v23 = true;
  else return -1;
  if (q == r.hi) return -1;
  const uint8_t part = r.at(q);
  if (!(part == 'a' || part == 'h' || part == 'o' || (v23 && (part == '*' || part == '-')))) return -1;
  ++q;
  if (q < r.hi && is_cpe(r.at(q))) return -1;
  while (q < r.hi && (is_cpe(r.at(q)) || r.at(q) == ':')) ++q;
  return q;
}

// Four octets separated by '.', exactly covering [i, end).
__device__ bool dotted_quad(const Rec& r, int64_t i, int64_t end) {
  for (int k = 0; k < 4; ++k) {
    const int64_t e = octet(r, i);
    if (e < 0) return false;
    if (k == 3) return e == end;
    if (e >= end || r.at(e) != '.') return false;
    i = e + 1;
  }
  return false;
}

// The address text S = [p, s) is read group by group: 1-4 hex digits, a ':'
// after every group but the last, one "::" at most (standing for at least
// one zero group, so at most seven written groups), and a dotted quad, worth
// two groups, only as the text's last group.  An address text is at most 45
// bytes long, so a longer S is rejected while it is scanned.
__device__ int64_t match_ipv6(const Rec& r, int64_t p) {
  const uint8_t c0 = r.at(p);
  if (!is_hex(c0) && c0 != ':') return -1;
  if (p > r.lo) {
    const uint8_t c = r.at(p - 1);
    if (is_word(c) || c == ':' || c == '.') return -1;
  }
  // The first group has at most 4 hex digits and a ':' follows it (a lone
  // group or a dotted quad alone is no address), so hashes, IPv4 addresses
  // and words are rejected after at most 5 bytes.
  int64_t e = p, s = p;
  bool colon = false;
  while (e < r.hi) {
    const uint8_t c = r.at(e);
    if (c == '.') {
      if (!colon) return -1;
      ++e;
      continue;
    }
    if (c == ':') colon = true;
    else if (!is_hex(c)) break;
    else if (!colon && e - p >= 4) return -1;
    s = ++e;
    if (s - p > 45) return -1;
  }
  if (!colon || !r.word_end(s)) return -1;
  int groups = 0;
  bool dbl = false;
  int64_t i = p;
  if (c0 == ':') {
    if (s - p < 2 || r.at(p + 1) != ':') return -1;
    dbl = true;
    i = p + 2;
  }
  while (i < s) {
    int64_t j = i;
    while (j < s && is_hex(r.at(j))) ++j;
    if (j < s && r.at(j) == '.') {
      if (!dotted_quad(r, i, s)) return -1;
      groups += 2;
      break;
    }
    if (j == i || j - i > 4) return -1;
    ++groups;
    i = j;
    if (i == s) break;
    ++i;  // the ':' after the group
    if (i == s) return -1;
    if (r.at(i) == ':') {
      if (dbl) return -1;
      dbl = true;
      if (++i == s) break;
    }
  }
  return (dbl ? groups <= 7 : groups == 8) ? s : -1;
}

constexpr int kRecognizers = kNumRecognizers;
// the IPv6 and CPE rules run in a kernel of their own (rx_extra_kernel)
constexpr int kIpv6 = 7;
constexpr int kCpe = 8;
constexpr int kWin = 1 + 256 + 1024;  // staged bytes per match workgroup (1 before, 1024 ahead)
struct RecTypes {
  int t[kRecognizers];  // type index per recognizer, 0 = off
};

// 64-bit union key of a span: longest first, then lowest priority (NER 0,
// recognizer k -> k+1), then leftmost begin (offset inside the record).
__device__ __forceinline__ unsigned long long span_key(int64_t len, int prio, int64_t local_begin) {
  const unsigned long long L = (unsigned long long)min(len, (int64_t)0xFFFFFF);
  return (L << 40) | ((unsigned long long)(255 - prio) << 32) | (0xFFFFFFFFull - (unsigned long long)local_begin);
}

// Record b's bytes, clamped to the text [0, n) (a malformed cu_bytes is
// flagged by rx_check_kernel and cannot send a read outside the text).
__device__ __forceinline__ void record_bounds(const int64_t* cu, int b, int64_t n, int64_t& lo, int64_t& hi) {
  lo = min(max(cu[b], (int64_t)0), n);
  hi = min(max(cu[b + 1], lo), n);
}

__device__ __forceinline__ int find_record(const int64_t* cu, int B, int64_t p) {
  int a = 0, b = B;  // cu[a] <= p < cu[b]
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (cu[m] <= p) a = m;
    else b = m;
  }
  return a;
}

// cu_bytes must rise from 0 to n, and records must be shorter than 16 MiB
// (the union key holds lengths in 24 bits).
__global__ __launch_bounds__(256) void rx_check_kernel(const int64_t* __restrict__ cu, int B, int64_t n,
                                                       uint32_t* err) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > B) return;
  if ((b == 0 && cu[0] != 0) || (b == B && cu[B] != n)) raise_error(err, ANON_ERR_TEXT);
  if (b < B && (cu[b + 1] < cu[b] || cu[b + 1] - cu[b] >= (int64_t(1) << 24))) raise_error(err, ANON_ERR_TEXT);
}

__global__ __launch_bounds__(256) void rx_clear_kernel(int* delta, int* starts, unsigned long long* key,
                                                       uint8_t* ner_type, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += (int64_t)gridDim.x * 256) {
    delta[i] = 0;
    starts[i] = 0;
    key[i] = 0;
    ner_type[i] = 0;
  }
}

// Every enabled rule at p; candidates go into the delta/start/key arrays.
__device__ void match_all(const Rec& r, int64_t p, const RecTypes& rt, int* delta, int* starts,
                          unsigned long long* key) {
  int count = 0;
  unsigned long long best = 0;
#pragma unroll
  for (int k = 0; k < kIpv6; ++k) {
    if (rt.t[k] == 0) continue;
    int64_t e;
    switch (k) {
      case 0: e = match_url(r, p); break;
      case 1: e = match_email(r, p); break;
      case 2: e = match_ipv4(r, p); break;
      case 3: e = match_mac(r, p); break;
      case 4: e = match_hash(r, p); break;
      case 5: e = match_cve(r, p); break;
      default: e = match_hostname(r, p); break;
    }
    if (e < 0) continue;
    ++count;
    atomicAdd(&delta[e], -1);
    const unsigned long long kk = span_key(e - p, 1 + k, p - r.lo);
    best = kk > best ? kk : best;
  }
  if (count) {
    atomicAdd(&delta[p], count);
    atomicAdd(&starts[p], count);
    atomicMax(&key[p], best);
  }
}

__device__ __forceinline__ bool is_alnum(uint8_t c) { return is_digit(c) || is_letter(c); }


// A rule can start at p only on a LOCAL byte (URL 'h', IPv4/MAC/hash/CVE
// word bytes, e-mail LOCAL, hostname LABEL) whose predecessor in the record
// is not alphanumeric (the word-boundary rules exclude a word byte before
// it, the e-mail rule a LOCAL byte, the hostname rule a LABEL byte or dot).
// Each workgroup first collects its 256 bytes that pass this test, then runs
// the rules on them with the lanes packed: most bytes sit inside words, and
// trying them all left most lanes of a wave idle behind a few long scans.
// A record's first byte whose predecessor (the previous record's last byte)
// is alphanumeric fails the test here and is tried by rx_recstart_kernel.
__global__ __launch_bounds__(256) void rx_match_kernel(const uint8_t* __restrict__ text,
                                                       const int64_t* __restrict__ cu, int B, int64_t n,
                                                       RecTypes rt, int* delta, int* starts,
                                                       unsigned long long* key) {
  // the workgroup's 256 start bytes, the byte before them and 1024 bytes of
  // lookahead, staged in LDS (coalesced loads)
  __shared__ uint8_t win[kWin];
  __shared__ int cand[256];
  __shared__ int ncand;
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  const int64_t wlo = p0 > 0 ? p0 - 1 : 0;
  const int64_t whi = min(wlo + kWin, n);
  for (int64_t i = wlo + threadIdx.x; i < whi; i += 256) win[i - wlo] = text[i];
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  const int64_t p = p0 + threadIdx.x;
  if (p < n && is_local(win[p - wlo]) && !(p > 0 && is_alnum(win[p - 1 - wlo])))
    cand[atomicAdd(&ncand, 1)] = threadIdx.x;
  __syncthreads();
  const int nc = ncand;
  for (int i = threadIdx.x; i < nc; i += 256) {
    const int64_t q = p0 + cand[i];
    const int b = find_record(cu, B, q);
    int64_t lo, hi;
    record_bounds(cu, b, n, lo, hi);
    if (q < lo || q >= hi) continue;  // only with a malformed cu_bytes
    match_all(Rec{text, lo, hi, win, wlo, whi}, q, rt, delta, starts, key);
  }
}

// Record starts whose previous byte is alphanumeric (see rx_match_kernel).
__global__ __launch_bounds__(256) void rx_recstart_kernel(const uint8_t* __restrict__ text,
                                                          const int64_t* __restrict__ cu, int B, int64_t n,
                                                          RecTypes rt, int* delta, int* starts,
                                                          unsigned long long* key) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  int64_t lo, hi;
  record_bounds(cu, b, n, lo, hi);
  if (hi <= lo || lo == 0 || !is_alnum(text[lo - 1]) || !is_local(text[lo])) return;
  match_all(Rec{text, lo, hi, nullptr, 0, 0}, lo, rt, delta, starts, key);
}

// The IPv6 and CPE rules over every byte, in a kernel of their own: inlined
// beside the other rules, either raises that kernel's register count from
// 66 to over 110 VGPRs and nearly halves its occupancy.  Each has an exact
// pre-filter on the staged window, which holds the 7 bytes after every start
// byte unless the text ends first: an IPv6 address starts with 1-4 hex
// digits or ':' and has a ':' within its first 5 bytes; a CPE name starts
// with "cpe:".  The rules then check the record bounds and boundaries.
// Contributions add to the same delta/start/key arrays with atomics, in any
// order.
__global__ __launch_bounds__(256) void rx_extra_kernel(const uint8_t* __restrict__ text,
                                                       const int64_t* __restrict__ cu, int B, int64_t n, int use_ipv6,
                                                       int use_cpe, int* delta, int* starts,
                                                       unsigned long long* key) {
  // an address is at most 45 bytes: 64 bytes of lookahead hold almost every
  // candidate's run (reads past the window go to global memory)
  constexpr int kWin6 = 1 + 256 + 64;
  __shared__ uint8_t win[kWin6];
  __shared__ int cand[256];
  __shared__ int ncand;
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  const int64_t wlo = p0 > 0 ? p0 - 1 : 0;
  const int64_t whi = min(wlo + kWin6, n);
  for (int64_t i = wlo + threadIdx.x; i < whi; i += 256) win[i - wlo] = text[i];
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  const int64_t p = p0 + threadIdx.x;
  if (p < n) {
    bool pass = false;
    if (use_ipv6) {
      for (int k = 0; k < 5 && p + k < whi; ++k) {
        const uint8_t c = win[p + k - wlo];
        if (c == ':') {
          pass = true;
          break;
        }
        if (!is_hex(c)) break;
      }
    }
    if (use_cpe && p + 3 < whi)
      pass = pass || (win[p - wlo] == 'c' && win[p + 1 - wlo] == 'p' && win[p + 2 - wlo] == 'e' &&
                      win[p + 3 - wlo] == ':');
    if (pass) cand[atomicAdd(&ncand, 1)] = threadIdx.x;
  }
  __syncthreads();
  const int nc = ncand;
  for (int i = threadIdx.x; i < nc; i += 256) {
    const int64_t q = p0 + cand[i];
    const int b = find_record(cu, B, q);
    int64_t lo, hi;
    record_bounds(cu, b, n, lo, hi);
    if (q < lo || q >= hi) continue;  // only with a malformed cu_bytes
    const Rec r{text, lo, hi, win, wlo, whi};
    int count = 0;
    unsigned long long best = 0;
    const int64_t e6 = use_ipv6 ? match_ipv6(r, q) : -1;
    if (e6 >= 0) {
      ++count;
      atomicAdd(&delta[e6], -1);
      best = span_key(e6 - q, 1 + kIpv6, q - lo);
    }
    const int64_t ec = use_cpe ? match_cpe(r, q) : -1;
    if (ec >= 0) {
      ++count;
      atomicAdd(&delta[ec], -1);
      const unsigned long long kk = span_key(ec - q, 1 + kCpe, q - lo);
      best = kk > best ? kk : best;
    }
    if (count) {
      atomicAdd(&delta[q], count);
      atomicAdd(&starts[q], count);
      atomicMax(&key[q], best);
    }
  }
}

// NER spans (record-relative [begin, end)) join the candidates.
__global__ __launch_bounds__(256) void rx_ner_kernel(const anon_span* __restrict__ spans,
                                                     const int* __restrict__ ner_cu, int B, int ner_cap,
                                                     const int64_t* __restrict__ cu, int64_t n, int n_types, int* delta,
                                                     int* starts, unsigned long long* key, uint8_t* ner_type,
                                                     uint32_t* err) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= min(ner_cu[B], ner_cap)) return;
  const anon_span s = spans[i];
  if (s.record < 0 || s.record >= B || s.type < 1 || s.type > n_types) {
    raise_error(err, ANON_ERR_SPAN);
    return;
  }
  int64_t lo, hi;
  record_bounds(cu, s.record, n, lo, hi);
  if (s.begin < 0 || s.end <= s.begin || s.end > hi - lo) {
    raise_error(err, ANON_ERR_SPAN);
    return;
  }
  const int64_t gb = lo + s.begin, ge = lo + s.end;
  atomicAdd(&delta[gb], 1);
  atomicAdd(&delta[ge], -1);
  atomicAdd(&starts[gb], 1);
  atomicMax(&key[gb], span_key(ge - gb, 0, s.begin));
  ner_type[gb] = (uint8_t)s.type;  // decoded NER spans of a record never share a begin
}

// cover[p] = exclusive scan of delta: spans covering byte p-1 (cover[p+1]
// covers p).  A union starts at p if a span begins there and no span begun
// earlier covers p; one ends at q if byte q-1 is covered and no span begun
// before q covers q.
__global__ __launch_bounds__(256) void rx_flags_kernel(const int* __restrict__ cover, const int* __restrict__ starts,
                                                       int64_t n, int* fstart, int* fend) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n; p += (int64_t)gridDim.x * 256) {
    const int cov_p = p < n ? cover[p + 1] : 0;
    const int carry = cov_p - (p < n ? starts[p] : 0);
    fstart[p] = (p < n && starts[p] > 0 && carry == 0) ? 1 : 0;
    fend[p] = (p >= 1 && cover[p] > 0 && carry == 0) ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void rx_runs_kernel(const int* __restrict__ fstart, const int* __restrict__ sstart,
                                                      const int* __restrict__ fend, const int* __restrict__ send,
                                                      const unsigned long long* __restrict__ key, int64_t n,
                                                      int64_t* run_begin, int64_t* run_end,
                                                      unsigned long long* run_key) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n; p += (int64_t)gridDim.x * 256) {
    if (fstart[p]) run_begin[sstart[p]] = p;
    if (fend[p]) run_end[send[p]] = p;
    if (p < n && key[p]) atomicMax(&run_key[sstart[p + 1] - 1], key[p]);
  }
}

__global__ __launch_bounds__(256) void rx_emit_kernel(const int* __restrict__ n_runs_p, const int64_t* __restrict__ run_begin,
                                                      const int64_t* __restrict__ run_end,
                                                      const unsigned long long* __restrict__ run_key,
                                                      const uint8_t* __restrict__ ner_type, const int64_t* __restrict__ cu,
                                                      int B, RecTypes rt, anon_span* out, int cap) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= min(*n_runs_p, cap)) return;
  const int64_t gb = run_begin[i], ge = run_end[i];
  const int b = find_record(cu, B, gb);
  const unsigned long long k = run_key[i];
  const int prio = 255 - (int)((k >> 32) & 0xFF);
  const int64_t wb = cu[b] + (int64_t)(0xFFFFFFFFull - (k & 0xFFFFFFFFull));
  const int type = prio == 0 ? (int)ner_type[wb] : rt.t[min(prio, kRecognizers) - 1];
  out[i] = anon_span{b, type, gb - cu[b], ge - cu[b]};
}

// cu_spans[b] = unions beginning before record b's first byte.
__global__ __launch_bounds__(256) void rx_cu_kernel(const int* __restrict__ n_runs_p, const int64_t* __restrict__ run_begin,
                                                    const int64_t* __restrict__ cu, int B, int cap, int* cu_spans,
                                                    uint32_t* err) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > B) return;
  const int total = *n_runs_p;
  if (b == B) {
    cu_spans[B] = total;
    if (total > cap) raise_error(err, ANON_ERR_SPAN_CAP);
    return;
  }
  const int64_t x = cu[b];
  int a = 0, c = total;  // first run with begin >= x
  while (a < c) {
    const int m = (a + c) >> 1;
    if (run_begin[m] < x) a = m + 1;
    else c = m;
  }
  cu_spans[b] = a;
}

}  // namespace

size_t recog_workspace_bytes(int64_t n) {
  Carver k(nullptr, SIZE_MAX);
  recog_layout(n, k);
  return k.used + 256;
}

RecogBuffers recog_layout(int64_t n, Carver& k) {
  RecogBuffers w;
  w.delta = k.take<int>(n + 1);
  w.starts = k.take<int>(n + 1);
  w.key = k.take<unsigned long long>(n + 1);
  w.ner_type = k.take<uint8_t>(n + 1);
  w.cover = k.take<int>(n + 2);
  w.fstart = k.take<int>(n + 1);
  w.fend = k.take<int>(n + 1);
  w.sstart = k.take<int>(n + 2);
  w.send = k.take<int>(n + 2);
  w.run_begin = k.take<int64_t>(n + 1);
  w.run_end = k.take<int64_t>(n + 1);
  w.run_key = k.take<unsigned long long>(n + 1);
  w.temp = k.take<uint8_t>(scan_temp_bytes(n + 1));
  return w;
}

void launch_recognize(const uint8_t* text, const int64_t* cu_bytes, int B, int64_t n,
                      const int rec_types[kNumRecognizers],
                      const anon_span* ner, const int* ner_cu, int ner_cap, int n_types, const RecogBuffers& w,
                      anon_span* out, int cap, int* cu_spans, uint32_t* err, hipStream_t s) {
  RecTypes rt;
  for (int k = 0; k < kRecognizers; ++k) rt.t[k] = rec_types[k];
  const int g = std::max(1, std::min(ceil_div(n + 2, 256), 8192));
  hipLaunchKernelGGL(rx_clear_kernel, dim3(g), dim3(256), 0, s, w.delta, w.starts, w.key, w.ner_type, n);
  // run_key is indexed by union number (at most n); the flag arrays are
  // written in full by rx_flags_kernel
  launch_fill_u8((uint8_t*)w.run_key, 0, (n + 1) * (int64_t)sizeof(unsigned long long), s);
  hipLaunchKernelGGL(rx_check_kernel, dim3(ceil_div(B + 1, 256)), dim3(256), 0, s, cu_bytes, B, n, err);
  if (n > 0) {
    hipLaunchKernelGGL(rx_match_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, text, cu_bytes, B, n, rt, w.delta,
                       w.starts, w.key);
    hipLaunchKernelGGL(rx_recstart_kernel, dim3(ceil_div(B, 256)), dim3(256), 0, s, text, cu_bytes, B, n, rt,
                       w.delta, w.starts, w.key);
    if (rt.t[kIpv6] != 0 || rt.t[kCpe] != 0)
      hipLaunchKernelGGL(rx_extra_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, text, cu_bytes, B, n,
                         rt.t[kIpv6] != 0 ? 1 : 0, rt.t[kCpe] != 0 ? 1 : 0, w.delta, w.starts, w.key);
  }
  if (ner && ner_cu && ner_cap > 0)
    hipLaunchKernelGGL(rx_ner_kernel, dim3(ceil_div(ner_cap, 256)), dim3(256), 0, s, ner, ner_cu, B, ner_cap,
                       cu_bytes, n, n_types, w.delta, w.starts, w.key, w.ner_type, err);
  launch_exclusive_scan_i32(w.delta, w.cover, n + 1, w.temp, s);
  hipLaunchKernelGGL(rx_flags_kernel, dim3(g), dim3(256), 0, s, w.cover, w.starts, n, w.fstart, w.fend);
  launch_exclusive_scan_i32(w.fstart, w.sstart, n + 1, w.temp, s);
  launch_exclusive_scan_i32(w.fend, w.send, n + 1, w.temp, s);
  hipLaunchKernelGGL(rx_runs_kernel, dim3(g), dim3(256), 0, s, w.fstart, w.sstart, w.fend, w.send, w.key, n,
                     w.run_begin, w.run_end, w.run_key);
  // the number of unions is sstart[n + 1]
  const int* n_runs = w.sstart + (n + 1);
  if (cap > 0)
    hipLaunchKernelGGL(rx_emit_kernel, dim3(ceil_div(cap, 256)), dim3(256), 0, s, n_runs, w.run_begin, w.run_end,
                       w.run_key, w.ner_type, cu_bytes, B, rt, out, cap);
  hipLaunchKernelGGL(rx_cu_kernel, dim3(ceil_div(B + 1, 256)), dim3(256), 0, s, n_runs, w.run_begin, cu_bytes, B,
                     cap, cu_spans, err);
}

}  // namespace anon
