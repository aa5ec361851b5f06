// Varlen self-attention over packed records (no padding), head dim 64.
//
// For each record and head: A = softmax(Q K^T / sqrt(d)) V over the keys of
// the same record only (bidirectional encoder attention).  Q already carries
// the 1/sqrt(d) = 1/8 factor (applied exactly in the QKV GEMM epilogue).
//
// BF16 operands (attn_stream_kernel): a persistent grid walks a work list of
// (record, head, block of 32*W query rows), longest records first.  Each
// workgroup streams the record's keys in tiles of KT through a two-stage LDS
// ring (K and V rows copied global -> LDS directly, XOR-swizzled), shared by
// its W waves, the next tile (also the next item's first) in flight while
// one is used; each wave owns 32 query rows and forms S^T = K Q^T with
// 32x32 MFMAs, so every lane holds the scores of one query row.  One pass:
// the probabilities are p = 2^(s log2(e) - r) against a running reference r
// that is an integer, the smallest one at or above max(s) log2(e) over the
// keys seen so far (updated every 64 keys, whatever the tile); when r grows,
// the FP32 output and row sum are rescaled by the exact power of two
// 2^(r_old - r_new).  A power-of-two reference scales every p by a power of
// two, so the bf16-rounded p are those of the final reference: the same
// values as rounding 2^(s log2(e) - ceil(max(s) log2(e))) with the record's
// true maximum, whatever the order of the keys.  The row sum is of the
// unrounded p; O^T += V^T P^T accumulates in FP32 and is divided by it at the
// end.  The MFMA k-index of P^T is a permutation of the 16 keys of a step; V
// is read transposed from LDS (ds_read_b64_tr_b16) in the same order.
//
// FP32 operands (attn_kernel, the plain FP32 path): work item = (q-block of
// 32*WAVES rows of one record, head); the block streams the record's keys in
// tiles of 64, K rows and V^T staged in LDS, in two passes: the first finds
// each row's exact maximum, the second forms p = exp(s - max) (FP32, base-2
// exponentials), sums it and accumulates O^T += V^T P^T.
#include <algorithm>

#include "kernels.hpp"

namespace anon {
namespace {

template <typename T>
struct AMfma;
template <>
struct AMfma<float> {
  typedef float frag;
  static constexpr int KI = 2, KPL = 1;
  __device__ static floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct AMfma<bf16_t> {
  typedef bf16x8 frag;
  static constexpr int KI = 16, KPL = 8;
  __device__ static floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ void st(float* p, float v) { *p = v; }
__device__ __forceinline__ void st(bf16_t* p, float v) { *p = static_cast<bf16_t>(v); }
__device__ __forceinline__ void st(fp8_t* p, float v) { p->v = f32_to_e4m3(v); }

// 2^x for x <= 0 with the bare v_exp_f32: results below 2^-126 may flush to
// zero, a difference far below the bf16 rounding of p and invisible in the
// FP32 row sums
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

constexpr int D = 64;    // head dim
constexpr int KT = 64;   // keys per LDS tile

// V^T fragment of PV step `st` in key block `kb` for lane half hh.
__device__ __forceinline__ float vfrag(const float* vrow, int kb, int st, int hh) {
  const int r = st;  // KPL = 1
  return vrow[kb * 32 + (r >> 2) * 8 + hh * 4 + (r & 3)];
}
__device__ __forceinline__ bf16x8 vfrag(const bf16_t* vrow, int kb, int st, int hh) {
  // registers 8*st .. 8*st+7 hold keys kb*32 + 16*st + hh*4 + {0..3} and
  // kb*32 + 16*st + 8 + hh*4 + {0..3}
  const bf16x4 lo = *(const bf16x4*)(vrow + kb * 32 + 16 * st + hh * 4);
  const bf16x4 hi = *(const bf16x4*)(vrow + kb * 32 + 16 * st + 8 + hh * 4);
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// V^T fragments of the record-resident kernel, read transposed from V kept
// row-major in LDS (64 elements per row; in rows with bit 1 set, bit 5 of the
// column is flipped).  ds_read_b64_tr_b16 works on groups of 16 lanes: each
// lane names a 4-element chunk, and lane j of the group receives element
// j % 4 of the chunks named by lanes j / 4 + 4k, k = 0..3.  Lane c of a group
// names row (base + c / 4), logical columns db*32 + 16*(group parity) +
// 4*(c % 4) (stored with the row's bit-5 flip), so
// lane l receives V[base + k][db*32 + l % 32], k = 0..3: four consecutive
// keys of its own V^T row.  base = kb*32 + 16*st + 8*q + 4*(l / 32) gives the
// same key order as the P^T fragment (pfrag).  For a half-wave the 4 rows x
// 32 columns then fall on 64 distinct banks.
__device__ __forceinline__ int vtr_lane_offset(int lane, int db) {
  const int c = lane & 15, g = (lane >> 4) & 1, hh = lane >> 5;
  // rows base + c/4 with base a multiple of 4: bit 1 of the row is bit 3 of
  // c; column bit 5 is db, flipped in those rows
  const int col = 16 * g + 4 * (c & 3) + ((((c >> 3) & 1) ^ db) << 5);
  return (hh * 4 + (c >> 2)) * D + col;
}
// vl: the lane's pointer for one 32-column half db (V + vtr_lane_offset)
__device__ __forceinline__ bf16x8 vfrag_tr(const bf16_t* vl, int kb, int st) {
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
  typedef __attribute__((address_space(3))) bf16_t lds_bf16;
  const bf16_t* p = vl + (kb * 32 + 16 * st) * D;
  const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(lds_bf16*)p);
  const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(lds_bf16*)(p + 8 * D));
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

template <typename T>
__device__ __forceinline__ typename AMfma<T>::frag pfrag(const floatx16& s, int st);
template <>
__device__ __forceinline__ float pfrag<float>(const floatx16& s, int st) {
  return s[st];
}
template <>
__device__ __forceinline__ bf16x8 pfrag<bf16_t>(const floatx16& s, int st) {
  bf16x8 f;
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] = static_cast<bf16_t>(s[st * 8 + j]);
  return f;
}

template <typename T, typename TO, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void attn_kernel(const T* __restrict__ qkv, TO* __restrict__ out,
                                                          const int4* __restrict__ qblocks,
                                                          const int* __restrict__ n_qblocks, int hidden,
                                                          float out_inv_scale, int window) {
  typedef AMfma<T> MF;
  typedef typename MF::frag frag;
  constexpr int NT = WAVES * 64;
  constexpr int EPC = 16 / (int)sizeof(T);
  constexpr int PAD = EPC;
  constexpr float LOG2E = 1.4426950408889634f;

  const int qb = blockIdx.x;
  if (qb >= *n_qblocks) return;
  const int head = blockIdx.y;
  const int4 desc = qblocks[qb];  // (first token, length, first query row, -)
  const int base = desc.x, L = desc.y, q0 = desc.z;
  const int ld = 3 * hidden;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hh = lane >> 5;
  const int qw = q0 + wave * 32;
  const bool active = qw < L;

  __shared__ T Ks[KT * (D + PAD)];
  __shared__ T Vt[D * (KT + PAD)];

  frag qf[D / MF::KI];
  const int qrow = qw + (lane & 31);
#pragma unroll
  for (int kk = 0; kk < D / MF::KI; ++kk) {
    if (qrow < L) {
      qf[kk] = *(const frag*)(qkv + (size_t)(base + qrow) * ld + head * D + kk * MF::KI + hh * MF::KPL);
    } else {
      qf[kk] = frag{};
    }
  }

  floatx16 o[2];
#pragma unroll
  for (int r = 0; r < 16; ++r) o[0][r] = o[1][r] = 0.f;
  float m = -INFINITY, lsum = 0.f;

  constexpr int CPR = D / EPC;  // 16-byte chunks per K/V row
  // scores of the current 64-key tile, base-2 scaled, -inf for missing keys
  auto scores = [&](floatx16 (&s)[2], int t0k, int nk) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[kb][r] = 0.f;
#pragma unroll
      for (int kk = 0; kk < D / MF::KI; ++kk) {
        const frag a = *(const frag*)&Ks[(kb * 32 + (lane & 31)) * (D + PAD) + kk * MF::KI + hh * MF::KPL];
        s[kb] = MF::mma(a, qf[kk], s[kb]);
      }
    }
    float mloc = -INFINITY;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int key = kb * 32 + (r >> 2) * 8 + hh * 4 + (r & 3);
        const int dk = qrow - (t0k + key);
        const bool seen = key < nk && (window <= 0 || (dk <= window && dk >= -window));
        const float v = seen ? s[kb][r] * LOG2E : -INFINITY;
        s[kb][r] = v;
        mloc = fmaxf(mloc, v);
      }
    return fmaxf(mloc, __shfl_xor(mloc, 32, 64));
  };
  auto load_tile = [&](int t0, int nk, bool with_v) {
    for (int c = tid; c < KT * CPR; c += NT) {
      const int r = c / CPR, cc = c % CPR;
      intx4 kv = {0, 0, 0, 0}, vv = {0, 0, 0, 0};
      if (r < nk) {
        const T* src = qkv + (size_t)(base + t0 + r) * ld + head * D + cc * EPC;
        kv = *(const intx4*)(src + hidden);
        if (with_v) vv = *(const intx4*)(src + 2 * hidden);
      }
      *(intx4*)&Ks[r * (D + PAD) + cc * EPC] = kv;
      if (with_v) {
        const T* ve = (const T*)&vv;
#pragma unroll
        for (int e = 0; e < EPC; ++e) Vt[(cc * EPC + e) * (KT + PAD) + r] = ve[e];
      }
    }
  };

  // Pass 1 (records longer than one tile): the exact row maximum, so that
  // the probabilities below are formed and rounded once, relative to it.
  const int ntiles = (L + KT - 1) / KT;
  if (ntiles > 1) {
    for (int t0 = 0; t0 < L; t0 += KT) {
      const int nk = min(KT, L - t0);
      __syncthreads();
      load_tile(t0, nk, false);
      __syncthreads();
      if (active) {
        floatx16 s[2];
        m = fmaxf(m, scores(s, t0, nk));
      }
    }
  }
  // Pass 2: p = exp(s - max), row sums in FP32, O^T += V^T P^T.
  for (int t0 = 0; t0 < L; t0 += KT) {
    const int nk = min(KT, L - t0);
    __syncthreads();
    load_tile(t0, nk, true);
    __syncthreads();
    if (active) {
      floatx16 s[2];
      const float mt = scores(s, t0, nk);
      if (ntiles == 1) m = mt;
      float ps = 0.f;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float pv = exp2_fast(s[kb][r] - m);
          s[kb][r] = pv;
          ps += pv;
        }
      lsum += ps;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int stp = 0; stp < 32 / MF::KI; ++stp) {
          const frag pb = pfrag<T>(s[kb], stp);
#pragma unroll
          for (int db = 0; db < 2; ++db) {
            const frag va = vfrag(&Vt[(db * 32 + (lane & 31)) * (KT + PAD)], kb, stp, hh);
            o[db] = MF::mma(va, pb, o[db]);
          }
        }
    }
  }
  if (active) {
    const float ltot = lsum + __shfl_xor(lsum, 32, 64);
    const float inv = 1.0f / ltot;
    if (qrow < L) {
      TO* dst = out + (size_t)(base + qrow) * hidden + head * D;
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float v = o[db][r] * inv;
          // FP8 output: round to bf16 (the stored attention output), then
          // scale and round to E4M3
          if (sizeof(TO) == 1) v = static_cast<float>(static_cast<bf16_t>(v)) * out_inv_scale;
          st(dst + db * 32 + (r >> 2) * 8 + hh * 4 + (r & 3), v);
        }
    }
  }
}

// ---- BF16 streaming kernel ------------------------------------------------
// Tile configurations: W waves (32 query rows each, so 32*W rows per work
// item), KT keys per LDS tile, WPE waves per SIMD the register budget is
// held to, SW the form of the output stores (1: 16-byte BF16 or 8-byte FP8
// stores after a half-wave exchange, 0: stores of the accumulator quads;
// which is faster depends on the record lengths).  Results do not depend on the
// configuration: every query row sees the same keys in the same 64-key
// reference steps, and both store forms write the same bytes.
struct AttnCfg {
  int w, kt, wpe;
  const char* name;
};
#define ANON_ATTN_CFGS(X)                    \
  X(0, 4, 64, 4, 1, "attn_w4_kt64_o4")       \
  X(1, 4, 64, 3, 1, "attn_w4_kt64_o3")       \
  X(2, 8, 64, 4, 1, "attn_w8_kt64_o4")       \
  X(3, 2, 64, 3, 1, "attn_w2_kt64_o3")       \
  X(4, 8, 128, 3, 1, "attn_w8_kt128_o3")     \
  X(5, 8, 64, 4, 0, "attn_w8_kt64_o4_st8")
#define ANON_ATTN_ROW(i, w, kt, wpe, sw, name) {w, kt, wpe, name},
const AttnCfg kAttnCfg[] = {ANON_ATTN_CFGS(ANON_ATTN_ROW)};
constexpr int kAttnCfgs = (int)(sizeof(kAttnCfg) / sizeof(AttnCfg));
constexpr int kAttnDefault = 0;
constexpr int kRowBytes = D * 2;  // one K or V row (64 bf16)
constexpr int kStages = 2;        // LDS ring: the tile being used and the one in flight

// K rows: 16-byte chunk c of row r sits in slot c ^ ((r >> 1) & 7), so the
// 16-byte fragment reads of 16 consecutive rows (one logical chunk) fall on
// 16 distinct bank groups.  V rows: chunk c of row r sits in slot
// c ^ (4 * ((r >> 1) & 1)), the layout the transposing reads expect
// (vtr_lane_offset).
__device__ __forceinline__ int kswz(int r) { return (r >> 1) & 7; }
__device__ __forceinline__ int vswz(int r) { return ((r >> 1) & 1) << 2; }

// A workgroup's walk over its work items and their key tiles.
struct Walk {
  int wi, t, nt;       // work item, tile within it, tiles of the item
  int base, L, q0, head;
};

template <typename TO, int W, int KT, int WPE, int SW>
__global__ __launch_bounds__(W * 64, WPE) void attn_stream_kernel(const bf16_t* __restrict__ qkv,
                                                                  TO* __restrict__ out,
                                                                  const int4* __restrict__ items,
                                                                  const int* __restrict__ n_items, int n_heads,
                                                                  int hidden, float out_inv_scale, int window) {
  typedef AMfma<bf16_t> MF;
  typedef bf16x8 frag;
  constexpr float LOG2E = 1.4426950408889634f;
  constexpr int TILE = KT * kRowBytes;   // bytes of the K (or V) rows of one tile
  constexpr int STAGE = 2 * TILE;
  constexpr int INS = KT / 8;            // load instructions per tile and matrix (8 rows of 128 B each)
  static_assert(INS % W == 0, "every wave issues the same number of loads");
  constexpr int IPW = INS / W;           // per wave, per matrix
  constexpr int NB = KT / 32;            // 32-key blocks per tile
  static_assert(KT % 64 == 0, "tile shape");
  __shared__ __align__(1024) char smem[kStages * STAGE];

  const int n_work = *n_items * n_heads;
  const int tid = threadIdx.x, lane = tid & 63, hh = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ld = 3 * hidden;
  // this lane's part of each load instruction: row (lane / 8) of the 8,
  // LDS slot (lane % 8); and its K fragment offsets within a stage
  const int lrow = lane >> 3, lslot = lane & 7;
  int koff[NB][D / 16];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int kk = 0; kk < D / 16; ++kk) {
      const int row = b * 32 + (lane & 31);
      koff[b][kk] = row * kRowBytes + (((kk * 2 + hh) ^ kswz(row)) * 16);
    }
  const int vl_off0 = TILE + 2 * vtr_lane_offset(lane, 0), vl_off1 = TILE + 2 * vtr_lane_offset(lane, 1);

  // with a window, an item's rows [q0, q0 + 32W) only see the key tiles
  // that meet [q0 - window, q0 + 32W - 1 + window]
  auto start = [&](Walk& c, int wi) {
    c.wi = wi;
    if (wi < n_work) {
      const int it = wi / n_heads;
      c.head = wi - it * n_heads;
      const int4 d = items[it];  // (first token, length, first query row, -)
      c.base = d.x, c.L = d.y, c.q0 = d.z;
      c.t = 0;
      c.nt = (c.L + KT - 1) / KT;
      if (window > 0) {
        c.t = max(c.q0 - window, 0) / KT;
        c.nt = min(c.q0 + 32 * W - 1 + window, c.L - 1) / KT + 1;
      }
    }
  };
  // tile c.t of work item c into ring stage st: rows past the record re-read
  // its last row (never used: their scores are masked, their p are zero)
  // the lane's byte offsets within a K row and a V row (its swizzled chunk)
  int kchunk[IPW], vchunk[IPW];
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    const int row = (wave * IPW + i) * 8 + lrow;
    kchunk[i] = (lslot ^ kswz(row)) * 16;
    vchunk[i] = 2 * hidden + (lslot ^ vswz(row)) * 16;
  }
  auto issue = [&](const Walk& c, int st) {
    // the record's first K row of this head (uniform), then 32-bit offsets
    const char* kb = (const char*)(qkv + (size_t)c.base * ld + hidden + c.head * D);
    char* sk = smem + st * STAGE;
    const int last = c.L - 1;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int row = (wave * IPW + i) * 8 + lrow;
      const uint32_t ro = (uint32_t)min(c.t * KT + row, last) * (uint32_t)(2 * ld);
      dma16(kb + ro + kchunk[i], sk + (wave * IPW + i) * 1024);
      dma16(kb + ro + vchunk[i], sk + TILE + (wave * IPW + i) * 1024);
    }
  };
  frag qf[D / 16];
  auto load_q = [&](const Walk& c) {
    const int qrow = c.q0 + wave * 32 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < D / 16; ++kk)
      qf[kk] = qrow < c.L ? *(const frag*)(qkv + (size_t)(c.base + qrow) * ld + c.head * D + kk * 16 + hh * 8)
                          : frag{};
  };

  // The issue walk runs one tile ahead of the compute walk, also across work
  // items: while the last tile of an item is used, the first tile of the
  // next is in flight, and the next item's Q rows are loaded during the
  // last tile of the one before it.
  // inx: the item after the issue walk's, its descriptor loaded one item
  // ahead so that a switch of the issue walk waits for no load
  Walk cw, iw, inx;
  start(cw, blockIdx.x);
  if (cw.wi >= n_work) return;
  iw = cw;
  start(inx, iw.wi + gridDim.x);
  issue(iw, 0);
  load_q(cw);
  floatx16 o[2];
  float lsum, ref;
  auto reset = [&]() {
#pragma unroll
    for (int r = 0; r < 16; ++r) o[0][r] = o[1][r] = 0.f;
    lsum = 0.f;
    ref = -INFINITY;
  };
  reset();

  // one tile from stage ST (a compile-time constant: the loop body is
  // unrolled over the two stages); returns false when the walk is over
  auto step = [&](auto stc) -> bool {
    constexpr int ST = decltype(stc)::value;
    // tile cw.t (and, after a switch, the item's Q rows) has landed for this
    // wave; after the barrier for everyone, who have also finished the
    // previous tile, whose stage takes the next one
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (++iw.t == iw.nt && iw.wi < n_work) {
      iw = inx;
      if (iw.wi < n_work) start(inx, iw.wi + gridDim.x);
    }
    if (iw.wi < n_work) issue(iw, ST ^ 1);
    const int qw = cw.q0 + wave * 32;  // this wave's first query row
    const bool active = qw < cw.L;
    // On the item's last tile the next item's Q rows go into qf as soon as
    // the tile's last QK products have read it, so their load runs behind
    // this tile's softmax and P V instead of ahead of the next tile.
    const bool last = cw.t + 1 == cw.nt;
    // the issue walk, one tile ahead, is at the next item's first tile now
    const Walk nw = iw;
    bool q_loaded = !last;
    auto next_q = [&]() {
      if (!q_loaded) {
        if (nw.wi < n_work) load_q(nw);
        q_loaded = true;
      }
    };
    if (active) {
      const char* ks = smem + ST * STAGE;
      const bool last_partial = (cw.t + 1) * KT > cw.L;
      // the last 64-key step of this tile that can run (keys left in the record)
      const int h_last = min(KT / 64, (cw.L - cw.t * KT + 63) / 64) - 1;
#pragma unroll
      for (int h64 = 0; h64 < KT / 64; ++h64) {
        // keys of this 64-key step still inside the record (uniform)
        const int k0 = cw.t * KT + h64 * 64;
        const int nv = cw.L - k0;
        if (nv <= 0) break;
        // with a window: steps outside this wave's band are skipped, steps
        // across its edge are masked key by key
        bool band_edge = false;
        if (window > 0) {
          if (k0 > qw + 31 + window || k0 + 63 < qw - window) continue;
          band_edge = k0 < qw + 31 - window || k0 + 63 > qw + window;
        }
        // scores of the 64 keys [t*KT + 64*h64, +64): two 32-key blocks
        // (the second only if it holds keys of the record)
        const bool two = nv > 32;
        floatx16 s[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (b == 1 && !two) break;
#pragma unroll
          for (int r = 0; r < 16; ++r) s[b][r] = 0.f;
#pragma unroll
          for (int kk = 0; kk < D / 16; ++kk) {
            const frag a = *(const frag*)(ks + koff[h64 * 2 + b][kk]);
            s[b] = MF::mma(a, qf[kk], s[b]);
          }
        }
        if (h64 == h_last) next_q();
        if (band_edge) {
          // key k of this lane's query q is seen iff |q - k| <= window
          const int dq = qw + (lane & 31) - (k0 + hh * 4);  // q - (key of r = 0 in block 0)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            if (b == 1 && !two) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int dk = dq - (b * 32 + (r >> 2) * 8 + (r & 3));
              if (dk > window || dk < -window) s[b][r] = -INFINITY;
            }
          }
        }
        // the block holding the record's end: keys past it -> -inf
        if (last_partial && nv < 64 && (nv & 31) != 0) {
          const int b = nv >> 5;
          const int thr = (nv & 31) - hh * 4;  // key (r>>2)*8 + (r&3) of this lane is valid iff below thr
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const bool past = (r >> 2) * 8 + (r & 3) >= thr;
            if (b == 0) s[0][r] = past ? -INFINITY : s[0][r];
            else s[1][r] = past ? -INFINITY : s[1][r];
          }
        }
        // reference update: the smallest integer at or above max * log2(e)
        float mx = -INFINITY;
        if (two) {
#pragma unroll
          for (int r = 0; r < 16; ++r) mx = fmaxf(mx, fmaxf(s[0][r], s[1][r]));
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) mx = fmaxf(mx, s[0][r]);
        }
        mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
        const float rn = ceilf(mx * LOG2E);
        if (rn > ref) {  // never for 64 keys all past the record (mx = -inf)
          if (ref > -INFINITY) {
            const int dl = (int)(ref - rn);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              o[0][r] = ldexpf(o[0][r], dl);
              o[1][r] = ldexpf(o[1][r], dl);
            }
            lsum = ldexpf(lsum, dl);
          }
          ref = rn;
        }
        // p = 2^(s log2(e) - ref); row sums of the unrounded p; O^T += V^T P^T
        // (a row that has seen no key yet has only -inf scores here: any
        // finite reference gives p = 0)
        const float nref = ref > -INFINITY ? ref : 0.f;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (b == 1 && !two) break;  // a block wholly past the record adds nothing
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float p = exp2_fast(fmaf(s[b][r], LOG2E, -nref));
            s[b][r] = p;
            lsum += p;
          }
#pragma unroll
          for (int stp = 0; stp < 2; ++stp) {
            const frag pb = pfrag<bf16_t>(s[b], stp);
            const int kb = h64 * 2 + b;
            const bf16_t* v0 = (const bf16_t*)(smem + ST * STAGE + vl_off0);
            const bf16_t* v1 = (const bf16_t*)(smem + ST * STAGE + vl_off1);
            o[0] = MF::mma(vfrag_tr(v0, kb, stp), pb, o[0]);
            o[1] = MF::mma(vfrag_tr(v1, kb, stp), pb, o[1]);
          }
        }
      }
    }
    next_q();  // (a wave without rows here, or a window that skipped the last steps)
    if (++cw.t < cw.nt) return true;
    // the item is done: normalise and store, then start the next one
    if (active && SW && sizeof(TO) == 2) {
      // BF16 output.  The two half-waves hold the same 32 rows, in quads of
      // 4 columns that alternate between them (columns 8g + 4hh + 0..3 of
      // quad g); exchanging quads 1 and 3 of the lower half with quads 0 and
      // 2 of the upper half (v_permlane32_swap) leaves every lane 8
      // consecutive columns, which go out in 16-byte stores: half the
      // store instructions, each touching 32 rows as before.
      const int qrow = cw.q0 + wave * 32 + (lane & 31);
      const float inv = 1.0f / (lsum + __shfl_xor(lsum, 32, 64));
      uint32_t w[2][4][2];
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const uint32_t lo = __builtin_bit_cast(uint16_t, static_cast<bf16_t>(o[db][g * 4 + 2 * k] * inv));
            const uint32_t hi = __builtin_bit_cast(uint16_t, static_cast<bf16_t>(o[db][g * 4 + 2 * k + 1] * inv));
            w[db][g][k] = lo | (hi << 16);
          }
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int g = 0; g < 4; g += 2)
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            // lower lanes keep quad g and take the upper half's quad g;
            // upper lanes take the lower half's quad g+1 and keep theirs
            const auto r = __builtin_amdgcn_permlane32_swap(w[db][g][k], w[db][g + 1][k], false, false);
            w[db][g][k] = r[0];
            w[db][g + 1][k] = r[1];
          }
      if (qrow < cw.L) {
        TO* dst = out + (size_t)(cw.base + qrow) * hidden + cw.head * D;
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int g = 0; g < 4; g += 2)
            *(uint4*)(dst + db * 32 + g * 8 + hh * 8) =
                uint4{w[db][g][0], w[db][g][1], w[db][g + 1][0], w[db][g + 1][1]};
      }
    } else if (active && SW && sizeof(TO) == 1) {
      // FP8 output: the same exchange on one dword (four E4M3 values) per
      // quad, then 8-byte stores of 8 consecutive columns
      const int qrow = cw.q0 + wave * 32 + (lane & 31);
      const float inv = 1.0f / (lsum + __shfl_xor(lsum, 32, 64));
      uint32_t w[2][4];
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          uint32_t x = 0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            // rounded to bf16 (the stored attention output), then scaled
            // and rounded to E4M3, as element by element below
            const float v = static_cast<float>(static_cast<bf16_t>(o[db][g * 4 + e] * inv)) * out_inv_scale;
            x |= (uint32_t)f32_to_e4m3(v) << (8 * e);
          }
          w[db][g] = x;
        }
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int g = 0; g < 4; g += 2) {
          const auto r = __builtin_amdgcn_permlane32_swap(w[db][g], w[db][g + 1], false, false);
          w[db][g] = r[0];
          w[db][g + 1] = r[1];
        }
      if (qrow < cw.L) {
        TO* dst = out + (size_t)(cw.base + qrow) * hidden + cw.head * D;
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int g = 0; g < 4; g += 2) *(uint2*)(dst + db * 32 + g * 8 + hh * 8) = uint2{w[db][g], w[db][g + 1]};
      }
    } else if (active) {
      const int qrow = cw.q0 + wave * 32 + (lane & 31);
      const float inv = 1.0f / (lsum + __shfl_xor(lsum, 32, 64));
      if (qrow < cw.L) {
        TO* dst = out + (size_t)(cw.base + qrow) * hidden + cw.head * D;
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float v = o[db][r] * inv;
            // FP8 output: round to bf16 (the stored attention output), then
            // scale and round to E4M3
            if (sizeof(TO) == 1) v = static_cast<float>(static_cast<bf16_t>(v)) * out_inv_scale;
            st(dst + db * 32 + (r >> 2) * 8 + hh * 4 + (r & 3), v);
          }
      }
    }
    cw = nw;
    if (cw.wi >= n_work) return false;
    reset();
    return true;
  };
  while (step(std::integral_constant<int, 0>()) && step(std::integral_constant<int, 1>())) {
  }
}

constexpr int kWaves = 4;
constexpr int kBQ = 32 * kWaves;

// One workgroup: validates cu_seqlens and lists (first token, length, first
// query row, record) items of bq query rows for the records whose length
// lies in [lo, hi].
__global__ __launch_bounds__(1024) void seq_plan_kernel(const int* __restrict__ cu, int B, int T_cap, int max_len,
                                                        int lo, int hi, int bq, int4* __restrict__ qblocks,
                                                        int max_q, int* __restrict__ n_qblocks, uint32_t* err,
                                                        const int* t_dev) {
  // Malformed (overlapping) cu_seqlens could ask for more items than the
  // buffer holds; writes stop at max_q and the error bit is raised.
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
  const int T = live_rows(T_cap, t_dev);
  if (tid == 0 && t_dev && *t_dev != T) raise_error(err, ANON_ERR_SEQLENS);
  const int per = (B + 1023) / 1024;
  const int s0 = min(B, tid * per), s1 = min(B, s0 + per);
  int cnt = 0;
  bool bad = false;
  for (int s = s0; s < s1; ++s) {
    const int a = cu[s], b = cu[s + 1];
    const int L = b - a;
    if (a < 0 || b > T || L < 0 || L > max_len) {
      bad = true;
      continue;
    }
    if (L >= lo && L <= hi) cnt += (L + bq - 1) / bq;
  }
  if (tid == 0 && (cu[0] != 0 || cu[B] != T)) bad = true;
  if (bad) raise_error(err, ANON_ERR_SEQLENS);
  sums[tid] = cnt;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = tid >= o ? sums[tid - o] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int pos = sums[tid] - cnt;
  for (int s = s0; s < s1; ++s) {
    const int a = cu[s], b = cu[s + 1];
    const int L = b - a;
    if (a < 0 || b > T || L < 0 || L > max_len) continue;
    if (L < lo || L > hi) continue;
    for (int q = 0; q < L && pos < max_q; q += bq) qblocks[pos++] = int4{a, L, q, s};
  }
  if (tid == 1023) {
    const int total = sums[1023];
    if (total > max_q) raise_error(err, ANON_ERR_SEQLENS);
    *n_qblocks = min(total, max_q);
  }
}

// One workgroup: the BF16 kernel's work list, longest records first (in
// bins of 32 keys), each record split into items of bq query rows.
__global__ __launch_bounds__(1024) void stream_plan_kernel(const int* __restrict__ cu, int B, int T_cap,
                                                           int max_len, int bq, int4* __restrict__ items,
                                                           int max_items, int* __restrict__ n_items, uint32_t* err,
                                                           const int* t_dev) {
  __shared__ int sums[1024];
  __shared__ int run;
  const int tid = threadIdx.x;
  const int T = live_rows(T_cap, t_dev);
  if (tid == 0 && t_dev && *t_dev != T) raise_error(err, ANON_ERR_SEQLENS);
  const int per = (B + 1023) / 1024;
  const int s0 = min(B, tid * per), s1 = min(B, s0 + per);
  bool bad = false;
  for (int s = s0; s < s1; ++s) {
    const int a = cu[s], b = cu[s + 1];
    if (a < 0 || b > T || b < a || b - a > max_len) bad = true;
  }
  if (tid == 0 && (cu[0] != 0 || cu[B] != T)) bad = true;
  if (bad) raise_error(err, ANON_ERR_SEQLENS);
  if (tid == 0) run = 0;
  const int nbins = (max_len + 31) / 32;
  for (int bin = nbins - 1; bin >= 0; --bin) {
    int cnt = 0;
    for (int s = s0; s < s1; ++s) {
      const int a = cu[s], b = cu[s + 1], L = b - a;
      if (a < 0 || b > T || L < 1 || L > max_len || (L - 1) / 32 != bin) continue;
      cnt += (L + bq - 1) / bq;
    }
    __syncthreads();  // `run` is final, `sums` free
    sums[tid] = cnt;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = tid >= o ? sums[tid - o] : 0;
      __syncthreads();
      sums[tid] += v;
      __syncthreads();
    }
    int pos = run + sums[tid] - cnt;
    for (int s = s0; s < s1; ++s) {
      const int a = cu[s], b = cu[s + 1], L = b - a;
      if (a < 0 || b > T || L < 1 || L > max_len || (L - 1) / 32 != bin) continue;
      for (int q = 0; q < L; q += bq, ++pos)
        if (pos < max_items) items[pos] = int4{a, L, q, s};
    }
    __syncthreads();  // every thread has read `run`
    if (tid == 1023) run += sums[1023];
  }
  __syncthreads();
  if (tid == 0) {
    if (run > max_items) raise_error(err, ANON_ERR_SEQLENS);
    *n_items = min(run, max_items);
  }
}

bool streamed(ElemType t) { return t == ET_BF16; }

int workgroups_per_cu(const AttnCfg& c) {
  const int by_regs = c.wpe * 4 / c.w;
  const int by_lds = 163840 / (kStages * 2 * c.kt * kRowBytes);
  return std::max(1, std::min(by_regs, by_lds));
}

template <typename TO, int W, int KT, int WPE, int SW>
void launch_stream(const bf16_t* qkv, TO* out, const int4* items, const int* n_items, int n_heads, int hidden,
                   float out_inv_scale, int window, int grid, hipStream_t s) {
  hipLaunchKernelGGL((attn_stream_kernel<TO, W, KT, WPE, SW>), dim3(grid), dim3(W * 64), 0, s, qkv, out, items,
                     n_items, n_heads, hidden, out_inv_scale, window);
}

template <typename TO>
void dispatch_stream(int ci, const bf16_t* qkv, TO* out, const int4* items, const int* n_items, int n_heads,
                     int hidden, float out_inv_scale, int window, int grid, hipStream_t s) {
#define ANON_ATTN_CASE(i, w, kt, wpe, sw, name)                                                                    \
  case i:                                                                                                          \
    launch_stream<TO, w, kt, wpe, sw>(qkv, out, items, n_items, n_heads, hidden, out_inv_scale, window, grid, s); \
    return;
  switch (ci) { ANON_ATTN_CFGS(ANON_ATTN_CASE) }
#undef ANON_ATTN_CASE
}

int cfg_index(int config) { return config >= 0 && config < kAttnCfgs ? config : kAttnDefault; }

}  // namespace

int attn_num_configs() { return kAttnCfgs; }

const char* attn_config_name(int config) {
  return config >= 0 && config < kAttnCfgs ? kAttnCfg[config].name : "?";
}

int attn_plan_items(ElemType t, int config, int T, int B) {
  // at most T / bq + B items of bq query rows
  const int bq = streamed(t) ? 32 * kAttnCfg[cfg_index(config)].w : kBQ;
  return T / bq + B + 1;
}

void launch_attn_plan(const int* cu_seqlens, int B, int T, int max_len, ElemType t, int config, int4* items,
                      int max_items, int* n_items, uint32_t* err, hipStream_t s, const int* t_dev) {
  if (streamed(t)) {
    const int bq = 32 * kAttnCfg[cfg_index(config)].w;
    hipLaunchKernelGGL(stream_plan_kernel, dim3(1), dim3(1024), 0, s, cu_seqlens, B, T, max_len, bq, items,
                       max_items, n_items, err, t_dev);
  } else {
    hipLaunchKernelGGL(seq_plan_kernel, dim3(1), dim3(1024), 0, s, cu_seqlens, B, T, max_len, 0, max_len, kBQ,
                       items, max_items, n_items, err, t_dev);
  }
}

void launch_attention(const void* qkv, void* out, const int4* items, int max_items, const int* n_items,
                      int n_heads, int hidden, ElemType t, ElemType out_t, float out_inv_scale, int config,
                      hipStream_t s, int window) {
  if (max_items <= 0) return;
  if (streamed(t)) {
    const int ci = cfg_index(config);
    // a persistent grid: as many workgroups as the CUs hold at once (no more
    // than there can be work items)
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = (int)std::min<int64_t>((int64_t)n_cu * workgroups_per_cu(kAttnCfg[ci]),
                                            (int64_t)max_items * n_heads);
    if (out_t == ET_FP8)
      dispatch_stream(ci, static_cast<const bf16_t*>(qkv), (fp8_t*)out, items, n_items, n_heads, hidden,
                      out_inv_scale, window, grid, s);
    else
      dispatch_stream(ci, static_cast<const bf16_t*>(qkv), (bf16_t*)out, items, n_items, n_heads, hidden,
                      out_inv_scale, window, grid, s);
    return;
  }
  dim3 grid(max_items, n_heads);
  if (t == ET_F32) {
    hipLaunchKernelGGL((attn_kernel<float, float, kWaves>), grid, dim3(kWaves * 64), 0, s, (const float*)qkv,
                       (float*)out, items, n_items, hidden, out_inv_scale, window);
  } else if (out_t == ET_FP8) {
    hipLaunchKernelGGL((attn_kernel<bf16_t, fp8_t, kWaves>), grid, dim3(kWaves * 64), 0, s, (const bf16_t*)qkv,
                       (fp8_t*)out, items, n_items, hidden, out_inv_scale, window);
  } else {
    hipLaunchKernelGGL((attn_kernel<bf16_t, bf16_t, kWaves>), grid, dim3(kWaves * 64), 0, s, (const bf16_t*)qkv,
                       (bf16_t*)out, items, n_items, hidden, out_inv_scale, window);
  }
}

}  // namespace anon
