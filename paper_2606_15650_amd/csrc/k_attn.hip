// Varlen self-attention over packed records (no padding), head dim 64.
//
// For each record and head: A = softmax(Q K^T / sqrt(d)) V over the keys of
// the same record only (bidirectional encoder attention).  Q already carries
// the 1/sqrt(d) = 1/8 factor (applied exactly in the QKV GEMM epilogue).
//
// Two kernels.  BF16 operands (records of at most 512 keys): one workgroup
// per (record, head) holds the record's whole K and V in LDS, V read back
// transposed (attn_resident_kernel, below).  FP32 operands: work item =
// (q-block of 32*WAVES rows of one record, head); the block streams the
// record's keys in tiles of 64, K rows and V^T staged in LDS.  In both, each
// wave owns 32 query rows and computes S^T = K Q^T with 32x32 MFMAs, so that
// every lane holds the scores of one query row.  Records longer than one key
// block take two passes over their keys: the first finds each row's exact
// maximum, the second forms p = exp(s - max) once (FP32, base-2
// exponentials), sums it in FP32, rounds it to the operand type and
// accumulates O^T += V^T P^T in FP32.  Rounding p relative to the final
// maximum (not a running one) makes the rounded values a function of the
// record alone, identical to the definition softmax(s) = exp(s - max) / sum.
// The MFMA k-index of P^T is a permutation of the 32 keys of a block; V^T is
// read from LDS with the same permutation, so the contraction is exact.
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
                                                          float out_inv_scale) {
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
  auto scores = [&](floatx16 (&s)[2], int nk) {
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
        const float v = key < nk ? s[kb][r] * LOG2E : -INFINITY;
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
        m = fmaxf(m, scores(s, nk));
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
      const float mt = scores(s, nk);
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

// Record-resident variant (bf16 operands, records of at most RMAX keys).
// One workgroup per (record, head) stages the record's whole K (row-major)
// and V^T in LDS once; its waves then take 32-row query chunks in turn and
// run both passes over the resident keys with no further barrier.  The V^T
// row stride (RMAX + 12 elements, 6 mod 64 dwords) keeps the 8-byte reads of
// 32 lanes on distinct banks.  Records are binned by length so that RMAX and
// the wave count follow the record (see kClassMax).
// LDS bytes of a record-resident workgroup (V rows unpadded, K rows padded
// by 8 elements) and the waves per SIMD that as many workgroups as fit
// in the 160 KB of a CU's LDS bring; the register budget is held to that
// occupancy.
constexpr int resident_lds_bytes(int rmax) { return (rmax * D + rmax * (D + 8)) * 2; }
constexpr int resident_waves_per_eu(int rmax, int waves) {
  return (163840 / resident_lds_bytes(rmax)) * waves / 4;
}

template <typename TO, int RMAX, int WAVES>
__global__ __launch_bounds__(WAVES * 64, resident_waves_per_eu(RMAX, WAVES)) void attn_resident_kernel(const bf16_t* __restrict__ qkv,
                                                                   TO* __restrict__ out,
                                                                   const int4* __restrict__ recs,
                                                                   const int* __restrict__ n_recs, int hidden,
                                                                   float out_inv_scale) {
  typedef AMfma<bf16_t> MF;
  typedef bf16x8 frag;
  constexpr int KS = D + 8;       // K row stride (16 bytes of padding)
  constexpr float LOG2E = 1.4426950408889634f;
  const int rb = blockIdx.x;
  if (rb >= *n_recs) return;
  const int head = blockIdx.y;
  const int4 desc = recs[rb];
  const int base = desc.x, L = desc.y;
  const int ld = 3 * hidden;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, hh = lane >> 5;

  // V first: its reads then sit below 64 KB, within reach of the
  // instructions' immediate offsets.  V is kept row-major (key, d), 64
  // elements per row, with bit 5 of the column flipped in rows whose bit 1 is
  // set; the PV step reads it transposed (vfrag_tr).
  __shared__ __align__(16) bf16_t lds[RMAX * D + RMAX * KS];
  static_assert(sizeof(lds) == resident_lds_bytes(RMAX), "LDS size");
  bf16_t* const Vs = lds;
  bf16_t* const Ks = lds + RMAX * D;

  // A workgroup has one wave per 32 keys of the class bound, so every thread
  // stages exactly NSTG 16-byte chunks of K and of V, and every wave owns at
  // most one 32-row query chunk.  All of the thread's loads (its K and V
  // chunks and its wave's Q fragments) are issued before the first LDS
  // write, so the workgroup waits for one memory round trip, not one per
  // chunk.
  constexpr int NT = WAVES * 64;
  constexpr int NSTG = RMAX * 8 / NT;
  static_assert(RMAX == 32 * WAVES && NSTG * NT == RMAX * 8, "one wave per 32 keys");
  const int Lp = (L + 31) & ~31;  // keys padded with zeros to whole 32-key blocks
  intx4 kv[NSTG], vv[NSTG];
#pragma unroll
  for (int i = 0; i < NSTG; ++i) {
    const int c = tid + i * NT, r = c >> 3, cc = c & 7;
    kv[i] = intx4{0, 0, 0, 0};
    vv[i] = intx4{0, 0, 0, 0};
    if (r < L) {
      const bf16_t* src = qkv + (size_t)(base + r) * ld + head * D + cc * 8;
      kv[i] = *(const intx4*)(src + hidden);
      vv[i] = *(const intx4*)(src + 2 * hidden);
    }
  }
  const int nkb = Lp / 32;
  const int nqc = (L + 31) / 32;
  const bool partial = (L & 31) != 0;  // only the last key block has missing keys
  const int qc = wave;
  const int qrow = qc * 32 + (lane & 31);
  frag qf[D / 16];
#pragma unroll
  for (int kk = 0; kk < D / 16; ++kk)
    qf[kk] = qrow < L ? *(const frag*)(qkv + (size_t)(base + qrow) * ld + head * D + kk * 16 + hh * 8) : frag{};
#pragma unroll
  for (int i = 0; i < NSTG; ++i) {
    const int c = tid + i * NT, r = c >> 3, cc = c & 7;
    if (r < Lp) {
      *(intx4*)&Ks[r * KS + cc * 8] = kv[i];
      *(intx4*)&Vs[r * D + (cc ^ (((r >> 1) & 1) << 2)) * 8] = vv[i];
    }
  }
  __syncthreads();

  if (qc < nqc) {
    // raw scores S^T of key block kb; missing keys of the last block -> -inf
    auto qk = [&](int kb, floatx16& s) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[r] = 0.f;
#pragma unroll
      for (int kk = 0; kk < D / 16; ++kk) {
        const frag a = *(const frag*)&Ks[(kb * 32 + (lane & 31)) * KS + kk * 16 + hh * 8];
        s = MF::mma(a, qf[kk], s);
      }
      if (partial && kb == nkb - 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (kb * 32 + (r >> 2) * 8 + hh * 4 + (r & 3) >= L) s[r] = -INFINITY;
      }
    };
    const bf16_t* const vl0 = Vs + vtr_lane_offset(lane, 0);
    const bf16_t* const vl1 = Vs + vtr_lane_offset(lane, 1);
    // pass 1: row maximum of the raw scores (the scale is positive, so the
    // maximum of the scaled scores is the scaled maximum)
    // Both passes are software-pipelined two blocks deep: the next block's
    // QK^T MFMAs are issued before the current block's VALU work (maximum,
    // exponentials), which then runs while the matrix core is busy.
    float mraw = -INFINITY;
    auto rowmax = [&](const floatx16& s) {
#pragma unroll
      for (int r = 0; r < 16; ++r) mraw = fmaxf(mraw, s[r]);
    };
    floatx16 sa, sb;
    qk(0, sa);
    if (nkb > 1) {
      for (int kb = 0; kb < nkb; kb += 2) {
        if (kb + 1 < nkb) qk(kb + 1, sb);
        rowmax(sa);
        if (kb + 1 < nkb) {
          if (kb + 2 < nkb) qk(kb + 2, sa);
          rowmax(sb);
        }
      }
    } else {
      rowmax(sa);
    }
    // sa and sb now hold the raw scores of the last two blocks, nkb-2 and
    // nkb-1 (sa holds nkb-1 when nkb is odd), or sa holds block 0 alone
    mraw = fmaxf(mraw, __shfl_xor(mraw, 32, 64));
    // K fragments are read from LDS again in pass 2 rather than kept live
    // across pass 1 (no instruction: it only stops the compiler from reusing
    // pass-1 loads, which would cost registers it does not have)
    __asm__ volatile("" ::: "memory");
    floatx16 o[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) o[0][r] = o[1][r] = 0.f;
    float lsum = 0.f;
    // pass 2: p = 2^(s*log2(e) - max*log2(e)) = exp(s - max), O^T += V^T P^T
    auto pv = [&](int kb, floatx16& s, floatx16 (&acc)[2]) {
      const float mb = mraw * LOG2E;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float p = exp2_fast(fmaf(s[r], LOG2E, -mb));
        s[r] = p;
        lsum += p;
      }
#pragma unroll
      for (int stp = 0; stp < 2; ++stp) {
        const frag pb = pfrag<bf16_t>(s, stp);
#pragma unroll
        for (int db = 0; db < 2; ++db) acc[db] = MF::mma(vfrag_tr(db ? vl1 : vl0, kb, stp), pb, acc[db]);
      }
    };
    // Pass 2 takes the blocks in the order nkb-2, nkb-1 (still in registers,
    // not recomputed), then 0 .. nkb-3: a fixed order given by the record's
    // length alone.  X holds the first block of the order, Y the second.
    auto pass2 = [&](floatx16& X, floatx16& Y) {
      const int first = nkb > 1 ? nkb - 2 : 0;
      auto seq = [&](int i) { return i < 2 ? first + i : i - 2; };
      pv(seq(0), X, o);
      for (int i = 1; i < nkb; i += 2) {
        if (i + 1 < nkb) qk(seq(i + 1), X);
        pv(seq(i), Y, o);
        if (i + 1 < nkb) {
          if (i + 2 < nkb) qk(seq(i + 2), Y);
          pv(seq(i + 1), X, o);
        }
      }
    };
    if (nkb > 1 && (nkb & 1)) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float t = sa[r];
        sa[r] = sb[r];
        sb[r] = t;
      }
    }
    pass2(sa, sb);
    const float ltot = lsum + __shfl_xor(lsum, 32, 64);
    const float inv = 1.0f / ltot;
    if (qrow < L) {
      TO* dst = out + (size_t)(base + qrow) * hidden + head * D;
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float v = o[db][r] * inv;
          if (sizeof(TO) == 1) v = static_cast<float>(static_cast<bf16_t>(v)) * out_inv_scale;
          st(dst + db * 32 + (r >> 2) * 8 + hh * 4 + (r & 3), v);
        }
    }
  }
}

constexpr int kWaves = 4;
constexpr int kBQ = 32 * kWaves;
// Record-resident length classes: records of (kClassMax[c-1], kClassMax[c]]
// keys go to a kernel whose LDS holds kClassMax[c] keys and whose waves
// cover that many query rows (32 each), so shorter records fit more
// workgroups per CU and leave fewer waves idle.
constexpr int kClasses = 4;
constexpr int kClassMax[kClasses] = {128, 256, 384, 512};
constexpr int kResidentMax = 512;

// One workgroup: validates cu_seqlens and lists (record, q-block) items for
// the records whose length lies in [lo, hi].
__global__ __launch_bounds__(1024) void seq_plan_kernel(const int* __restrict__ cu, int B, int T, int max_len,
                                                        int lo, int hi, int bq, int4* __restrict__ qblocks,
                                                        int max_q, int* __restrict__ n_qblocks, uint32_t* err) {
  // Malformed (overlapping) cu_seqlens could ask for more items than the
  // buffer holds; writes stop at max_q and the error bit is raised.
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
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

bool resident(ElemType t, int max_len) { return t == ET_BF16 && max_len <= kResidentMax; }

template <typename TO>
void launch_resident(const bf16_t* q, TO* out, const int4* items, int per_class, const int* counts, int n_heads,
                     int hidden, float out_inv_scale, hipStream_t s) {
  const dim3 grid(per_class, n_heads);
  hipLaunchKernelGGL((attn_resident_kernel<TO, 128, 4>), grid, dim3(4 * 64), 0, s, q, out, items, counts,
                     hidden, out_inv_scale);
  hipLaunchKernelGGL((attn_resident_kernel<TO, 256, 8>), grid, dim3(8 * 64), 0, s, q, out,
                     items + per_class, counts + 1, hidden, out_inv_scale);
  hipLaunchKernelGGL((attn_resident_kernel<TO, 384, 12>), grid, dim3(12 * 64), 0, s, q, out,
                     items + 2 * per_class, counts + 2, hidden, out_inv_scale);
  hipLaunchKernelGGL((attn_resident_kernel<TO, 512, 16>), grid, dim3(16 * 64), 0, s, q, out,
                     items + 3 * per_class, counts + 3, hidden, out_inv_scale);
}

}  // namespace

int attn_plan_items(ElemType t, int max_len, int T, int B) {
  // resident: one item per record in each length class;
  // tiled: one item per 128-row q-block
  return resident(t, max_len) ? kClasses * (B + 1) : T / kBQ + B + 1;
}

int attn_plan_counts() { return kClasses; }

void launch_attn_plan(const int* cu_seqlens, int B, int T, int max_len, ElemType t, int4* items, int max_items,
                      int* counts, uint32_t* err, hipStream_t s) {
  if (resident(t, max_len)) {
    const int per = max_items / kClasses;
    for (int c = 0; c < kClasses; ++c) {
      const int lo = c == 0 ? 1 : kClassMax[c - 1] + 1;
      hipLaunchKernelGGL(seq_plan_kernel, dim3(1), dim3(1024), 0, s, cu_seqlens, B, T, max_len, lo, kClassMax[c],
                         1 << 30, items + c * per, per, counts + c, err);
    }
  } else {
    hipLaunchKernelGGL(seq_plan_kernel, dim3(1), dim3(1024), 0, s, cu_seqlens, B, T, max_len, 0, max_len, kBQ,
                       items, max_items, counts, err);
  }
}

void launch_attention(const void* qkv, void* out, const int4* items, int max_items, const int* counts,
                      int max_len, int n_heads, int hidden, ElemType t, ElemType out_t, float out_inv_scale,
                      hipStream_t s) {
  if (max_items <= 0) return;
  if (resident(t, max_len)) {
    const int per = max_items / kClasses;
    if (out_t == ET_FP8)
      launch_resident(static_cast<const bf16_t*>(qkv), (fp8_t*)out, items, per, counts, n_heads, hidden,
                      out_inv_scale, s);
    else
      launch_resident(static_cast<const bf16_t*>(qkv), (bf16_t*)out, items, per, counts, n_heads, hidden,
                      out_inv_scale, s);
    return;
  }
  dim3 grid(max_items, n_heads);
  if (t == ET_F32) {
    hipLaunchKernelGGL((attn_kernel<float, float, kWaves>), grid, dim3(kWaves * 64), 0, s, (const float*)qkv,
                       (float*)out, items, counts, hidden, out_inv_scale);
  } else if (out_t == ET_FP8) {
    hipLaunchKernelGGL((attn_kernel<bf16_t, fp8_t, kWaves>), grid, dim3(kWaves * 64), 0, s, (const bf16_t*)qkv,
                       (fp8_t*)out, items, counts, hidden, out_inv_scale);
  } else {
    hipLaunchKernelGGL((attn_kernel<bf16_t, bf16_t, kWaves>), grid, dim3(kWaves * 64), 0, s, (const bf16_t*)qkv,
                       (bf16_t*)out, items, counts, hidden, out_inv_scale);
  }
}

}  // namespace anon
