// Dense GEMMs of the encoder on CDNA4 matrix cores, with fused epilogues.
//
// C[M,N] = A[M,K] * W[N,K]^T, A = packed token activations (no padding), W =
// a weight matrix stored transposed so that both operands are K-contiguous.
// One workgroup owns a BM x BN output tile; its waves form a WGM x WGN grid
// and each wave accumulates (BM/WGM) x (BN/WGN) with 32x32 MFMA tiles:
//   fp32: v_mfma_f32_32x32x2_f32      (K step 2)
//   bf16: v_mfma_f32_32x32x16_bf16    (K step 16)
//   fp8 : v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 operands (K step 64)
// Two main loops: BF16/FP8 operands stream global -> LDS directly through a
// ring of ST K tiles (global_load_lds_dwordx4, XOR-swizzled rows); FP32
// operands go through registers into double-buffered, padded LDS.  In both
// the MFMA operands of k-step s+1 are read from LDS while those of step s
// are multiplied.
//
// The K loop always runs in increasing k with one MFMA shape per precision,
// so each output element's sum is formed in the same order whatever the tile
// shape or the row's position in the batch (batch invariance; tile
// configurations are interchangeable bit for bit).
//
// Epilogues: bias (+ exact scaling of the Q columns by 1/sqrt(d)); bias + GELU;
// bias + residual added in FP32 and rounded once to the output type.
#include <algorithm>

#include "kernels.hpp"

namespace anon {
namespace {

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  typedef float frag;
  static constexpr int KI = 2, KPL = 1;
  __device__ static floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<bf16_t> {
  typedef bf16x8 frag;
  static constexpr int KI = 16, KPL = 8;
  __device__ static floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<fp8_t> {
  typedef intx8 frag;
  static constexpr int KI = 64, KPL = 32;
  // operand formats 0/0 = E4M3 x E4M3; block scales 127 = 2^0 (unscaled)
  __device__ static floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};

__device__ __forceinline__ float ld(const float* p) { return *p; }
__device__ __forceinline__ float ld(const bf16_t* p) { return static_cast<float>(*p); }
__device__ __forceinline__ void st(float* p, float v) { *p = v; }
__device__ __forceinline__ void st(bf16_t* p, float v) { *p = static_cast<bf16_t>(v); }
__device__ __forceinline__ void st(fp8_t* p, float v) { p->v = f32_to_e4m3(v); }

// GELU(v) = v/2 (1 + erf(v / sqrt 2)) with erf from Abramowitz & Stegun
// formula 7.1.26 (rational approximation, |error| <= 1.5e-7): far below the
// bf16 output rounding and the FP32 path's 1e-4 logit tolerance, and a third
// of the instructions of a full-precision erff in an epilogue that runs
// once per output element.
__device__ __forceinline__ float gelu_erf(float v) {
  // Phi(v) = 1 - q for v >= 0 and q for v < 0, with q = P(t) exp(-v^2/2) / 2,
  // t = 1 / (1 + p |v| / sqrt 2); the 1/2 and 1/sqrt 2 are folded into the
  // constants, and exp(-v^2/2) = exp2(-(v sqrt(log2(e)/2))^2)
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, fabsf(v), 1.0f));
  const float P = ((((0.5f * 1.061405429f * t - 0.5f * 1.453152027f) * t + 0.5f * 1.421413741f) * t -
                    0.5f * 0.284496736f) * t + 0.5f * 0.254829592f) * t;
  const float sv = v * 0.84932180028801904f;
  const float r = v * (P * __builtin_amdgcn_exp2f(-(sv * sv)));
  // v - r for v >= 0 and r for v < 0: since q <= 1/2, r = v q lies between
  // 0 and v/2, so the wanted value is always the larger of the two
  return fmaxf(v - r, r);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so that the tiles sharing an A row-block (and the
// weight panel) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int X = 8;
  const int per = nb / X, rem = nb % X;
  const int x = bid % X, loc = bid / X;
  return x * per + min(x, rem) + loc;
}

// Linear tile index -> (row block, column block), in groups of `gm` row
// blocks walked column by column: the tiles in flight on one XCD then share
// a few A row blocks and a few weight column panels, a working set that fits
// its L2, instead of cycling through the whole weight matrix per row block.
__device__ __forceinline__ void group_tile(int t, int ntm, int ntn, int gm, int& mb, int& nb) {
  const int per_group = gm * ntn;
  const int g = t / per_group, r = t - g * per_group;
  const int m0 = g * gm, gsz = min(ntm - m0, gm);
  mb = m0 + r % gsz;
  nb = r / gsz;
}

struct DevParams {
  const void* A;
  const void* W;
  const float* bias;
  const void* resid;
  void* C;
  int M, N, K;
  float qscale;
  int qcols;
  float acc_scale;
  float out_inv_scale;
  int group_m;
  int ldc;            // output row stride (elements)
  const int* pos;     // EPI_ROPE: position of each row within its record
  const float* rope;  // EPI_ROPE: [max_pos][64] cos (first 32) and sin (last 32)
  int rope_cols;      // EPI_ROPE: columns below this are rotated
  const int* m_dev;   // non-null: rows to compute (device), M is the grid's capacity
};

// The MFMAs take the weight fragment as their first operand, so each
// accumulator holds a 32x32 block of C^T: lane l, register r holds row
// (l & 31) and column (r/4)*8 + (l/32)*4 + r%4 of the block -- four
// consecutive columns of one row per register quad.
//
// Epilogue: once the K loop is done, the operand LDS is reused.  Each wave
// forms its outputs -- bias, Q scaling, GELU or the residual (copied first
// into the LDS slots its outputs take, added in FP32, rounded once) -- and
// parks them in its own LDS region in the output type, then writes the
// region back with 16-byte row-contiguous stores.  Loads come before stores wherever possible: on
// this architecture loads and stores share one counter, so a load issued
// after a store waits for the store to be acknowledged.  The region holds
// whole 32-row strips (see Staging::NS).  Rows are unpadded, with 16-byte chunks
// XOR-permuted by the row (chunk c of row r in slot c ^ (r mod 16)) so that
// the 32 rows a register quad spans land on distinct bank groups.
template <typename TO, int EPI, int TM, int TN, int NW, int SMEM>
struct Staging {
  // output columns of a wave: the gated epilogue writes one of each pair
  // of 32-column sub-blocks
  static constexpr int OTN = EPI == EPI_GEGLU ? TN / 2 : TN;
  static constexpr int ROWB = OTN * 32 * (int)sizeof(TO);       // bytes per staged row
  static constexpr int CPR = ROWB / 16;                          // 16-byte chunks per row
  static constexpr int SWZ = (CPR < 16 ? CPR : 16) - 1;
  static constexpr int STRIP = 32 * ROWB;                        // one 32-row strip of one wave
  static constexpr int FIT = SMEM / (NW * STRIP) < TM ? SMEM / (NW * STRIP) : TM;
  // strips per pass: the residual epilogue loads, so it stages as much as
  // fits before its first store; the others load nothing after the bias and
  // go strip by strip, one strip's stores draining under the next's math
  static constexpr int NS = EPI == EPI_RESID ? FIT : 1;
  static_assert(NS >= 1 && CPR >= 4 && (CPR & (CPR - 1)) == 0, "epilogue staging does not fit");
  static_assert((NS * 32 * CPR) % 64 == 0, "write-back covers whole waves");
};

template <typename T>
__device__ __forceinline__ void ld4(const T* p, float (&v)[4]);
template <>
__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
  const floatx4 x = *(const floatx4*)p;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = x[e];
}
template <>
__device__ __forceinline__ void ld4(const bf16_t* p, float (&v)[4]) {
  const bf16x4 x = *(const bf16x4*)p;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = static_cast<float>(x[e]);
}

__device__ __forceinline__ void st4(float* p, const float (&v)[4]) { *(floatx4*)p = floatx4{v[0], v[1], v[2], v[3]}; }
__device__ __forceinline__ void st4(bf16_t* p, const float (&v)[4]) {
  *(bf16x4*)p = bf16x4{static_cast<bf16_t>(v[0]), static_cast<bf16_t>(v[1]), static_cast<bf16_t>(v[2]),
                       static_cast<bf16_t>(v[3])};
}
__device__ __forceinline__ void st4(fp8_t* p, const float (&v)[4]) {
  float c[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) c[e] = fminf(fmaxf(v[e], -448.0f), 448.0f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
  *(int*)p = w;
}

// Applies the epilogue to a wave's (TM*32) x (TN*32) accumulator block whose
// top-left output element is (wrow0, wcol0).
template <typename TO, typename TR, int EPI, int TM, int TN, int NW, int SMEM>
__device__ __forceinline__ void epilogue(const DevParams& p, floatx16 (&acc)[TM][TN], char* smem, int wave, int lane,
                                         int wrow0, int wcol0) {
  typedef Staging<TO, EPI, TM, TN, NW, SMEM> SG;
  constexpr int ROWB = SG::ROWB, CPR = SG::CPR, SWZ = SG::SWZ, NS = SG::NS;
  const int M = live_rows(p.M, p.m_dev), N = p.N;
  constexpr bool PAIRED = EPI == EPI_ROPE || EPI == EPI_GEGLU;
  static_assert(!PAIRED || TN % 2 == 0, "paired epilogues need whole 64-column blocks per wave");
  static_assert(EPI != EPI_GEGLU || sizeof(TO) >= 2, "the gated epilogue writes bf16 or fp32");
  // where this wave's outputs start in a row of C
  const int ocol0 = EPI == EPI_GEGLU ? wcol0 / 2 : wcol0;
  char* stg = smem + wave * NS * SG::STRIP;
  const int lrow = lane & 31, lq = (lane >> 5) * 4;
  // bias of the lane's columns (loaded before any store)
  floatx4 bias[TN][4];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) bias[j][q] = *(const floatx4*)(p.bias + wcol0 + j * 32 + q * 8 + lq);
#pragma unroll
  for (int i0 = 0; i0 < TM; i0 += NS) {
    if constexpr (EPI == EPI_RESID) {
      // 0. the residual of strips [i0, i0 + NS) straight into the staging
      // slots its outputs take (residual and output have one element size):
      // 16-byte row-contiguous global -> LDS copies, lane l of a copy taking
      // slot l % CPR of staged row (copy rows) + l / CPR, i.e. the chunk
      // that the row's XOR permutation puts there.  Read per lane in the
      // accumulator layout instead, every load would touch 32 rows for 16
      // bytes of each.
      static_assert(sizeof(TR) == sizeof(TO), "the residual is staged in the output's layout");
      static_assert(ROWB <= 1024 && 1024 % ROWB == 0, "whole staged rows per copy instruction");
      constexpr int RPC = 1024 / ROWB;  // staged rows per copy instruction
      const int nss = min(TM - i0, NS);  // strips of this pass
      const int crow = lane / CPR, cslot = lane % CPR;
      // a uniform base row (rows past M re-read row M-1, which the clamped
      // base keeps at or below every lane's row) and 32-bit lane offsets
      const int brow = min(wrow0 + i0 * 32, M - 1);
      const char* rbase = (const char*)p.resid + ((size_t)brow * N + wcol0) * sizeof(TR);
#pragma unroll
      for (int t = 0; t < NS * 32 / RPC; ++t) {
        if (t * RPC >= nss * 32) break;
        const int srow = t * RPC + crow;
        const int grow = min(wrow0 + (i0 + (srow >> 5)) * 32 + (srow & 31), M - 1);
        const uint32_t off = (uint32_t)((grow - brow) * N * (int)sizeof(TR) + (cslot ^ (srow & SWZ)) * 16);
        dma16(rbase + off, stg + t * 1024);
      }
      wait_vmcnt<0>();
    }
    // 1. outputs of strips [i0, i0 + NS) into LDS
#pragma unroll
    for (int is = 0; is < NS && i0 + is < TM; ++is) {
      const int i = i0 + is;
      const int srow = is * 32 + lrow;  // staged row
      const int grow = min(wrow0 + i * 32 + lrow, M - 1);
      if constexpr (PAIRED) {
        // sub-blocks j and j+1 hold the two members of each pair: columns
        // c and c + 32 of a 64-column head block (RoPE), or the input and
        // the gate half of the gated MLP (weights interleaved in 32-column
        // blocks)
        int prow = 0;
        if constexpr (EPI == EPI_ROPE) prow = p.pos[grow];
#pragma unroll
        for (int j = 0; j < TN; j += 2) {
          const bool rot = EPI == EPI_ROPE && wcol0 + j * 32 < p.rope_cols;
          const bool qs = EPI == EPI_ROPE && wcol0 + j * 32 < p.qcols;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int d0 = q * 8 + lq;  // index within the 32-column sub-block
            float a[4], b[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              a[e] = acc[i][j][q * 4 + e] * p.acc_scale + bias[j][q][e];
              b[e] = acc[i][j + 1][q * 4 + e] * p.acc_scale + bias[j + 1][q][e];
            }
            if constexpr (EPI == EPI_ROPE) {
              if (rot) {
                const floatx4 cs = *(const floatx4*)(p.rope + (size_t)prow * 64 + d0);
                const floatx4 sn = *(const floatx4*)(p.rope + (size_t)prow * 64 + 32 + d0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const float x1 = a[e], x2 = b[e];
                  a[e] = x1 * cs[e] - x2 * sn[e];
                  b[e] = x2 * cs[e] + x1 * sn[e];
                }
              }
              if (qs) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  a[e] *= p.qscale;
                  b[e] *= p.qscale;
                }
              }
              const int ba = (j * 32 + d0) * (int)sizeof(TO), bb = ((j + 1) * 32 + d0) * (int)sizeof(TO);
              st4((TO*)(stg + srow * ROWB + (((ba >> 4) ^ (srow & SWZ)) * 16) + (ba & 15)), a);
              st4((TO*)(stg + srow * ROWB + (((bb >> 4) ^ (srow & SWZ)) * 16) + (bb & 15)), b);
            } else {
              float y[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) y[e] = gelu_erf(a[e]) * b[e];
              const int by = ((j / 2) * 32 + d0) * (int)sizeof(TO);
              st4((TO*)(stg + srow * ROWB + (((by >> 4) ^ (srow & SWZ)) * 16) + (by & 15)), y);
            }
          }
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        // the Q columns are whole 32-column blocks (qcols is a multiple of 64)
        const bool qs = EPI == EPI_BIAS && wcol0 + j * 32 < p.qcols;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int cl = j * 32 + q * 8 + lq;  // column within the wave's block
          const int byte = cl * (int)sizeof(TO);
          const int chunk = (byte >> 4) ^ (srow & SWZ);
          char* slot = stg + srow * ROWB + chunk * 16 + (byte & 15);
          float rv[4] = {0.f, 0.f, 0.f, 0.f};
          if constexpr (EPI == EPI_RESID) ld4((const TR*)slot, rv);  // staged above
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float x = acc[i][j][q * 4 + e] * p.acc_scale + bias[j][q][e];
            if (EPI == EPI_BIAS) {
              if (qs) x *= p.qscale;
            } else if (EPI == EPI_GELU) {
              x = gelu_erf(x);
              // FP8 output: the activation is a bf16 value first (as in the
              // BF16 path), then scaled and rounded to E4M3
              if (sizeof(TO) == 1) x = static_cast<float>(static_cast<bf16_t>(x)) * p.out_inv_scale;
            } else {
              x += rv[e];
            }
            v[e] = x;
          }
          st4((TO*)slot, v);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // 2. the strips back to memory, 16 bytes per lane, row-contiguous
    constexpr int NCH = NS * 32 * CPR;
#pragma unroll
    for (int c0 = 0; c0 < NCH; c0 += 64) {
      const int c = c0 + lane;  // NCH is a multiple of 64
      const int srow = c / CPR, cc = c % CPR;
      const int i = i0 + srow / 32;  // past TM only in a last, partial pass
      const int grow = wrow0 + i * 32 + (srow & 31);
      const intx4 v = *(const intx4*)(stg + srow * ROWB + ((cc ^ (srow & SWZ)) * 16));
      // (single-use streams: the next kernel reads them from memory)
      if (i < TM && grow < M)
        __builtin_nontemporal_store(v, (intx4*)((char*)p.C + ((size_t)grow * p.ldc + ocol0) * sizeof(TO) + cc * 16));
    }
    if (i0 + NS < TM) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }
}

// Register-staged kernel (FP32 operands): the next K tile is fetched into
// registers while the current one is multiplied from double-buffered,
// row-padded LDS (16 bytes of padding per row keeps the 16-byte fragment
// reads of 16 lanes on distinct banks).
template <typename TI, typename TO, typename TR, int EPI, int BM, int BN, int BK, int WGM, int WGN, int OCC>
__global__ __launch_bounds__(WGM* WGN * 64, OCC) void gemm_kernel(DevParams p) {
  typedef Mfma<TI> MF;
  typedef typename MF::frag frag;
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TM = WTM / 32, TN = WTN / 32;
  constexpr int EPC = 16 / (int)sizeof(TI);  // elements per 16-byte chunk
  constexpr int CPR = BK / EPC;              // chunks per tile row
  constexpr int LDK = BK + EPC;              // padded LDS row (16 bytes)
  constexpr int A_CH = BM * CPR / NT, B_CH = BN * CPR / NT;
  constexpr int NKS = BK / MF::KI;
  static_assert((BM * CPR) % NT == 0 && (BN * CPR) % NT == 0, "tile/threads mismatch");
  static_assert(TM >= 1 && TN >= 1 && BK % MF::KI == 0, "bad tile");
  constexpr int OPND_BYTES = 2 * (BM + BN) * LDK * (int)sizeof(TI);
  __shared__ __align__(16) char smem[OPND_BYTES];
  TI(*As)[BM * LDK] = reinterpret_cast<TI(*)[BM * LDK]>(smem);
  TI(*Bs)[BN * LDK] = reinterpret_cast<TI(*)[BN * LDK]>(smem + 2 * BM * LDK * sizeof(TI));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int N = p.N, K = p.K;
  // the tiles of the rows to compute; with a device row count the grid may
  // hold more workgroups, which leave at once, and the live tiles are spread
  // over the XCDs as in a launch of exactly their number
  const int M = live_rows(p.M, p.m_dev);
  const int ntn = N / BN;
  const int ntm = (M + BM - 1) / BM;
  if ((int)blockIdx.x >= ntm * ntn) return;
  int mb, nb;
  group_tile(xcd_remap(blockIdx.x, ntm * ntn), ntm, ntn, p.group_m, mb, nb);
  const int m0 = mb * BM, n0 = nb * BN;

  const TI* __restrict__ A = (const TI*)p.A;
  const TI* __restrict__ W = (const TI*)p.W;

  intx4 ra[A_CH], rb[B_CH];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
      const int c = tid + i * NT, r = c / CPR, cc = c % CPR;
      // rows past M (last tile only) re-read row M-1: their results are
      // never stored, and the load needs no branch
      const int gm = min(m0 + r, M - 1);
      ra[i] = *(const intx4*)(A + (size_t)gm * K + k0 + cc * EPC);
    }
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
      const int c = tid + i * NT, r = c / CPR, cc = c % CPR;
      rb[i] = *(const intx4*)(W + (size_t)(n0 + r) * K + k0 + cc * EPC);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
      const int c = tid + i * NT, r = c / CPR, cc = c % CPR;
      *(intx4*)&As[buf][r * LDK + cc * EPC] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
      const int c = tid + i * NT, r = c / CPR, cc = c % CPR;
      *(intx4*)&Bs[buf][r * LDK + cc * EPC] = rb[i];
    }
  };

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = K / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int arow = wm * WTM + (lane & 31), brow = wn * WTN + (lane & 31);
  const int kofs = (lane >> 5) * MF::KPL;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * BK);
    const TI* as = As[buf];
    const TI* bs = Bs[buf];
    frag a[2][TM], b[2][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a[0][i] = *(const frag*)&as[(arow + i * 32) * LDK + kofs];
#pragma unroll
    for (int j = 0; j < TN; ++j) b[0][j] = *(const frag*)&bs[(brow + j * 32) * LDK + kofs];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < NKS) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
          a[cur ^ 1][i] = *(const frag*)&as[(arow + i * 32) * LDK + (ks + 1) * MF::KI + kofs];
#pragma unroll
        for (int j = 0; j < TN; ++j)
          b[cur ^ 1][j] = *(const frag*)&bs[(brow + j * 32) * LDK + (ks + 1) * MF::KI + kofs];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(b[cur][j], a[cur][i], acc[i][j]);
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }
  epilogue<TO, TR, EPI, TM, TN, WGM * WGN, OPND_BYTES>(p, acc, smem, wave, lane, m0 + wm * WTM, n0 + wn * WTN);
}

// LDS-ring kernel (BF16 / FP8 operands).  Each K tile travels from global
// memory straight into LDS (global_load_lds_dwordx4: no register staging),
// ST tiles deep, so the loads of tile k+ST-1 are in flight while tile k is
// multiplied.  One barrier per K tile: after it, every wave's copy of tile k
// has landed and every wave has finished reading tile k-1, whose slot then
// takes tile k+ST-1.
//
// LDS layout: rows of BK elements, unpadded, with the 16-byte chunks of a
// row XOR-permuted by a function of the row (chunk c of row r sits in slot
// c ^ swz(r)): a 16-lane group reading the same logical chunk of 16
// consecutive rows then touches 16 distinct 16-byte bank groups, and one
// wave's load instruction fills 1024 contiguous bytes.
template <int CPR>
__device__ __forceinline__ int lds_swz(int r) {
  static_assert(CPR == 4 || CPR == 8, "rows of 64 or 128 bytes");
  return CPR == 8 ? (r >> 1) & 7 : (r >> 2) & 3;
}

// Instruction order of one k-step (a scheduling region): the next k-step's
// fragment reads go out two per MFMA from the first MFMA on, so their
// latency hides behind the rest of the step's MFMA chain; then the ring
// refill loads (last k-step of a tile), two per MFMA; then the other MFMAs.
template <int NMF, int NRD, int NVM>
__device__ __forceinline__ void sched_step() {
  constexpr int RG = (NRD + 1) / 2, VG = (NVM + 1) / 2;
#pragma unroll
  for (int r = 0; r < NRD / 2; ++r) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // DS read
  }
  if constexpr (NRD % 2) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
#pragma unroll
  for (int v = 0; v < NVM / 2; ++v) {
    if (RG + v < NMF) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x010, 2, 0);  // VMEM
  }
  if constexpr (NVM % 2) {
    if (RG + VG - 1 < NMF) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
  }
  if constexpr (NMF > RG + VG) __builtin_amdgcn_sched_group_barrier(0x008, NMF - RG - VG, 0);
}

template <typename TI, typename TO, typename TR, int EPI, int BM, int BN, int BK, int WGM, int WGN, int ST,
          int OCC>
__global__ __launch_bounds__(WGM* WGN * 64, OCC) void gemm_dma_kernel(DevParams p) {
  typedef Mfma<TI> MF;
  typedef typename MF::frag frag;
  constexpr int NW = WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TM = WTM / 32, TN = WTN / 32;
  constexpr int EPC = 16 / (int)sizeof(TI);    // elements per 16-byte chunk
  constexpr int CPR = BK / EPC;                // chunks per row
  constexpr int ROWB = BK * (int)sizeof(TI);   // bytes per row
  constexpr int RPI = 64 / CPR;                // rows per wave load instruction
  constexpr int A_INS = BM / RPI / NW, B_INS = BN / RPI / NW;
  constexpr int LPT = A_INS + B_INS;           // load instructions per wave per K tile
  constexpr int A_BYTES = BM * ROWB, STAGE = (BM + BN) * ROWB;
  constexpr int NKS = BK / MF::KI;             // MFMA k-steps per K tile
  constexpr int NCH = MF::KPL * (int)sizeof(TI) / 16;  // chunks per lane fragment
  constexpr int CPS = MF::KI / EPC;            // chunks per k-step
  static_assert(BM % (RPI * NW) == 0 && BN % (RPI * NW) == 0, "tile/waves mismatch");
  static_assert(TM >= 1 && TN >= 1 && BK % MF::KI == 0 && ST >= 2, "bad tile");
  static_assert((ST - 1) * LPT < 64, "vmcnt range");
  constexpr int SMEM = ST * STAGE;
  static_assert(SMEM <= 160 * 1024, "LDS ring exceeds the CU's 160 KB");
  __shared__ __align__(1024) char smem[SMEM];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int N = p.N, K = p.K;
  // the tiles of the rows to compute; with a device row count the grid may
  // hold more workgroups, which leave at once, and the live tiles are spread
  // over the XCDs as in a launch of exactly their number
  const int M = live_rows(p.M, p.m_dev);
  const int ntn = N / BN;
  const int ntm = (M + BM - 1) / BM;
  if ((int)blockIdx.x >= ntm * ntn) return;
  int mb, nb;
  group_tile(xcd_remap(blockIdx.x, ntm * ntn), ntm, ntn, p.group_m, mb, nb);
  const int m0 = mb * BM, n0 = nb * BN;

  // this lane's source of each load instruction, as a byte offset from the
  // tile's first row at k = 0 (uniform bases stay in scalar registers; rows
  // past M, in the last row block only, re-read row M-1: never stored, no
  // branch)
  const char* const abase = (const char*)p.A + (size_t)m0 * K * sizeof(TI);
  const char* const bbase = (const char*)p.W + (size_t)n0 * K * sizeof(TI);
  uint32_t ga[A_INS], gb[B_INS];
  {
    const int rl = lane / CPR, slot = lane % CPR;
#pragma unroll
    for (int i = 0; i < A_INS; ++i) {
      const int r = (wave * A_INS + i) * RPI + rl;
      ga[i] = (uint32_t)((min(m0 + r, M - 1) - m0) * K + (slot ^ lds_swz<CPR>(r)) * EPC) * (uint32_t)sizeof(TI);
    }
#pragma unroll
    for (int i = 0; i < B_INS; ++i) {
      const int r = (wave * B_INS + i) * RPI + rl;
      gb[i] = (uint32_t)(r * K + (slot ^ lds_swz<CPR>(r)) * EPC) * (uint32_t)sizeof(TI);
    }
  }
  auto issue = [&](int kt, int stage) {
    char* sa = smem + stage * STAGE + wave * A_INS * 1024;
    char* sb = smem + stage * STAGE + A_BYTES + wave * B_INS * 1024;
    const char* ak = abase + (size_t)kt * BK * sizeof(TI);
    const char* bk = bbase + (size_t)kt * BK * sizeof(TI);
#pragma unroll
    for (int i = 0; i < A_INS; ++i) dma16(ak + ga[i], sa + i * 1024);
#pragma unroll
    for (int i = 0; i < B_INS; ++i) dma16(bk + gb[i], sb + i * 1024);
  };

  // fragment addresses: row (lane & 31) of each 32-row sub-tile; the swizzle
  // is the same for rows 32 apart, so one slot offset per (k-step, chunk)
  const int ra = wm * WTM + (lane & 31), rb = wn * WTN + (lane & 31);
  int aoff[NKS][NCH], boff[NKS][NCH];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int kc = ks * CPS + (lane >> 5) * NCH + q;
      aoff[ks][q] = ra * ROWB + (kc ^ lds_swz<CPR>(ra)) * 16;
      boff[ks][q] = A_BYTES + rb * ROWB + (kc ^ lds_swz<CPR>(rb)) * 16;
    }
  auto rdfrag = [&](const char* base, const int (&off)[NCH], int sub) {
    frag f;
    if constexpr (NCH == 1) {
      f = *(const frag*)(base + off[0] + sub * 32 * ROWB);
    } else {
      const intx4 lo = *(const intx4*)(base + off[0] + sub * 32 * ROWB);
      const intx4 hi = *(const intx4*)(base + off[1] + sub * 32 * ROWB);
      f = frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
    return f;
  };

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = K / BK;
  // The ring always holds ST tiles in flight or resident; with more than two
  // stages, refills past the last tile re-read tile KT-1 (valid memory, never
  // multiplied), so the wait counts stay constants.
#pragma unroll
  for (int s = 0; s < ST; ++s) issue(min(s, KT - 1), s);
  wait_vmcnt<(ST - 1) * LPT>();
  __builtin_amdgcn_s_barrier();

  // Fragments are double-buffered across k-steps, also across tiles: the
  // buffer of a k-step is the parity of its global k-step index, a
  // compile-time value once the tile loop is unrolled by two.
  frag fa[2][TM], fb[2][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) fa[0][i] = rdfrag(smem, aoff[0], i);
#pragma unroll
  for (int j = 0; j < TN; ++j) fb[0][j] = rdfrag(smem, boff[0], j);
  int stage = 0;
  // One K tile.  During its last k-step the next tile is made ready: wait for
  // it, barrier (every wave has then also finished reading this tile, whose
  // slot takes tile kt+ST), and read its first fragments while this tile's
  // last MFMAs run.
  auto tile_body = [&](int kt, auto tpar) {
    constexpr int TP = decltype(tpar)::value;
    const char* base = smem + stage * STAGE;
    const int nstage = stage + 1 == ST ? 0 : stage + 1;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int cur = (TP * NKS + ks) & 1;
      if (ks + 1 < NKS) {
#pragma unroll
        for (int i = 0; i < TM; ++i) fa[cur ^ 1][i] = rdfrag(base, aoff[ks + 1 < NKS ? ks + 1 : 0], i);
#pragma unroll
        for (int j = 0; j < TN; ++j) fb[cur ^ 1][j] = rdfrag(base, boff[ks + 1 < NKS ? ks + 1 : 0], j);
      } else {
        // this wave's reads of the tile have returned before anyone may
        // overwrite it; tile kt+1 has landed for this wave.  (No instruction
        // crosses this point: the previous k-step's MFMAs stay ahead of the
        // wait, covering the latency of the reads it waits for.)
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) (vmcnt, expcnt at maxima)
        wait_vmcnt<(ST - 2) * LPT>();
        __builtin_amdgcn_s_barrier();
        // past the last tile: a two-stage ring waits for every load, so the
        // refill is left out (nothing to land before the epilogue); deeper
        // rings re-read tile KT-1 to keep their wait counts constant
        if (ST > 2 || kt + ST < KT) issue(min(kt + ST, KT - 1), stage);
        const char* nbase = smem + nstage * STAGE;
#pragma unroll
        for (int i = 0; i < TM; ++i) fa[cur ^ 1][i] = rdfrag(nbase, aoff[0], i);
#pragma unroll
        for (int j = 0; j < TN; ++j) fb[cur ^ 1][j] = rdfrag(nbase, boff[0], j);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(fb[cur][j], fa[cur][i], acc[i][j]);
      // (with two workgroups per CU the hardware interleaves them better)
      if constexpr (OCC == 1) {
        if (ks + 1 < NKS) sched_step<TM * TN, (TM + TN) * NCH, 0>();
        else sched_step<TM * TN, (TM + TN) * NCH, LPT>();
      }
    }
    stage = nstage;
  };
  for (int kt = 0; kt < KT; kt += 2) {
    tile_body(kt, std::integral_constant<int, 0>());
    if (kt + 1 < KT) tile_body(kt + 1, std::integral_constant<int, 1>());
  }
  // the refills issued by the last tiles must land before the staging below
  // reuses the ring
  wait_vmcnt<0>();
  // and every wave must have finished reading it
  __syncthreads();
  epilogue<TO, TR, EPI, TM, TN, NW, SMEM>(p, acc, smem, wave, lane, m0 + wm * WTM, n0 + wn * WTN);
}

struct Cfg {
  int bm, bn, bk, wgm, wgn, st, occ;
  const char* name;
};

// Whether a tile serves an epilogue: the paired epilogues need an even
// number of 32-column sub-blocks per wave, and one 32-row output strip per
// wave must fit the kernel's LDS (mirrors Staging).
constexpr bool staging_fits(int bm, int bn, int bk, int wgm, int wgn, int st, int in_bytes, int out_bytes, int epi) {
  const int tn = bn / wgn / 32;
  if ((epi == EPI_ROPE || epi == EPI_GEGLU) && tn % 2 != 0) return false;
  const int smem = st == 0 ? 2 * (bm + bn) * (bk + 16 / in_bytes) * in_bytes : st * (bm + bn) * bk * in_bytes;
  const int otn = epi == EPI_GEGLU ? tn / 2 : tn;
  return smem >= wgm * wgn * 32 * otn * 32 * out_bytes;
}

// Tile configurations per input type; index = GemmParams::config.
// Columns: BM, BN, BK, wave grid WGM x WGN, LDS ring stages (0: the
// register-staged kernel), workgroups per CU the registers are sized for.
#define ANON_BF16_CFGS(X)                                      \
  X(0, 256, 256, 64, 4, 2, 0, 2, "bf16_256x256x64_w4x2")       \
  X(1, 256, 128, 32, 4, 2, 0, 2, "bf16_256x128x32_w4x2")       \
  X(2, 128, 256, 32, 2, 4, 0, 2, "bf16_128x256x32_w2x4")       \
  X(3, 256, 256, 32, 4, 2, 3, 1, "bf16_256x256x32_w4x2_s3")    \
  X(4, 256, 128, 64, 4, 2, 3, 1, "bf16_256x128x64_w4x2_s3")    \
  X(5, 128, 256, 64, 2, 4, 3, 1, "bf16_128x256x64_w2x4_s3")    \
  X(6, 256, 128, 32, 4, 2, 3, 2, "bf16_256x128x32_w4x2_s3")    \
  X(7, 128, 256, 32, 2, 4, 3, 2, "bf16_128x256x32_w2x4_s3")    \
  X(8, 256, 256, 64, 4, 2, 2, 1, "bf16_256x256x64_w4x2_s2")    \
  X(9, 256, 256, 32, 4, 2, 4, 1, "bf16_256x256x32_w4x2_s4")    \
  X(10, 256, 128, 32, 4, 2, 4, 1, "bf16_256x128x32_w4x2_s4")    \
  X(11, 256, 256, 64, 2, 4, 2, 1, "bf16_256x256x64_w2x4_s2")
#define ANON_F32_CFGS(X)                                 \
  X(0, 128, 128, 32, 2, 2, 0, 2, "f32_128x128x32_w2x2") \
  X(1, 64, 64, 32, 2, 2, 0, 2, "f32_64x64x32_w2x2")     \
  X(2, 128, 128, 16, 2, 2, 0, 2, "f32_128x128x16_w2x2") \
  X(3, 256, 128, 16, 2, 2, 0, 1, "f32_256x128x16_w2x2")
#define ANON_FP8_CFGS(X)                                    \
  X(0, 256, 256, 64, 4, 2, 0, 2, "fp8_256x256x64_w4x2")     \
  X(1, 256, 256, 64, 4, 2, 3, 1, "fp8_256x256x64_w4x2_s3")  \
  X(2, 256, 256, 128, 4, 2, 2, 1, "fp8_256x256x128_w4x2_s2") \
  X(3, 256, 128, 128, 4, 2, 3, 1, "fp8_256x128x128_w4x2_s3") \
  X(4, 256, 128, 64, 4, 2, 3, 2, "fp8_256x128x64_w4x2_s3")  \
  X(5, 128, 256, 64, 2, 4, 3, 2, "fp8_128x256x64_w2x4_s3")  \
  X(6, 256, 256, 64, 4, 2, 4, 1, "fp8_256x256x64_w4x2_s4")  \
  X(7, 256, 256, 128, 2, 4, 2, 1, "fp8_256x256x128_w2x4_s2")

#define ANON_CFG_ROW(i, bm, bn, bk, wgm, wgn, st, occ, name) {bm, bn, bk, wgm, wgn, st, occ, name},
const Cfg kCfgBF16[] = {ANON_BF16_CFGS(ANON_CFG_ROW)};
const Cfg kCfgF32[] = {ANON_F32_CFGS(ANON_CFG_ROW)};
const Cfg kCfgFP8[] = {ANON_FP8_CFGS(ANON_CFG_ROW)};

const Cfg* cfgs(ElemType t, int* n) {
  if (t == ET_BF16) {
    *n = (int)(sizeof(kCfgBF16) / sizeof(Cfg));
    return kCfgBF16;
  }
  if (t == ET_F32) {
    *n = (int)(sizeof(kCfgF32) / sizeof(Cfg));
    return kCfgF32;
  }
  *n = (int)(sizeof(kCfgFP8) / sizeof(Cfg));
  return kCfgFP8;
}

template <typename TI, typename TO, typename TR, int EPI, int BM, int BN, int BK, int WGM, int WGN, int ST, int OCC>
bool run(const GemmParams& g, hipStream_t s) {
  if constexpr (!staging_fits(BM, BN, BK, WGM, WGN, ST, (int)sizeof(TI), (int)sizeof(TO), EPI)) {
    return false;  // no pairs in a wave's columns, or the output strips do not fit the LDS
  } else {
  // tile order: by default, groups of 8 row blocks when a row block spans 8
  // or more column blocks (its weight panels would otherwise cycle through
  // the XCD's L2 once per row block), else plain row-major order
  const int gm = g.group_m > 0 ? g.group_m : (g.N / BN >= 8 ? 8 : 1);
  DevParams p{g.A, g.W, g.bias, g.resid, g.C, g.M, g.N, g.K, g.qscale, g.qcols, g.acc_scale, g.out_inv_scale, gm,
              g.ldc > 0 ? g.ldc : (g.epi == EPI_GEGLU ? g.N / 2 : g.N), g.pos, g.rope, g.rope_cols, g.m_dev};
  const int tiles = ((g.M + BM - 1) / BM) * (g.N / BN);
  if constexpr (ST == 0) {
    hipLaunchKernelGGL((gemm_kernel<TI, TO, TR, EPI, BM, BN, BK, WGM, WGN, OCC>), dim3(tiles),
                       dim3(WGM * WGN * 64), 0, s, p);
  } else {
    static_assert(sizeof(TI) <= 2, "the LDS ring kernel serves BF16 and FP8 operands");
    hipLaunchKernelGGL((gemm_dma_kernel<TI, TO, TR, EPI, BM, BN, BK, WGM, WGN, ST, OCC>), dim3(tiles),
                       dim3(WGM * WGN * 64), 0, s, p);
  }
  return true;
  }
}

#define ANON_CFG_CASE(i, bm, bn, bk, wgm, wgn, st, occ, name) \
  case i:                                                      \
    return run<TI, TO, TR, EPI, bm, bn, bk, wgm, wgn, st, occ>(g, s);

template <typename TI, typename TO, typename TR, int EPI>
bool dispatch_tile(const GemmParams& g, int ci, hipStream_t s) {
  if constexpr (sizeof(TI) == 2) {
    switch (ci) { ANON_BF16_CFGS(ANON_CFG_CASE) }
  } else if constexpr (sizeof(TI) == 4) {
    switch (ci) { ANON_F32_CFGS(ANON_CFG_CASE) }
  } else {
    switch (ci) { ANON_FP8_CFGS(ANON_CFG_CASE) }
  }
  return false;
}

template <typename TI>
bool dispatch_epi(const GemmParams& g, int ci, hipStream_t s) {
  // Supported (epilogue, output, residual) combinations per input type.
  if constexpr (sizeof(TI) == 4) {
    if (g.epi == EPI_BIAS && g.out == ET_F32) return dispatch_tile<TI, float, float, EPI_BIAS>(g, ci, s);
    if (g.epi == EPI_GELU && g.out == ET_F32) return dispatch_tile<TI, float, float, EPI_GELU>(g, ci, s);
    if (g.epi == EPI_RESID && g.res == ET_F32 && g.out == ET_F32)
      return dispatch_tile<TI, float, float, EPI_RESID>(g, ci, s);
    if (g.epi == EPI_ROPE && g.out == ET_F32) return dispatch_tile<TI, float, float, EPI_ROPE>(g, ci, s);
    if (g.epi == EPI_GEGLU && g.out == ET_F32) return dispatch_tile<TI, float, float, EPI_GEGLU>(g, ci, s);
  } else {
    if constexpr (sizeof(TI) == 2) {
      // the ModernBERT-style encoder: rotary QKV, gated MLP, FP32 residual stream
      if (g.epi == EPI_ROPE && g.out == ET_BF16) return dispatch_tile<TI, bf16_t, float, EPI_ROPE>(g, ci, s);
      if (g.epi == EPI_GEGLU && g.out == ET_BF16) return dispatch_tile<TI, bf16_t, float, EPI_GEGLU>(g, ci, s);
      if (g.epi == EPI_RESID && g.res == ET_F32 && g.out == ET_F32)
        return dispatch_tile<TI, float, float, EPI_RESID>(g, ci, s);
    }
    if (g.epi == EPI_BIAS && g.out == ET_BF16) return dispatch_tile<TI, bf16_t, float, EPI_BIAS>(g, ci, s);
    if constexpr (sizeof(TI) == 2) {
      if (g.epi == EPI_GELU && g.out == ET_BF16) return dispatch_tile<TI, bf16_t, float, EPI_GELU>(g, ci, s);
    } else {
      if (g.epi == EPI_GELU && g.out == ET_FP8) return dispatch_tile<TI, fp8_t, float, EPI_GELU>(g, ci, s);
    }
    if (g.epi == EPI_RESID && g.res == ET_BF16 && g.out == ET_BF16)
      return dispatch_tile<TI, bf16_t, bf16_t, EPI_RESID>(g, ci, s);
  }
  return false;
}

}  // namespace

int gemm_num_configs(ElemType in) {
  int n;
  cfgs(in, &n);
  return n;
}

const char* gemm_config_name(ElemType in, int config) {
  int n;
  const Cfg* c = cfgs(in, &n);
  return (config >= 0 && config < n) ? c[config].name : "?";
}

bool gemm_config_fits(ElemType in, int config, int N, int K) {
  int n;
  const Cfg* c = cfgs(in, &n);
  if (config < 0 || config >= n) return false;
  return N % c[config].bn == 0 && K % c[config].bk == 0;
}

static int elem_bytes(ElemType t) { return t == ET_F32 ? 4 : (t == ET_BF16 ? 2 : 1); }

bool gemm_config_serves(const GemmParams& g, int config) {
  int n;
  const Cfg* c = cfgs(g.in, &n);
  if (!gemm_config_fits(g.in, config, g.N, g.K)) return false;
  const Cfg& k = c[config];
  return staging_fits(k.bm, k.bn, k.bk, k.wgm, k.wgn, k.st, elem_bytes(g.in), elem_bytes(g.out), g.epi);
}

int default_gemm_config(const GemmParams& g) {
  // the preferred tile of the type if it serves the shape and epilogue,
  // else the first one that does
  const int n = gemm_num_configs(g.in);
  const int pref = g.in == ET_BF16 ? 11 : (g.in == ET_FP8 ? 7 : 0);
  if (gemm_config_serves(g, pref)) return pref;
  for (int c = 0; c < n; ++c)
    if (gemm_config_serves(g, c)) return c;
  return -1;
}

bool launch_gemm(const GemmParams& g, hipStream_t s) {
  int ci = g.config;
  if (ci < 0) ci = default_gemm_config(g);
  if (ci < 0 || !gemm_config_serves(g, ci)) {
    set_error(ANON_EINVAL, "gemm: no tile configuration divides N=" + std::to_string(g.N) + " K=" +
                               std::to_string(g.K));
    return false;
  }
  if ((g.epi == EPI_BIAS || g.epi == EPI_ROPE) && (g.qcols % 64 != 0 || g.rope_cols % 64 != 0)) {
    set_error(ANON_EINVAL, "gemm: scaled and rotated columns must be whole 64-column blocks");
    return false;
  }
  if (g.M <= 0) return true;
  bool ok = false;
  if (g.in == ET_F32) ok = dispatch_epi<float>(g, ci, s);
  else if (g.in == ET_BF16) ok = dispatch_epi<bf16_t>(g, ci, s);
  else ok = dispatch_epi<fp8_t>(g, ci, s);
  if (!ok) set_error(ANON_EINVAL, "gemm: unsupported type/epilogue combination");
  return ok;
}

}  // namespace anon
