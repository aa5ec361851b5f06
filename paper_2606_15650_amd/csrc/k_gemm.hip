// Dense GEMMs of the encoder on CDNA4 matrix cores, with fused epilogues.
//
// C[M,N] = A[M,K] * W[N,K]^T, A = packed token activations (no padding), W =
// a weight matrix stored transposed so that both operands are K-contiguous.
// One workgroup owns a BM x BN output tile; its waves form a WGM x WGN grid
// and each wave accumulates (BM/WGM) x (BN/WGN) with 32x32 MFMA tiles:
//   fp32: v_mfma_f32_32x32x2_f32      (K step 2)
//   bf16: v_mfma_f32_32x32x16_bf16    (K step 16)
//   fp8 : v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 operands (K step 64)
// A and W tiles are staged through double-buffered, row-padded LDS (16 bytes
// of padding per row keeps the 16-byte fragment reads of 16 lanes on distinct
// banks).  The next K tile is fetched into registers while the current one is
// multiplied, and the MFMA operands of k-step s+1 are read from LDS while the
// MFMAs of step s run.
//
// The K loop always runs in increasing k with one MFMA shape per precision,
// so each output element's sum is formed in the same order whatever the tile
// shape or the row's position in the batch (batch invariance; tile
// configurations are interchangeable bit for bit).
//
// Epilogues: bias (+ exact scaling of the Q columns by 1/sqrt(d)); bias + GELU;
// bias + residual into an FP32 pre-LayerNorm buffer.
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
  const float x = v * 0.70710678118654752f;
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly = ((((1.061405429f * t - 1.453152027f) * t + 1.421413741f) * t - 0.284496736f) * t +
                      0.254829592f) * t;
  const float e = 1.0f - poly * __expf(-ax * ax);
  return 0.5f * v * (1.0f + copysignf(e, x));
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
};

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

  // Epilogue staging (reuses the operand LDS once the K loop is done): each
  // wave parks SR rows of its tile in row-major order, then writes them back
  // with 16-byte row-contiguous accesses.  TS is the staged type: FP32 for
  // the residual epilogue (the residual is added before rounding), else TO.
  typedef typename std::conditional<EPI == EPI_RESID, float, TO>::type TS;
  constexpr int OPND_BYTES = 2 * (BM + BN) * LDK * (int)sizeof(TI);
  constexpr int SPAD = 16 / (int)sizeof(TS);
  constexpr int SROW = WTN + SPAD;
  constexpr int SR = (WGM * WGN * 32 * SROW * (int)sizeof(TS) <= OPND_BYTES) ? 32 : 16;
  static_assert(WGM * WGN * SR * SROW * (int)sizeof(TS) <= OPND_BYTES, "epilogue staging does not fit");
  __shared__ __align__(16) char smem[OPND_BYTES];
  TI(*As)[BM * LDK] = reinterpret_cast<TI(*)[BM * LDK]>(smem);
  TI(*Bs)[BN * LDK] = reinterpret_cast<TI(*)[BN * LDK]>(smem + 2 * BM * LDK * sizeof(TI));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int M = p.M, N = p.N, K = p.K;
  const int ntn = N / BN;
  const int ntm = (M + BM - 1) / BM;
  const int tile = xcd_remap(blockIdx.x, ntm * ntn);
  const int m0 = (tile / ntn) * BM, n0 = (tile % ntn) * BN;

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
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(a[cur][i], b[cur][j], acc[i][j]);
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: lane owns column (lane & 31) of each 32x32 tile and rows
  // (r/4)*8 + (lane/32)*4 + r%4 of accumulator register r.
  TO* __restrict__ C = (TO*)p.C;
  TS* stg = reinterpret_cast<TS*>(smem) + wave * SR * SROW;
  const int wrow0 = m0 + wm * WTM, wcol0 = n0 + wn * WTN;
  float bias[TN], qs[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = wcol0 + j * 32 + (lane & 31);
    bias[j] = p.bias[col];
    qs[j] = (EPI == EPI_BIAS && col < p.qcols) ? p.qscale : 1.0f;
  }
  constexpr int CH = 16 / (int)sizeof(TS);  // staged elements per 16-byte chunk
  constexpr int CPRS = WTN / CH;            // chunks per staged row
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int pass = 0; pass < 32 / SR; ++pass) {
      // 1. stage rows [pass*SR, pass*SR + SR) of sub-tile i, row-major;
      //    accumulator registers r hold rows (r/4)*8 + (lane/32)*4 + r%4, so
      //    SR rows are the registers [pass*SR/2, (pass+1)*SR/2)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int r = pass * (SR / 2); r < (pass + 1) * (SR / 2); ++r) {
          const int rin = (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3) - pass * SR;
          float v = acc[i][j][r] * p.acc_scale + bias[j];
          if (EPI == EPI_BIAS) {
            v *= qs[j];
          } else if (EPI == EPI_GELU) {
            v = gelu_erf(v);
            // FP8 output: the activation is a bf16 value first (as in the
            // BF16 path), then scaled and rounded to E4M3
            if (sizeof(TO) == 1) v = static_cast<float>(static_cast<bf16_t>(v)) * p.out_inv_scale;
          }
          st(stg + rin * SROW + j * 32 + (lane & 31), v);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      // 2. write the rows back with 16-byte (staged) chunks
      for (int c = lane; c < SR * CPRS; c += 64) {
        const int rr = c / CPRS, cc = c % CPRS;
        const int grow = wrow0 + i * 32 + pass * SR + rr, gcol = wcol0 + cc * CH;
        if (grow >= M) continue;
        const TS* src = stg + rr * SROW + cc * CH;
        if constexpr (EPI == EPI_RESID) {
          // CH = 4 FP32 sums; add the residual, round once to the output type
          const floatx4 s4 = *(const floatx4*)src;
          const TR* rp = (const TR*)p.resid + (size_t)grow * N + gcol;
          float rv[4];
          if constexpr (sizeof(TR) == 2) {
            const bf16x4 r4 = *(const bf16x4*)rp;
#pragma unroll
            for (int k = 0; k < 4; ++k) rv[k] = static_cast<float>(r4[k]);
          } else {
            const floatx4 r4 = *(const floatx4*)rp;
#pragma unroll
            for (int k = 0; k < 4; ++k) rv[k] = r4[k];
          }
          TO* dst = C + (size_t)grow * N + gcol;
          if constexpr (sizeof(TO) == 2) {
            *(bf16x4*)dst = bf16x4{static_cast<bf16_t>(s4[0] + rv[0]), static_cast<bf16_t>(s4[1] + rv[1]),
                                   static_cast<bf16_t>(s4[2] + rv[2]), static_cast<bf16_t>(s4[3] + rv[3])};
          } else {
            *(floatx4*)dst = floatx4{s4[0] + rv[0], s4[1] + rv[1], s4[2] + rv[2], s4[3] + rv[3]};
          }
        } else {
          *(intx4*)(C + (size_t)grow * N + gcol) = *(const intx4*)src;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }
}

struct Cfg {
  int bm, bn, bk, wgm, wgn, occ;
  const char* name;
};

// Tile configurations per input type; index = GemmParams::config.
#define ANON_BF16_CFGS(X)                          \
  X(0, 128, 128, 64, 2, 2, 2, "bf16_128x128x64_w2x2") \
  X(1, 256, 128, 64, 2, 2, 1, "bf16_256x128x64_w2x2") \
  X(2, 128, 256, 64, 2, 2, 1, "bf16_128x256x64_w2x2") \
  X(3, 256, 256, 64, 2, 2, 1, "bf16_256x256x64_w2x2") \
  X(4, 128, 256, 32, 2, 2, 2, "bf16_128x256x32_w2x2") \
  X(5, 256, 256, 64, 4, 2, 2, "bf16_256x256x64_w4x2") \
  X(6, 256, 256, 32, 4, 2, 2, "bf16_256x256x32_w4x2") \
  X(7, 128, 128, 32, 2, 2, 2, "bf16_128x128x32_w2x2") \
  X(8, 256, 128, 32, 4, 2, 2, "bf16_256x128x32_w4x2") \
  X(9, 128, 256, 32, 2, 4, 2, "bf16_128x256x32_w2x4") \
  X(10, 256, 128, 64, 4, 2, 2, "bf16_256x128x64_w4x2")
#define ANON_F32_CFGS(X)                        \
  X(0, 128, 128, 32, 2, 2, 2, "f32_128x128x32_w2x2") \
  X(1, 64, 64, 32, 2, 2, 2, "f32_64x64x32_w2x2")     \
  X(2, 128, 128, 16, 2, 2, 2, "f32_128x128x16_w2x2") \
  X(3, 256, 128, 16, 2, 2, 1, "f32_256x128x16_w2x2")
#define ANON_FP8_CFGS(X)                           \
  X(0, 128, 128, 128, 2, 2, 2, "fp8_128x128x128_w2x2") \
  X(1, 256, 128, 128, 2, 2, 1, "fp8_256x128x128_w2x2") \
  X(2, 128, 256, 128, 2, 2, 1, "fp8_128x256x128_w2x2") \
  X(3, 256, 256, 64, 4, 2, 2, "fp8_256x256x64_w4x2")   \
  X(4, 256, 128, 128, 4, 2, 2, "fp8_256x128x128_w4x2") \
  X(5, 128, 128, 64, 2, 2, 2, "fp8_128x128x64_w2x2")

#define ANON_CFG_ROW(i, bm, bn, bk, wgm, wgn, occ, name) {bm, bn, bk, wgm, wgn, occ, name},
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

template <typename TI, typename TO, typename TR, int EPI, int BM, int BN, int BK, int WGM, int WGN, int OCC>
void run(const GemmParams& g, hipStream_t s) {
  DevParams p{g.A, g.W, g.bias, g.resid, g.C, g.M, g.N, g.K, g.qscale, g.qcols, g.acc_scale, g.out_inv_scale};
  const int tiles = ((g.M + BM - 1) / BM) * (g.N / BN);
  hipLaunchKernelGGL((gemm_kernel<TI, TO, TR, EPI, BM, BN, BK, WGM, WGN, OCC>), dim3(tiles), dim3(WGM * WGN * 64),
                     0, s, p);
}

#define ANON_CFG_CASE(i, bm, bn, bk, wgm, wgn, occ, name) \
  case i:                                                  \
    run<TI, TO, TR, EPI, bm, bn, bk, wgm, wgn, occ>(g, s); \
    return true;

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
  } else {
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

int default_gemm_config(const GemmParams& g) {
  // the preferred tile of the type if it divides the shape, else the first
  // one that does
  const int n = gemm_num_configs(g.in);
  const int pref = g.in == ET_BF16 ? 5 : (g.in == ET_FP8 ? 3 : 0);
  if (gemm_config_fits(g.in, pref, g.N, g.K)) return pref;
  for (int c = 0; c < n; ++c)
    if (gemm_config_fits(g.in, c, g.N, g.K)) return c;
  return -1;
}

bool launch_gemm(const GemmParams& g, hipStream_t s) {
  int ci = g.config;
  if (ci < 0) ci = default_gemm_config(g);
  if (ci < 0 || !gemm_config_fits(g.in, ci, g.N, g.K)) {
    set_error(ANON_EINVAL, "gemm: no tile configuration divides N=" + std::to_string(g.N) + " K=" +
                               std::to_string(g.K));
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
