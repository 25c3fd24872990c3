// Split-bfloat16 GEMM of the correction sweeps (the bf16x3 and bf16x6 update forms).
//
//   rows[m][n] = src[(s + m) * lds + n] - sum_k X[m][k] * Y[n][k]
//
// X holds rows s.. of the FP32 copy of A and Y the FP32 change D of H made so far in the
// sweep.  Both matrices are symmetric, so the operand "column" the product needs is read as
// a row: every operand tile is a set of contiguous k-runs, which is the order in which the
// bfloat16 matrix instructions take their inputs (8 consecutive k per lane).
//
// Each FP32 value v is split on its way into LDS into bfloat16 terms, rounding to nearest
// even: t0 = bf16(v), t1 = bf16(v - t0), and for three terms t2 = bf16(v - t0 - t1); each
// difference is exact in FP32.  The product keeps the term pairs (i, j) with i + j < TERMS:
// 3 products for two terms (about 16 significant bits per operand), 6 for three terms
// (about FP32's 24).  Every bf16 x bf16 product is exact in the FP32 accumulator of
// v_mfma_f32_16x16x32_bf16.
//
// Work units are (column tile, row tile, K chunk).  Column tiles that start at or after
// `ncut` only sum k < klim (D is zero beyond the sets already processed this sweep), so they
// have fewer chunks.  With one chunk per tile the kernel writes the rows directly; otherwise
// each unit stores its FP32 partial product and split_finalize subtracts the partials from
// src in a fixed order (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace ibmi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef bf16x8 __attribute__((may_alias)) bf16x8_a;
typedef uint2 __attribute__((may_alias)) uint2_a;

__device__ __forceinline__ int64_t smin64(int64_t a, int64_t b) { return a < b ? a : b; }

typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));

// The TERMS bfloat16 terms of four consecutive values, each term packed as 4 x 16 bits.  Each
// pair converts with one v_cvt_pk_bf16_f32 (round to nearest even); converting back to FP32
// (a shift) and subtracting is exact.
template <int TERMS>
__device__ __forceinline__ void split4(const float4 v, uint2 (&out)[TERMS]) {
  v2f_t r0 = {v.x, v.y}, r1 = {v.z, v.w};
#pragma unroll
  for (int t = 0; t < TERMS; ++t) {
    const v2bf_t b0 = __builtin_convertvector(r0, v2bf_t);
    const v2bf_t b1 = __builtin_convertvector(r1, v2bf_t);
    uint32_t u0, u1;
    __builtin_memcpy(&u0, &b0, 4);
    __builtin_memcpy(&u1, &b1, 4);
    out[t] = make_uint2(u0, u1);
    if (t + 1 < TERMS) {
      r0 -= v2f_t{__uint_as_float(u0 << 16), __uint_as_float(u0 & 0xFFFF0000u)};
      r1 -= v2f_t{__uint_as_float(u1 << 16), __uint_as_float(u1 & 0xFFFF0000u)};
    }
  }
}

struct SplitArgs {
  const float* X;
  int64_t ldx, xrow0;
  const float* Y;
  int64_t ldy;
  int64_t M, N, K, klim, kchunk;
  int mtc, ntc, ntf, cf, cl, per_xcd;
  const double* src;
  int64_t lds, s;
  double* out;
  int64_t ldo;
  float* part;  // [chunk][M][N] when units write partials
  int direct;
};

// Workgroup tile BM x BN over WM x WN waves (each wave (BM/WM) x (BN/WN) of 16x16 tiles);
// K staged BK at a time through double-buffered LDS.  Rows of the LDS tiles are padded by
// 16 bytes so the 16 rows one matrix instruction reads fall on distinct banks.
// FULL: every K range is a whole number of stages, so every stage takes the vector loads and
// the loop has no branches; rows past M (N) load the last valid row instead, which only feeds
// outputs that are never stored.
template <int BM, int BN, int BK, int WM, int WN, int TERMS, bool FULL>
__global__ void __launch_bounds__(64 * WM * WN) split_gemm_kernel(SplitArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int KQ = BK / 4;  // float4 per row and stage
  // float4 loads per thread and stage; when the thread count does not divide a tile, the
  // last round is partial (XFULL / YFULL false) and guarded.
  constexpr int XL = (BM * KQ + NT - 1) / NT, YL = (BN * KQ + NT - 1) / NT;
  constexpr bool XFULL = XL * NT == BM * KQ, YFULL = YL * NT == BN * KQ;
  constexpr int LDK = BK + 8;
  static_assert(TM * 16 == WTM && TN * 16 == WTN && BK % 32 == 0, "bad wave tile");

  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][TERMS][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][TERMS][BN][LDK];

  // Unit of this workgroup: ids are dealt to the 8 XCDs round-robin; each XCD takes a
  // contiguous range, in which the row tiles of one column tile and chunk are adjacent.
  const int bx = blockIdx.x;
  const int q = (bx & 7) * a.per_xcd + (bx >> 3);
  const int uf = a.ntf * a.mtc * a.cf;
  const int total = uf + (a.ntc - a.ntf) * a.mtc * a.cl;
  if (q >= total) return;
  int nt, z, mt;
  int64_t kt;
  if (q < uf) {
    nt = q / (a.mtc * a.cf);
    const int r = q - nt * a.mtc * a.cf;
    z = r / a.mtc;
    mt = r - z * a.mtc;
    kt = a.K;
  } else {
    const int q2 = q - uf;
    const int t = q2 / (a.mtc * a.cl);
    const int r = q2 - t * a.mtc * a.cl;
    nt = a.ntf + t;
    z = r / a.mtc;
    mt = r - z * a.mtc;
    kt = smin64(a.K, a.klim);
  }
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int64_t kb = (int64_t)z * a.kchunk;
  const int64_t ke = smin64(kt, kb + a.kchunk);
  const int nk = ke > kb ? (int)((ke - kb + BK - 1) / BK) : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lk = lane >> 4;

  // Loads: float4 f = tid + v * NT of a stage covers row f / KQ, k offset 4 * (f % KQ).
  const bool rows_in = FULL || (m0 + BM <= a.M && n0 + BN <= a.N);
  const float* xbase = a.X + a.xrow0 * a.ldx;
  int64_t xo[XL], yo[YL];  // per-thread row offsets (rows clamped in the full form)
#pragma unroll
  for (int v = 0; v < XL; ++v) {
    const int f = tid + v * NT;
    const int64_t m = FULL ? smin64(m0 + f / KQ, a.M - 1) : m0 + f / KQ;
    xo[v] = m * a.ldx + 4 * (f % KQ);
  }
#pragma unroll
  for (int v = 0; v < YL; ++v) {
    const int f = tid + v * NT;
    const int64_t n = FULL ? smin64(n0 + f / KQ, a.N - 1) : n0 + f / KQ;
    yo[v] = n * a.ldy + 4 * (f % KQ);
  }
  float4 xr[XL], yr[YL];
  auto gload = [&](int kt_) {
    const int64_t k0 = kb + (int64_t)kt_ * BK;
    if (FULL || (rows_in && k0 + BK <= ke)) {
#pragma unroll
      for (int v = 0; v < XL; ++v) {
        const int f = tid + v * NT;
        if (!XFULL && f >= BM * KQ) continue;
        xr[v] = *(const float4*)(xbase + xo[v] + k0);
      }
#pragma unroll
      for (int v = 0; v < YL; ++v) {
        const int f = tid + v * NT;
        if (!YFULL && f >= BN * KQ) continue;
        yr[v] = *(const float4*)(a.Y + yo[v] + k0);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < XL; ++v) {
      const int f = tid + v * NT;
      if (!XFULL && f >= BM * KQ) continue;
      const int64_t m = m0 + f / KQ, k = k0 + 4 * (f % KQ);
      float e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        e[u] = (m < a.M && k + u < ke) ? a.X[(a.xrow0 + m) * a.ldx + k + u] : 0.0f;
      xr[v] = make_float4(e[0], e[1], e[2], e[3]);
    }
#pragma unroll
    for (int v = 0; v < YL; ++v) {
      const int f = tid + v * NT;
      if (!YFULL && f >= BN * KQ) continue;
      const int64_t n = n0 + f / KQ, k = k0 + 4 * (f % KQ);
      float e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        e[u] = (n < a.N && k + u < ke) ? a.Y[n * a.ldy + k + u] : 0.0f;
      yr[v] = make_float4(e[0], e[1], e[2], e[3]);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XL; ++v) {
      const int f = tid + v * NT;
      if (!XFULL && f >= BM * KQ) continue;
      uint2 t[TERMS];
      split4<TERMS>(xr[v], t);
#pragma unroll
      for (int w = 0; w < TERMS; ++w) *(uint2_a*)&Xs[buf][w][f / KQ][4 * (f % KQ)] = t[w];
    }
#pragma unroll
    for (int v = 0; v < YL; ++v) {
      const int f = tid + v * NT;
      if (!YFULL && f >= BN * KQ) continue;
      uint2 t[TERMS];
      split4<TERMS>(yr[v], t);
#pragma unroll
      for (int w = 0; w < TERMS; ++w) *(uint2_a*)&Ys[buf][w][f / KQ][4 * (f % KQ)] = t[w];
    }
  };

  v4f_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f_t{0, 0, 0, 0};

  auto compute = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 xa[TERMS][TM], yb[TERMS][TN];
#pragma unroll
      for (int w = 0; w < TERMS; ++w) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
          xa[w][i] = *(const bf16x8_a*)&Xs[cur][w][wm * WTM + 16 * i + lr][kk + 8 * lk];
#pragma unroll
        for (int j = 0; j < TN; ++j)
          yb[w][j] = *(const bf16x8_a*)&Ys[cur][w][wn * WTN + 16 * j + lr][kk + 8 * lk];
      }
      // Smaller terms first, the leading product last.
#pragma unroll
      for (int d = TERMS - 1; d >= 0; --d)
#pragma unroll
        for (int ti = 0; ti <= d; ++ti)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[ti][i], yb[d - ti][j],
                                                                  acc[i][j], 0, 0, 0);
    }
  };

  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  // The next stage's loads are in flight while the matrix cores work on the current one; the
  // last stage is peeled so the loop body has no conditions.
  for (int it = 0; it + 1 < nk; ++it) {
    gload(it + 1);
    compute(it & 1);
    sstore((it + 1) & 1);
    __syncthreads();
  }
  if (nk > 0) compute((nk - 1) & 1);

  // Result layout of the 16x16 FP32-accumulating instructions: register r of lane l holds
  // row 4 (l / 16) + r, column l % 16.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WTM + 16 * i + 4 * lk + r;
        const int64_t n = n0 + wn * WTN + 16 * j + lr;
        if (m >= a.M || n >= a.N) continue;
        if (a.direct)
          a.out[m * a.ldo + n] = a.src[(a.s + m) * a.lds + n] - (double)acc[i][j][r];
        else
          a.part[((int64_t)z * a.M + m) * a.N + n] = acc[i][j][r];
      }
}

__global__ void split_finalize_kernel(const float* __restrict__ part, int64_t M, int64_t N,
                                      int64_t nfull, int cf, int cl,
                                      const double* __restrict__ src, int64_t lds, int64_t s,
                                      double* __restrict__ out, int64_t ldo) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / N, n = i - m * N;
    const int nz = n < nfull ? cf : cl;
    double acc = 0.0;
    for (int z = 0; z < nz; ++z) acc += (double)part[z * total + i];
    out[m * ldo + n] = src[(s + m) * lds + n] - acc;
  }
}

// (BM, BN, BK, WM, WN) of every split configuration, in SplitCfg order.
#define IBMI_SPLIT_CONFIGS(X_)      \
  X_(SPLIT_128x128, 128, 128, 32, 2, 2) \
  X_(SPLIT_64x128, 64, 128, 32, 1, 2)   \
  X_(SPLIT_96x128, 96, 128, 32, 2, 2)   \
  X_(SPLIT_192x128, 192, 128, 32, 3, 2) \
  X_(SPLIT_144x128, 144, 128, 32, 3, 2) \
  X_(SPLIT_64x64, 64, 64, 32, 1, 1)     \
  X_(SPLIT_192x256, 192, 256, 32, 2, 4)

// One configuration and term count; configurations whose LDS would not fit (160 KiB per
// workgroup) with three terms are rejected.
template <int BM, int BN, int BK, int WM, int WN, int TERMS>
hipError_t launch_split(bool full, dim3 grid, const SplitArgs& a, hipStream_t st) {
  if constexpr (2 * TERMS * (BM + BN) * (BK + 8) * 2 > 160 * 1024) {
    return hipErrorInvalidValue;
  } else {
    if (full)
      hipLaunchKernelGGL((split_gemm_kernel<BM, BN, BK, WM, WN, TERMS, true>), grid,
                         dim3(64 * WM * WN), 0, st, a);
    else
      hipLaunchKernelGGL((split_gemm_kernel<BM, BN, BK, WM, WN, TERMS, false>), grid,
                         dim3(64 * WM * WN), 0, st, a);
    return hipGetLastError();
  }
}

}  // namespace

SplitDims split_dims(SplitCfg c) {
  switch (c) {
#define IBMI_SDIMS(NAME, BM_, BN_, BK_, WM_, WN_) \
  case NAME:                                      \
    return {BM_, BN_, BK_};
    IBMI_SPLIT_CONFIGS(IBMI_SDIMS)
#undef IBMI_SDIMS
    default: return {0, 0, 0};
  }
}

int64_t split_max_chunks(int64_t K, int64_t kchunk) {
  return kchunk > 0 ? std::max<int64_t>((K + kchunk - 1) / kchunk, 1) : 1;
}

hipError_t gemm_split_subfrom(SplitCfg cfg, int terms, const float* X, int64_t ldx,
                              int64_t xrow0, const float* Y, int64_t ldy, int64_t M, int64_t N,
                              int64_t K, int64_t ncut, int64_t klim, int64_t kchunk,
                              const double* src, int64_t lds, int64_t s, double* out,
                              int64_t ldo, float* part, hipStream_t st) {
  const SplitDims d = split_dims(cfg);
  if (d.bm == 0 || (terms != 2 && terms != 3)) return hipErrorInvalidValue;
  if (M <= 0 || N <= 0) return hipSuccess;
  // Vector loads need 16-byte aligned row starts and K chunks that are whole stages.
  if ((uintptr_t)X % 16 || (uintptr_t)Y % 16 || ldx % 4 || ldy % 4) return hipErrorInvalidValue;
  kchunk = kchunk > 0 ? (kchunk + d.bk - 1) / d.bk * d.bk : std::max<int64_t>(K, 1);
  SplitArgs a{};
  a.X = X;
  a.ldx = ldx;
  a.xrow0 = xrow0;
  a.Y = Y;
  a.ldy = ldy;
  a.M = M;
  a.N = N;
  a.K = K;
  // Rows klim .. of Y are zero in the column tiles that stop at klim: rounding up to whole
  // stages adds zeros only and spares those tiles a ragged last stage.
  klim = std::min(K, (std::max<int64_t>(klim, 0) + d.bk - 1) / d.bk * d.bk);
  a.klim = klim;
  a.kchunk = kchunk;
  a.mtc = (int)((M + d.bm - 1) / d.bm);
  a.ntc = (int)((N + d.bn - 1) / d.bn);
  a.ntf = (int)std::min<int64_t>(a.ntc, ncut <= 0 ? 0 : (ncut + d.bn - 1) / d.bn);
  const int64_t kl = std::min(K, std::max<int64_t>(klim, 0));
  a.cf = (int)split_max_chunks(K, kchunk);
  a.cl = (int)split_max_chunks(kl, kchunk);
  a.direct = (a.ntf == 0 || a.cf == 1) && (a.ntf == a.ntc || a.cl == 1);
  const int64_t units =
      (int64_t)a.ntf * a.mtc * a.cf + (int64_t)(a.ntc - a.ntf) * a.mtc * a.cl;
  a.per_xcd = (int)((units + 7) / 8);
  a.src = src;
  a.lds = lds;
  a.s = s;
  a.out = out;
  a.ldo = ldo;
  a.part = part;
  if (!a.direct && !part) return hipErrorInvalidValue;
  const dim3 grid(8 * a.per_xcd);
  // Whole stages everywhere (K, the chunks and the rounded klim are multiples of BK).
  const bool full = K % d.bk == 0;
#define IBMI_SCASE(NAME, BM_, BN_, BK_, WM_, WN_)                                       \
  case NAME:                                                                            \
    e = terms == 2 ? launch_split<BM_, BN_, BK_, WM_, WN_, 2>(full, grid, a, st)        \
                   : launch_split<BM_, BN_, BK_, WM_, WN_, 3>(full, grid, a, st);       \
    break;
  hipError_t e = hipSuccess;
  switch (cfg) {
    IBMI_SPLIT_CONFIGS(IBMI_SCASE)
    default: return hipErrorInvalidValue;
  }
#undef IBMI_SCASE
  if (e != hipSuccess || a.direct) return e;
  const int64_t total = M * N;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(split_finalize_kernel, dim3(blocks), dim3(256), 0, st, part, M, N,
                     (int64_t)a.ntf * d.bn, a.cf, a.cl, src, lds, s, out, ldo);
  return hipGetLastError();
}

}  // namespace ibmi
