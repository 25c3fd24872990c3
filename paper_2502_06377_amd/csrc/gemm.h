// Device-side MFMA GEMM templates of libibmi (gfx950), shared by the translation units that
// instantiate them.  Internal; not part of the C ABI.
//
// The hot path of a sweep is three dense FP64 contractions per set I (eq. (IBMI)):
//   panel  V = W H[I^c,I^c]             (b x c x c, the dominant 2 b c^2 term)
//   diag   G = W H[I^c,I]  -> H[I,I]    (b x b x c, the 2 b^2 c term, split over K)
//   resid  ||I - A H||_F                (p x p x p, once per sweep)
// All run on one MFMA GEMM template that reads both operands as "row k, column x" through
// index maps, so the two-segment complement I^c = [0,s) u [e,p) is addressed in place and
// never gathered into a copy.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace ibmi {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Integer min/max written out: the generic device min/max templates route 64-bit integers
// through floating point.
__device__ __forceinline__ int64_t mn64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t mx64(int64_t a, int64_t b) { return a > b ? a : b; }
__device__ __forceinline__ int mn32(int a, int b) { return a < b ? a : b; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// MFMA 16x16x4 for the two element types, with their result layouts as measured on gfx950:
// register r of lane l holds row 4r + l/16 (FP64) or row 4(l/16) + r (FP32), column l%16.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ v4d op(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ v4f op(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

// ---------------------------------------------------------------------------------------
// MFMA GEMM: C[m][n] = sum_k X(k, m) Y(k, n), operands of type T, C accumulated in T.
//
// Workgroup tile BM x BN, K staged BK at a time through LDS (double buffered: global loads
// for stage t+1 are in flight while stage t feeds the matrix cores).  WM x WN waves, each
// owning a (BM/WM) x (BN/WN) block of 16x16 MFMA tiles; every tile is an independent
// accumulation chain (on gfx950 two chains per wave with 4 waves per SIMD already keep the
// FP64 matrix pipe at 99% of peak in an MFMA-only measurement, so resident waves matter
// more than chains per wave).
// Operand tiles sit in LDS as they sit in memory ([k][x], x contiguous), which is also the
// order the MFMA fragments are read in: lane l takes X(k0 + l/16, x0 + l%16), so each
// ds_read touches 4 rows of 16 consecutive elements.
//
// Tile order: workgroup ids are dealt to the 8 XCDs round-robin, so id -> (xcd = id & 7,
// slot = id >> 3) and each XCD walks its own contiguous range of tiles; within that range
// tiles go in groups of `gm` M-tiles per N column so the workgroups resident on one XCD share
// operand panels in that XCD's L2.
// ---------------------------------------------------------------------------------------
// LDS of one tile configuration, declared in a function that does not depend on the
// epilogue (a kernel running the tile code with two epilogues holds one copy).  FP32
// fragments read 16 consecutive 4-byte words from 4 rows per instruction; padding each row by
// 64 bytes puts the 4 rows on different LDS banks.  FP64 rows are left unpadded (no bank
// conflicts measured).
template <typename T, int BM, int BN, int BK>
struct GemmSmem {
  static constexpr int PAD = sizeof(T) == 4 ? 16 : 0;
  T Xs[2][BK][BM + PAD];
  T Ys[2][BK][BN + PAD];
};
template <typename T, int BM, int BN, int BK>
__device__ __forceinline__ GemmSmem<T, BM, BN, BK>& gemm_smem() {
  __shared__ __attribute__((aligned(16))) GemmSmem<T, BM, BN, BK> sm;
  return sm;
}

// VEC-wide loads need every thread to own a multiple of VEC elements of each operand tile.
template <int XE, int YE, int VEC>
struct VecWidth {
  static constexpr int value =
      (XE % VEC == 0 && YE % VEC == 0) ? VEC : ((XE % 2 == 0 && YE % 2 == 0) ? 2 : 1);
};

// Work of one output tile: rows [mt*BM, ..) and columns [nt*BN, ..) of C, summed over k in
// [kb, ke), which is K chunk `z` of a split-K product; `slot` is where the residual
// epilogues put this tile's partial sum.  FULL: the caller guarantees VEC-wide loads are
// valid, M and N are multiples of VEC and ke - kb is a multiple of BK, so every stage takes
// the vector load path and the K loop has no branches.  Edge tiles then load the last valid
// VEC columns in place of the columns past M (N): those only feed outputs past M (N), which
// are never stored.
template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI, int VREQ, bool FULL = false>
__device__ __forceinline__ void gemm_tile(const Opnd& X, const Opnd& Y, int64_t M, int64_t N,
                                          int64_t kb, int64_t ke, int mt, int nt, int z,
                                          int64_t slot, const EpiArgs& ea) {
  typedef Mfma<T> MF;
  typedef typename MF::acc_t acc_t;
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int XE = BK * BM / NT, YE = BK * BN / NT;
  constexpr int VEC = VREQ == 1 ? 1 : VecWidth<XE, YE, VREQ>::value;
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  constexpr int XV = XE / VEC, YV = YE / VEC;
  static_assert(XE * NT == BK * BM && YE * NT == BK * BN, "tile not divisible by threads");
  static_assert(XV * VEC == XE && YV * VEC == YE && BM % VEC == 0 && BN % VEC == 0, "bad VEC");
  static_assert(TM * 16 == WTM && TN * 16 == WTN && BK % 4 == 0, "bad wave tile");

  auto& sm = gemm_smem<T, BM, BN, BK>();
  auto& Xs = sm.Xs;
  auto& Ys = sm.Ys;
  // The per-wave partial sums of the residual epilogues reuse the operand buffers: they are
  // written after the loop's last barrier, when no wave reads the operands any more.  (A
  // separate array would push the 64x64x16 tile's LDS just past a fifth of the CU's.)
  double* red_s = reinterpret_cast<double*>(&sm.Xs[0][0][0]);
  static_assert(sizeof(sm.Xs) >= (NT / 64) * sizeof(double), "no room for the wave sums");

  const int tid = threadIdx.x;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int nk = ke > kb ? (int)((ke - kb + BK - 1) / BK) : 0;

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lr = lane & 15, lk = lane >> 4;
  const T* __restrict__ xp = (const T*)X.ptr;
  const T* __restrict__ yp = (const T*)Y.ptr;

  // Interior tiles (all columns in range) take a branch-free path of VEC-wide loads: per stage
  // the operand's row base is a wave-uniform pointer and each thread adds a fixed 32-bit
  // offset (its row within the stage times ld, plus its mapped column), bumped by skip*ld
  // for rows past the map's cut.  Edge tiles and a ragged last K stage take the
  // bounds-checked scalar path.  The choice is uniform over the workgroup.
  const bool interior = FULL || (VEC > 1 && m0 + BM <= M && n0 + BN <= N);
  int xkk[XV], xoff[XV], ykk[YV], yoff[YV];
#pragma unroll
  for (int v = 0; v < XV; ++v) {
    const int idx = (tid + v * NT) * VEC;
    xkk[v] = idx / BM;
    const int64_t m = FULL ? mn64(m0 + idx % BM, M - VEC) : m0 + idx % BM;
    xoff[v] = interior ? xkk[v] * (int)X.ld + (int)X.c(m) : 0;
  }
#pragma unroll
  for (int v = 0; v < YV; ++v) {
    const int idx = (tid + v * NT) * VEC;
    ykk[v] = idx / BN;
    const int64_t n = FULL ? mn64(n0 + idx % BN, N - VEC) : n0 + idx % BN;
    yoff[v] = interior ? ykk[v] * (int)Y.ld + (int)Y.c(n) : 0;
  }
  const int xskipld = (int)(X.r.skip * X.ld), yskipld = (int)(Y.r.skip * Y.ld);

  T xr[XE], yr[YE];
  auto gload = [&](int kt) {
    const int64_t k0 = kb + (int64_t)kt * BK;
    if (FULL || (interior && k0 + BK <= ke)) {
      const T* xb = xp + (X.r.base + k0) * X.ld;
      const T* yb = yp + (Y.r.base + k0) * Y.ld;
      const int xcut = (int)mn64(mx64(X.r.cut - k0, -1), BK + 1);
      const int ycut = (int)mn64(mx64(Y.r.cut - k0, -1), BK + 1);
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int off = xoff[v] + (xkk[v] >= xcut ? xskipld : 0);
        const vec_t t = *(const vec_t*)(xb + off);
#pragma unroll
        for (int u = 0; u < VEC; ++u) xr[v * VEC + u] = t[u];
      }
#pragma unroll
      for (int v = 0; v < YV; ++v) {
        const int off = yoff[v] + (ykk[v] >= ycut ? yskipld : 0);
        const vec_t t = *(const vec_t*)(yb + off);
#pragma unroll
        for (int u = 0; u < VEC; ++u) yr[v * VEC + u] = t[u];
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < XE; ++e) {
      const int idx = (tid + (e / VEC) * NT) * VEC + e % VEC;
      const int64_t gk = k0 + idx / BM, gx = m0 + idx % BM;
      xr[e] = (gk < ke && gx < M) ? xp[X.r(gk) * X.ld + X.c(gx)] : T(0);
    }
#pragma unroll
    for (int e = 0; e < YE; ++e) {
      const int idx = (tid + (e / VEC) * NT) * VEC + e % VEC;
      const int64_t gk = k0 + idx / BN, gx = n0 + idx % BN;
      yr[e] = (gk < ke && gx < N) ? yp[Y.r(gk) * Y.ld + Y.c(gx)] : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = (tid + v * NT) * VEC;
      vec_t t;
#pragma unroll
      for (int u = 0; u < VEC; ++u) t[u] = xr[v * VEC + u];
      *(vec_t*)&Xs[buf][idx / BM][idx % BM] = t;
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = (tid + v * NT) * VEC;
      vec_t t;
#pragma unroll
      for (int u = 0; u < VEC; ++u) t[u] = yr[v * VEC + u];
      *(vec_t*)&Ys[buf][idx / BN][idx % BN] = t;
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  auto compute = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = Xs[cur][kk + lk][wm * WTM + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Ys[cur][kk + lk][wn * WTN + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i], b[j], acc[i][j]);
    }
  };

  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  // Stages 0 .. nk-2 prefetch the next stage into registers while the matrix cores work on
  // the current one; the last stage is peeled so the loop body has no conditions.
  for (int kt = 0; kt + 1 < nk; ++kt) {
    gload(kt + 1);
    compute(kt & 1);
    sstore((kt + 1) & 1);
    __syncthreads();
  }
  if (nk > 0) {
    compute((nk - 1) & 1);
    __syncthreads();
  }

  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WTM + 16 * i + MF::row(r, lk);
        const int64_t n = n0 + wn * WTN + 16 * j + lr;
        const double v = (double)acc[i][j][r];
        if (m >= M || n >= N) continue;
        if constexpr (EPI == EPI_STORE) {
          ea.out[m * ea.ldo + n] = v;
        } else if constexpr (EPI == EPI_PANEL) {
          const int64_t gn = ea.g(n);
          ea.out[(ea.s + m) * ea.ldo + gn] = -v;
          ea.out[gn * ea.ldo + ea.s + m] = -v;
        } else if constexpr (EPI == EPI_PARTIAL) {
          ea.out[(int64_t)z * M * N + m * N + n] = v;
        } else if constexpr (EPI == EPI_RESID) {
          const double d = (m == n ? 1.0 : 0.0) - v;
          ss += d * d;
        } else if constexpr (EPI == EPI_RESID_STORE) {
          const double d = (m == n ? 1.0 : 0.0) - v;
          ea.out[m * ea.ldo + n] = d;
          ss += d * d;
        } else if constexpr (EPI == EPI_SUMSQ) {
          ss += v * v;
        } else if constexpr (EPI == EPI_SUBFROM) {
          ea.out[m * ea.ldo + n] = ea.src[(ea.s + m) * ea.lds + n] - v;
        } else {
          // EPI_CORR: C = Delta[m][n] (m over I^c, n over I).  Store Delta, then add it to
          // H[g(m)][s+n] and mirror the new value to H[s+n][g(m)]; the same for the FP32
          // change D, so H and D stay bitwise symmetric.
          ea.out[m * ea.ldo + n] = v;
          const int64_t gm_ = ea.g(m), cn = ea.s + n;
          const double hn = ea.H[gm_ * ea.ldh + cn] + v;
          ea.H[gm_ * ea.ldh + cn] = hn;
          ea.H[cn * ea.ldh + gm_] = hn;
          const float dn = ea.D[gm_ * ea.ldd + cn] + (float)v;
          ea.D[gm_ * ea.ldd + cn] = dn;
          ea.D[cn * ea.ldd + gm_] = dn;
        }
      }
  if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_STORE || EPI == EPI_SUMSQ) {
    ss = wave_sum(ss);
    if (lane == 0) red_s[wave] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red_s[w];
      ea.red[slot] = t;
    }
  }
}

// (BM, BN, BK, WM, WN) of every configuration, in GemmCfg order.
#define IBMI_GEMM_CONFIGS(X_)                                                                  \
  X_(GEMM_64x64, 64, 64, 32, 2, 2)                                                             \
  X_(GEMM_64x64_K16, 64, 64, 16, 2, 2)                                                         \
  X_(GEMM_128x128_W8, 128, 128, 16, 2, 4)                                                      \
  X_(GEMM_96x128_W8, 96, 128, 32, 2, 4)                                                        \
  X_(GEMM_96x64_K16, 96, 64, 16, 2, 2)                                                         \
  X_(GEMM_64x128_K16, 64, 128, 16, 2, 2)                                                       \
  X_(GEMM_64x64_W1, 64, 64, 16, 1, 1)                                                          \
  X_(GEMM_32x64_W1, 32, 64, 16, 1, 1)                                                          \
  X_(GEMM_64x64_W2, 64, 64, 32, 2, 1)                                                          \
  X_(GEMM_96x128, 96, 128, 32, 2, 2)                                                           \
  X_(GEMM_192x96, 192, 96, 16, 2, 2)

// Waves per SIMD that the LDS of one workgroup allows (160 KiB per CU, 4 SIMDs), capped at 8.
// The 8-wave tiles of the residual epilogues that store or square the product ask the
// compiler for at least this occupancy: left alone it spends a few registers more than that
// occupancy leaves and loses a wave per SIMD (measured: 57.7 against 65.8 TFLOP/s for the
// stored residual at p = 16384).
template <typename T, int BM, int BN, int BK, int WM, int WN>
constexpr int gemm_lds_waves() {
  constexpr int pad = sizeof(T) == 4 ? 16 : 0;
  constexpr int lds = 2 * BK * (BM + BN + 2 * pad) * (int)sizeof(T);
  constexpr int wgs = (160 * 1024) / lds;
  constexpr int w = wgs * WM * WN / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}
template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI>
constexpr int gemm_min_waves() {
  if ((EPI != EPI_RESID_STORE && EPI != EPI_SUMSQ) || WM * WN != 8) return 1;
  return gemm_lds_waves<T, BM, BN, BK, WM, WN>();
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI, int VREQ, bool FULL>
__global__ void __launch_bounds__(64 * WM * WN)
__attribute__((amdgpu_waves_per_eu(gemm_min_waves<T, BM, BN, BK, WM, WN, EPI>())))
gemm_kernel(Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, int64_t kchunk, int mtc, int ntc,
            int per_xcd, int gm, EpiArgs ea) {
  const int bx = blockIdx.x;
  const int q = (bx & 7) * per_xcd + (bx >> 3);
  const int tiles = mtc * ntc;
  if (q >= tiles) return;
  int mt, nt;
  {
    const int width = gm * ntc;
    const int grp = q / width;
    const int first_m = grp * gm;
    const int gsz = mn32(mtc - first_m, gm);
    const int rem = q - grp * width;
    mt = first_m + rem % gsz;
    nt = rem / gsz;
  }
  const int64_t n0 = (int64_t)nt * BN;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = mn64(n0 >= ea.ncut ? mn64(K, ea.klim) : K, kb + kchunk);
  gemm_tile<T, BM, BN, BK, WM, WN, EPI, VREQ, FULL>(X, Y, M, N, kb, ke, mt, nt, (int)blockIdx.y,
                                                     q, ea);
}

// Grouped form: many independent products in one launch.  Workgroup b finds its task t by
// binary search of the tile prefix sums (tile_off[t] <= b < tile_off[t+1]), skips tasks of
// matrices that are no longer active, and runs tile b - tile_off[t] of that task.
template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI, int VREQ>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_grouped_kernel(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_off,
                    int ntasks, const int* __restrict__ active) {
  const int bx = blockIdx.x;
  int lo = 0, hi = ntasks;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_off[mid] <= bx) lo = mid;
    else hi = mid;
  }
  const GemmTask tk = tasks[lo];
  if (active && !active[tk.mat]) return;
  const int local = bx - tile_off[lo];
  const int per = tk.mtc * tk.ntc;
  const int z = local / per, rem = local - z * per;
  const int mt = rem % tk.mtc, nt = rem / tk.mtc;
  const int64_t kb = (int64_t)z * tk.kchunk;
  const int64_t ke = mn64(tk.K, kb + tk.kchunk);
  gemm_tile<T, BM, BN, BK, WM, WN, EPI, VREQ>(tk.X, tk.Y, tk.M, tk.N, kb, ke, mt, nt, z, local,
                                               tk.ea);
}

// The fast path also needs every per-thread offset (row-in-stage * ld + column + skip * ld)
// to fit in 32 bits.
template <typename T>
inline bool vec_ok(const Opnd& o, int vec, int64_t ncols) {
  auto m = [vec](int64_t v) { return v % vec == 0; };
  const int64_t span = 64 * o.ld + o.c(ncols > 0 ? ncols - 1 : 0) + o.r.skip * o.ld;
  return ((uintptr_t)o.ptr % 16) == 0 && m(o.ld) && m(o.c.base) && m(o.c.skip) &&
         (o.c.cut == INT64_MAX || m(o.c.cut)) && span < INT32_MAX;
}

template <typename T, int EPI>
inline hipError_t launch_gemm(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                              int splits, EpiArgs ea, hipStream_t st, int64_t* n_tiles) {
  constexpr int VMAX = 16 / sizeof(T);
  const bool vec = vec_ok<T>(X, VMAX, M) && vec_ok<T>(Y, VMAX, N);
  const GemmDims d = gemm_dims(cfg);
  const int mtc = (int)((M + d.bm - 1) / d.bm), ntc = (int)((N + d.bn - 1) / d.bn);
  const int tiles = mtc * ntc;
  if (n_tiles) *n_tiles = tiles;
  if (tiles == 0) return hipSuccess;
  const int per_xcd = (tiles + 7) / 8;
  // Square residual-type products walk groups of 8 row tiles; the panel and diagonal
  // products (few row tiles) walk whole columns.
  const int gm = (EPI == EPI_RESID || EPI == EPI_RESID_STORE || EPI == EPI_SUMSQ) ? 8 : mtc;
  const int bk = d.bk;
  // Split-K chunks are whole stages, so that with K a multiple of BK every K range is.
  const int64_t kchunk =
      splits > 1 ? ((K + splits - 1) / splits + bk - 1) / bk * bk : (K > 0 ? K : 1);
  const dim3 grid(8 * per_xcd, splits > 1 ? splits : 1);
  // Every K range a whole number of stages and M, N whole vectors: the branch-free loop.
  const bool full = vec && M % VMAX == 0 && N % VMAX == 0 && K > 0 && K % bk == 0 &&
                    (ea.ncut == INT64_MAX || ea.klim % bk == 0 || ea.klim >= K);
#define IBMI_LAUNCH(BM_, BN_, BK_, WM_, WN_)                                                   \
  do {                                                                                         \
    if (full)                                                                                  \
      hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, VMAX, true>), grid,     \
                         dim3(64 * WM_ * WN_), 0, st, X, Y, M, N, K, kchunk, mtc, ntc, per_xcd, \
                         gm, ea);                                                              \
    else if (vec)                                                                              \
      hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, VMAX, false>), grid,    \
                         dim3(64 * WM_ * WN_), 0, st, X, Y, M, N, K, kchunk, mtc, ntc, per_xcd, \
                         gm, ea);                                                              \
    else                                                                                       \
      hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, 1, false>), grid,       \
                         dim3(64 * WM_ * WN_), 0, st, X, Y, M, N, K, kchunk, mtc, ntc, per_xcd, \
                         gm, ea);                                                              \
  } while (0)
  switch (cfg) {
#define IBMI_CASE(NAME, BM_, BN_, BK_, WM_, WN_) \
  case NAME:                                     \
    IBMI_LAUNCH(BM_, BN_, BK_, WM_, WN_);        \
    break;
    IBMI_GEMM_CONFIGS(IBMI_CASE)
#undef IBMI_CASE
    default: return hipErrorInvalidValue;
  }
#undef IBMI_LAUNCH
  return hipGetLastError();
}

template <typename T, int EPI>
inline hipError_t launch_grouped(GemmCfg cfg, const GemmTask* tasks, const int* tile_off,
                                 int ntasks, int total_tiles, const int* active, bool vec,
                                 hipStream_t st) {
  constexpr int VMAX = 16 / sizeof(T);
  const dim3 grid(total_tiles);
#define IBMI_GLAUNCH(BM_, BN_, BK_, WM_, WN_)                                                   \
  do {                                                                                          \
    if (vec)                                                                                    \
      hipLaunchKernelGGL((gemm_grouped_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, VMAX>), grid,    \
                         dim3(64 * WM_ * WN_), 0, st, tasks, tile_off, ntasks, active);         \
    else                                                                                        \
      hipLaunchKernelGGL((gemm_grouped_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, 1>), grid,       \
                         dim3(64 * WM_ * WN_), 0, st, tasks, tile_off, ntasks, active);         \
  } while (0)
  switch (cfg) {
#define IBMI_GCASE(NAME, BM_, BN_, BK_, WM_, WN_) \
  case NAME:                                      \
    IBMI_GLAUNCH(BM_, BN_, BK_, WM_, WN_);        \
    break;
    IBMI_GEMM_CONFIGS(IBMI_GCASE)
#undef IBMI_GCASE
    default: return hipErrorInvalidValue;
  }
#undef IBMI_GLAUNCH
  return hipGetLastError();
}

}  // namespace ibmi
