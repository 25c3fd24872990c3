// gfx950 (CDNA4) kernels of the IBMI library.
//
// The hot path of a sweep is three dense FP64 contractions per set I (eq. (IBMI)):
//   panel  V = W H[I^c,I^c]             (b x c x c, the dominant 2 b c^2 term)
//   diag   G = W H[I^c,I]  -> H[I,I]    (b x b x c, the 2 b^2 c term, split over K)
//   resid  ||I - A H||_F                (p x p x p, once per sweep)
// All three run on one FP64 MFMA GEMM template (v_mfma_f64_16x16x4f64) that reads both
// operands as "row k, column x" through index maps, so the two-segment complement
// I^c = [0,s) u [e,p) is addressed in place and never gathered into a copy.  Block factors
// (Cholesky, L^{-1}, A_I^{-1}) run once per plan.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace ibmi {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

enum {
  EPI_STORE = 0,        // out[m][n] = C
  EPI_PANEL = 1,        // H[s+m][g(n)] = H[g(n)][s+m] = -C
  EPI_PARTIAL = 2,      // out[z][m][n] = C over K chunk z
  EPI_RESID = 3,        // red[tile] = sum (delta_mn - C)^2
  EPI_RESID_STORE = 4,  // out[m][n] = delta_mn - C and red[tile] = sum of its squares
  EPI_SUBFROM = 5,      // out[m][n] = src[(s+m)][n] - C
  EPI_CORR = 6          // correction of H[I^c,I] and D (see below)
};

struct EpiArgs {
  double* out = nullptr;   // primary output
  int64_t ldo = 0;
  int64_t s = 0;           // first row of I
  IdxMap g;                // column map of I^c
  double* red = nullptr;   // per-tile partial sums (residual epilogues)
  const double* src = nullptr;  // subtrahend rows (EPI_SUBFROM)
  int64_t lds = 0;
  double* H = nullptr;     // EPI_CORR targets
  int64_t ldh = 0;
  float* D = nullptr;
  int64_t ldd = 0;
  int64_t ncut = INT64_MAX;  // column tiles starting at or after ncut stop K at klim
  int64_t klim = 0;
};

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
// accumulation chain, and a wave needs about 8 of them in flight to keep the FP64 matrix
// pipe busy (a measured property of gfx950: 4 chains per wave reach ~60% of peak).
// Operand tiles sit in LDS as they sit in memory ([k][x], x contiguous), which is also the
// order the MFMA fragments are read in: lane l takes X(k0 + l/16, x0 + l%16), so each
// ds_read touches 4 rows of 16 consecutive elements.
//
// Tile order: workgroup ids are dealt to the 8 XCDs round-robin, so id -> (xcd = id & 7,
// slot = id >> 3) and each XCD walks its own contiguous range of tiles; within that range
// tiles go in groups of `gm` M-tiles per N column so the workgroups resident on one XCD share
// operand panels in that XCD's L2.
// ---------------------------------------------------------------------------------------
// VEC-wide loads need every thread to own a multiple of VEC elements of each operand tile.
template <int XE, int YE, int VEC>
struct VecWidth {
  static constexpr int value =
      (XE % VEC == 0 && YE % VEC == 0) ? VEC : ((XE % 2 == 0 && YE % 2 == 0) ? 2 : 1);
};

template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI, int VREQ>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_kernel(Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, int64_t kchunk, int mtc, int ntc,
            int per_xcd, int gm, EpiArgs ea) {
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

  __shared__ __attribute__((aligned(16))) T Xs[2][BK][BM];
  __shared__ __attribute__((aligned(16))) T Ys[2][BK][BN];
  __shared__ double red_s[NT / 64];

  const int tid = threadIdx.x;
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
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = mn64(n0 >= ea.ncut ? mn64(K, ea.klim) : K, kb + kchunk);
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
  const bool interior = VEC > 1 && m0 + BM <= M && n0 + BN <= N;
  int xkk[XV], xoff[XV], ykk[YV], yoff[YV];
#pragma unroll
  for (int v = 0; v < XV; ++v) {
    const int idx = (tid + v * NT) * VEC;
    xkk[v] = idx / BM;
    xoff[v] = interior ? xkk[v] * (int)X.ld + (int)X.c(m0 + idx % BM) : 0;
  }
#pragma unroll
  for (int v = 0; v < YV; ++v) {
    const int idx = (tid + v * NT) * VEC;
    ykk[v] = idx / BN;
    yoff[v] = interior ? ykk[v] * (int)Y.ld + (int)Y.c(n0 + idx % BN) : 0;
  }
  const int xskipld = (int)(X.r.skip * X.ld), yskipld = (int)(Y.r.skip * Y.ld);

  T xr[XE], yr[YE];
  auto gload = [&](int kt) {
    const int64_t k0 = kb + (int64_t)kt * BK;
    if (interior && k0 + BK <= ke) {
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

  if (nk > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
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
    if (kt + 1 < nk) sstore(cur ^ 1);
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
          ea.out[(int64_t)blockIdx.y * M * N + m * N + n] = v;
        } else if constexpr (EPI == EPI_RESID) {
          const double d = (m == n ? 1.0 : 0.0) - v;
          ss += d * d;
        } else if constexpr (EPI == EPI_RESID_STORE) {
          const double d = (m == n ? 1.0 : 0.0) - v;
          ea.out[m * ea.ldo + n] = d;
          ss += d * d;
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
  if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_STORE) {
    ss = wave_sum(ss);
    if (lane == 0) red_s[wave] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red_s[w];
      ea.red[q] = t;
    }
  }
}

// (BM, BN, BK, WM, WN) of every configuration, in GemmCfg order.
#define IBMI_GEMM_CONFIGS(X_)                                                                  \
  X_(GEMM_64x64, 64, 64, 32, 2, 2)                                                             \
  X_(GEMM_128x128, 128, 128, 32, 2, 2)                                                         \
  X_(GEMM_96x128, 96, 128, 32, 2, 2)                                                           \
  X_(GEMM_128x64, 128, 64, 32, 2, 2)                                                           \
  X_(GEMM_192x64, 192, 64, 32, 2, 2)                                                           \
  X_(GEMM_64x64_W1, 64, 64, 16, 1, 1)                                                          \
  X_(GEMM_32x64_W1, 32, 64, 16, 1, 1)                                                          \
  X_(GEMM_64x64_K16, 64, 64, 16, 2, 2)                                                         \
  X_(GEMM_128x64_K16, 128, 64, 16, 2, 2)                                                       \
  X_(GEMM_64x128_K16, 64, 128, 16, 2, 2)                                                       \
  X_(GEMM_128x128_W8, 128, 128, 16, 2, 4)                                                      \
  X_(GEMM_128x128_W16, 128, 128, 16, 4, 4)                                                     \
  X_(GEMM_96x64_K16, 96, 64, 16, 2, 2)                                                         \
  X_(GEMM_192x128_W8, 192, 128, 16, 2, 4)                                                      \
  X_(GEMM_64x64_W2, 64, 64, 32, 2, 1)

GemmDims gemm_dims(GemmCfg c) {
  switch (c) {
#define IBMI_DIMS(NAME, BM_, BN_, BK_, WM_, WN_) \
  case NAME:                                     \
    return {BM_, BN_};
    IBMI_GEMM_CONFIGS(IBMI_DIMS)
#undef IBMI_DIMS
    default: return {64, 64};
  }
}

// True when every VEC-wide run of columns x, x+1, .. (x a multiple of VEC) of the operand is
// contiguous and 16-byte aligned in memory.
// The fast path also needs every per-thread offset (row-in-stage * ld + column + skip * ld)
// to fit in 32 bits.
template <typename T>
static bool vec_ok(const Opnd& o, int vec, int64_t ncols) {
  auto m = [vec](int64_t v) { return v % vec == 0; };
  const int64_t span = 64 * o.ld + o.c(ncols > 0 ? ncols - 1 : 0) + o.r.skip * o.ld;
  return ((uintptr_t)o.ptr % 16) == 0 && m(o.ld) && m(o.c.base) && m(o.c.skip) &&
         (o.c.cut == INT64_MAX || m(o.c.cut)) && span < INT32_MAX;
}

template <typename T, int EPI>
static hipError_t launch_gemm(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                              int splits, EpiArgs ea, hipStream_t st, int64_t* n_tiles) {
  constexpr int VMAX = 16 / sizeof(T);
  const bool vec = vec_ok<T>(X, VMAX, M) && vec_ok<T>(Y, VMAX, N);
  const GemmDims d = gemm_dims(cfg);
  const int mtc = (int)((M + d.bm - 1) / d.bm), ntc = (int)((N + d.bn - 1) / d.bn);
  const int tiles = mtc * ntc;
  if (n_tiles) *n_tiles = tiles;
  if (tiles == 0) return hipSuccess;
  const int per_xcd = (tiles + 7) / 8;
  const int gm = EPI == EPI_RESID ? 8 : mtc;
  const int64_t kchunk = splits > 1 ? (K + splits - 1) / splits : (K > 0 ? K : 1);
  const dim3 grid(8 * per_xcd, splits > 1 ? splits : 1);
#define IBMI_LAUNCH(BM_, BN_, BK_, WM_, WN_)                                                   \
  do {                                                                                         \
    if (vec)                                                                                   \
      hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, VMAX>), grid,           \
                         dim3(64 * WM_ * WN_), 0, st, X, Y, M, N, K, kchunk, mtc, ntc, per_xcd, \
                         gm, ea);                                                              \
    else                                                                                       \
      hipLaunchKernelGGL((gemm_kernel<T, BM_, BN_, BK_, WM_, WN_, EPI, 1>), grid,              \
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

hipError_t gemm_store(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* out,
                      int64_t ldo, hipStream_t st) {
  EpiArgs ea;
  ea.out = out;
  ea.ldo = ldo;
  return launch_gemm<double, EPI_STORE>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

hipError_t gemm_panel(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* H,
                      int64_t ldh, int64_t s, IdxMap g, hipStream_t st) {
  EpiArgs ea;
  ea.out = H;
  ea.ldo = ldh;
  ea.s = s;
  ea.g = g;
  return launch_gemm<double, EPI_PANEL>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

hipError_t gemm_partial(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, int splits,
                        double* out, hipStream_t st) {
  EpiArgs ea;
  ea.out = out;
  return launch_gemm<double, EPI_PARTIAL>(cfg, X, Y, M, N, K, splits, ea, st, nullptr);
}

int64_t gemm_tiles(GemmCfg cfg, int64_t M, int64_t N) {
  const GemmDims d = gemm_dims(cfg);
  return ((M + d.bm - 1) / d.bm) * ((N + d.bn - 1) / d.bn);
}

hipError_t gemm_resid(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* red,
                      int64_t* n_red, double* out, int64_t ldo, hipStream_t st) {
  EpiArgs ea;
  ea.red = red;
  if (out) {
    ea.out = out;
    ea.ldo = ldo;
    return launch_gemm<double, EPI_RESID_STORE>(cfg, X, Y, M, N, K, 1, ea, st, n_red);
  }
  return launch_gemm<double, EPI_RESID>(cfg, X, Y, M, N, K, 1, ea, st, n_red);
}

hipError_t gemm_f32_subfrom(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                            int64_t ncut, int64_t klim, const double* src, int64_t lds,
                            int64_t s, double* out, int64_t ldo, hipStream_t st) {
  EpiArgs ea;
  ea.out = out;
  ea.ldo = ldo;
  ea.src = src;
  ea.lds = lds;
  ea.s = s;
  ea.ncut = ncut;
  ea.klim = klim;
  return launch_gemm<float, EPI_SUBFROM>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

hipError_t gemm_corr(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* delta,
                     int64_t ld_delta, double* H, int64_t ldh, float* D, int64_t ldd, int64_t s,
                     IdxMap g, hipStream_t st) {
  EpiArgs ea;
  ea.out = delta;
  ea.ldo = ld_delta;
  ea.H = H;
  ea.ldh = ldh;
  ea.D = D;
  ea.ldd = ldd;
  ea.s = s;
  ea.g = g;
  return launch_gemm<double, EPI_CORR>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

// ---------------------------------------------------------------------------------------
// Cholesky factor of every diagonal block, one workgroup (16 waves) per set.
// Right-looking, panels of NB columns held in LDS (row stride NB+1 to spread banks):
// factor the panel, write it back as L (lower) and L^T (strict upper, so that row i of the
// upper part is column i of L and reads stay contiguous), then update the trailing lower
// triangle.  A non-positive or non-finite pivot records the set index (atomicMin) and stops.
// ---------------------------------------------------------------------------------------
constexpr int CH_NB = 16;
constexpr int CH_THREADS = 1024;

__global__ void __launch_bounds__(CH_THREADS)
chol_factor_kernel(const BlockDesc* desc, const double* A, int64_t lda, double* fac,
                   int* status) {
  extern __shared__ double Ps[];  // rows x (CH_NB + 1)
  constexpr int LDP = CH_NB + 1;
  const BlockDesc bd = desc[blockIdx.x];
  const int b = (int)bd.b;
  const int64_t s = bd.s;
  double* L = fac + bd.l_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = CH_THREADS / 64;

  for (int64_t e = tid; e < (int64_t)b * b; e += CH_THREADS) {
    const int64_t i = e / b, j = e % b;
    L[e] = A[(s + i) * lda + s + j];
  }
  __syncthreads();

  for (int jb = 0; jb < b; jb += CH_NB) {
    const int nb = mn32(CH_NB, b - jb);
    const int rows = b - jb;
    for (int e = tid; e < rows * nb; e += CH_THREADS) {
      const int r = e / nb, c = e % nb;
      Ps[r * LDP + c] = L[(int64_t)(jb + r) * b + jb + c];
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      const double piv = Ps[c * LDP + c];
      if (!(piv > 0.0) || !(piv < INFINITY)) {  // uniform: every thread read the same value
        if (tid == 0) atomicMin(status, (int)blockIdx.x);
        return;
      }
      const double l = sqrt(piv);
      __syncthreads();
      for (int r = c + tid; r < rows; r += CH_THREADS)
        Ps[r * LDP + c] = (r == c) ? l : Ps[r * LDP + c] / l;
      __syncthreads();
      const int w = nb - c - 1;
      if (w > 0) {
        for (int e = tid; e < rows * w; e += CH_THREADS) {
          const int r = e / w, d = c + 1 + e % w;
          if (r >= d) Ps[r * LDP + d] -= Ps[r * LDP + c] * Ps[d * LDP + c];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * nb; e += CH_THREADS) {
      const int r = e / nb, c = e % nb;
      if (r >= c) {
        const double v = Ps[r * LDP + c];
        L[(int64_t)(jb + r) * b + jb + c] = v;
        if (r > c) L[(int64_t)(jb + c) * b + jb + r] = v;
      }
    }
    // trailing update of the lower triangle: rows/cols >= nb (panel-relative)
    for (int i = nb + wave; i < rows; i += NW) {
      double* Lrow = L + (int64_t)(jb + i) * b + jb;
      for (int j = nb + lane; j <= i; j += 64) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < CH_NB; ++t)
          if (t < nb) acc += Ps[i * LDP + t] * Ps[j * LDP + t];
        Lrow[j] -= acc;
      }
    }
    __syncthreads();
  }
}

// L^{-1} by forward substitution, one wave per pair of columns (no LDS, no barriers).
// Column j of L^{-1} is y with L y = e_j; lane l keeps y[l + 64u] in registers.  The row of
// L is read contiguously (t < i selects the lower part).  Writes L^{-1} row-major, zeros
// above the diagonal.
constexpr int LINV_SLOTS = 16;  // b <= 1024

__global__ void __launch_bounds__(64) chol_linv_kernel(const BlockDesc* desc, double* fac) {
  const BlockDesc bd = desc[blockIdx.y];
  const int b = (int)bd.b;
  const int j0 = blockIdx.x * 2;
  if (j0 >= b) return;
  const int j1 = j0 + 1;
  const double* L = fac + bd.l_off;
  double* Linv = fac + bd.linv_off;
  const int lane = threadIdx.x;
  const int nu = (b + 63) / 64;
  double y0[LINV_SLOTS], y1[LINV_SLOTS];
#pragma unroll
  for (int u = 0; u < LINV_SLOTS; ++u) y0[u] = y1[u] = 0.0;
  for (int i = j0; i < b; ++i) {
    const double* Li = L + (int64_t)i * b;
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int u = 0; u < LINV_SLOTS; ++u) {
      const int t = lane + 64 * u;
      if (u < nu && t < i) {
        const double l = Li[t];
        p0 += l * y0[u];
        p1 += l * y1[u];
      }
    }
    p0 = wave_sum(p0);
    p1 = wave_sum(p1);
    const double lii = Li[i];
    const double v0 = ((i == j0 ? 1.0 : 0.0) - p0) / lii;
    const double v1 = i >= j1 ? ((i == j1 ? 1.0 : 0.0) - p1) / lii : 0.0;
    const int ou = i >> 6, ol = i & 63;
#pragma unroll
    for (int u = 0; u < LINV_SLOTS; ++u)
      if (u == ou && lane == ol) {
        y0[u] = v0;
        y1[u] = v1;
      }
  }
#pragma unroll
  for (int u = 0; u < LINV_SLOTS; ++u) {
    const int t = lane + 64 * u;
    if (u < nu && t < b) {
      Linv[(int64_t)t * b + j0] = y0[u];
      if (j1 < b) Linv[(int64_t)t * b + j1] = y1[u];
    }
  }
}

hipError_t chol_factor(const BlockDesc* d_desc, int n_blocks, int64_t b_max, const double* A,
                       int64_t lda, double* fac, int* d_status, hipStream_t st) {
  const size_t lds = (size_t)b_max * (CH_NB + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)chol_factor_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chol_factor_kernel, dim3(n_blocks), dim3(CH_THREADS), lds, st, d_desc, A,
                     lda, fac, d_status);
  return hipGetLastError();
}

hipError_t chol_linv(const BlockDesc* d_desc, int n_blocks, int64_t b_max, double* fac,
                     hipStream_t st) {
  hipLaunchKernelGGL(chol_linv_kernel, dim3((unsigned)((b_max + 1) / 2), n_blocks), dim3(64), 0,
                     st, d_desc, fac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Small elementwise kernels.
// ---------------------------------------------------------------------------------------
__global__ void symmetrize_kernel(const double* x, double* out, int64_t b) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    out[e] = 0.5 * (x[e] + x[j * b + i]);
  }
}

hipError_t symmetrize_block(const double* x, double* out, int64_t b, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(grid), dim3(256), 0, st, x, out, b);
  return hipGetLastError();
}

// H[I,I] = A_I^{-1} - (G + G^T)/2; G[m][n] = sum_z partial[z][m][n] in z order.  Both
// (m,n) and (n,m) use the same sums, so the block is bitwise symmetric.
__global__ void diag_finalize_kernel(const double* ainv, const double* part, int splits,
                                     int64_t b, double* H, int64_t ldh, int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double gij = 0.0, gji = 0.0;
    for (int z = 0; z < splits; ++z) {
      gij += part[z * n + i * b + j];
      gji += part[z * n + j * b + i];
    }
    H[(s + i) * ldh + s + j] = ainv[e] - 0.5 * (gij + gji);
  }
}

hipError_t diag_finalize(const double* ainv, const double* partial, int splits, int64_t b,
                         double* H, int64_t ldh, int64_t s, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(diag_finalize_kernel, dim3(grid), dim3(256), 0, st, ainv, partial, splits,
                     b, H, ldh, s);
  return hipGetLastError();
}

__global__ void fill_identity_kernel(double* H, int64_t ldh, int64_t p, double diag) {
  const int64_t n = p * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / p, j = e % p;
    H[i * ldh + j] = (i == j) ? diag : 0.0;
  }
}

hipError_t fill_identity(double* H, int64_t ldh, int64_t p, double diag, hipStream_t st) {
  const int64_t n = p * p;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_identity_kernel, dim3(grid), dim3(256), 0, st, H, ldh, p, diag);
  return hipGetLastError();
}

__global__ void copy_block_kernel(const double* src, int64_t b, double* H, int64_t ldh,
                                  int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    H[(s + i) * ldh + s + j] = src[e];
  }
}

hipError_t copy_block(const double* src, int64_t b, double* H, int64_t ldh, int64_t s,
                      hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(copy_block_kernel, dim3(grid), dim3(256), 0, st, src, b, H, ldh, s);
  return hipGetLastError();
}

// Sum of squares with a fixed grid: workgroup g takes rows g, g + G, ... in order.
constexpr int SUMSQ_GRID = 1024;
__global__ void __launch_bounds__(256) sumsq_kernel(const double* H, int64_t ldh, int64_t p,
                                                    double* red) {
  __shared__ double ws[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x; i < p; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < p; j += blockDim.x) {
      const double v = H[i * ldh + j];
      acc += v * v;
    }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) red[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

hipError_t sumsq(const double* H, int64_t ldh, int64_t p, double* red, int64_t* n_red,
                 hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(SUMSQ_GRID), dim3(256), 0, st, H, ldh, p, red);
  *n_red = SUMSQ_GRID;
  return hipGetLastError();
}

__global__ void __launch_bounds__(1024) reduce_sum_kernel(const double* red, int64_t n,
                                                          double* out) {
  __shared__ double ws[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += red[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += ws[w];
    out[0] = t;
  }
}

hipError_t reduce_sum(const double* red, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, red, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Mixed (FP32-update) form helpers.
// ---------------------------------------------------------------------------------------
__global__ void to_f32_kernel(const double* a, int64_t lda, float* out, int64_t p) {
  const int64_t n = p * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / p, j = e % p;
    out[e] = (float)a[i * lda + j];
  }
}

hipError_t to_f32(const double* a, int64_t lda, float* out, int64_t p, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(8192), dim3(256), 0, st, a, lda, out, p);
  return hipGetLastError();
}

__global__ void zero_f32_kernel(float* x, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

hipError_t zero_f32(float* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_f32_kernel, dim3(8192), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

// TT[i][j] = RkT[i][s + j] - sum_z P[z][j][i]   (i, j < b): the transpose of
// T = R[I,I] - Delta^T A[I^c,I], with R[I,I] read from the current residual columns.
__global__ void corr_diag_kernel(const double* rkt, int64_t ldr, int64_t s, const double* part,
                                 int splits, int64_t b, double* tt) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double g = 0.0;
    for (int z = 0; z < splits; ++z) g += part[z * n + j * b + i];
    tt[e] = rkt[i * ldr + s + j] - g;
  }
}

hipError_t corr_diag(const double* rkt, int64_t ldr, int64_t s, const double* part, int splits,
                     int64_t b, double* tt, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(corr_diag_kernel, dim3(grid), dim3(256), 0, st, rkt, ldr, s, part, splits,
                     b, tt);
  return hipGetLastError();
}

// H[s+i][s+j] += (X[i][j] + X[j][i]) / 2 and the same increment (rounded) into D.
__global__ void corr_apply_kernel(const double* x, int64_t b, double* H, int64_t ldh, float* D,
                                  int64_t ldd, int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    const double inc = 0.5 * (x[e] + x[j * b + i]);
    H[(s + i) * ldh + s + j] += inc;
    D[(s + i) * ldd + s + j] += (float)inc;
  }
}

hipError_t corr_apply(const double* x, int64_t b, double* H, int64_t ldh, float* D, int64_t ldd,
                      int64_t s, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(corr_apply_kernel, dim3(grid), dim3(256), 0, st, x, b, H, ldh, D, ldd, s);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace ibmi
