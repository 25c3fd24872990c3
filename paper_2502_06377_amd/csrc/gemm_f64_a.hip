// FP64 GEMM launches: plain store, panel scatter into H, split-K partials; tile table.
#include "gemm.h"

namespace ibmi {

GemmDims gemm_dims(GemmCfg c) {
  switch (c) {
#define IBMI_DIMS(NAME, BM_, BN_, BK_, WM_, WN_) \
  case NAME:                                     \
    return {BM_, BN_, BK_};
    IBMI_GEMM_CONFIGS(IBMI_DIMS)
#undef IBMI_DIMS
    default: return {64, 64, 16};
  }
}

// True when every VEC-wide run of columns x, x+1, .. (x a multiple of VEC) of the operand is
// contiguous and 16-byte aligned in memory.
int64_t gemm_tiles(GemmCfg cfg, int64_t M, int64_t N) {
  const GemmDims d = gemm_dims(cfg);
  return ((M + d.bm - 1) / d.bm) * ((N + d.bn - 1) / d.bn);
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

size_t panel_sk_part_bytes(GemmCfg cfg) {
  const GemmDims d = gemm_dims(cfg);
  return (size_t)2 * kSkMaxWorkgroups * d.bm * d.bn * sizeof(double);
}

namespace {

// Launch with a stream-K tail for one configuration; *used = false (nothing launched) when the
// panel's tiles are no more than, or a multiple of, the resident workgroups (no tail to
// remove).
template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_sk(Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, EpiArgs ea, double* part,
                     bool vec, hipStream_t st, bool* used) {
  *used = false;
  constexpr int NT = 64 * WM * WN;
  auto kern = vec ? panel_sk_kernel<double, BM, BN, BK, WM, WN, 2>
                  : panel_sk_kernel<double, BM, BN, BK, WM, WN, 1>;
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
  if (e != hipSuccess) return e;
  const int G = std::min(cus * occ / 8 * 8, kSkMaxWorkgroups);
  const int mtc = (int)((M + BM - 1) / BM), ntc = (int)((N + BN - 1) / BN);
  const int64_t tiles = (int64_t)mtc * ntc;
  if (G < 8 || tiles <= G || tiles % G == 0 || K <= 0) return hipSuccess;
  const int nk = (int)((K + BK - 1) / BK);
  const int dp_rounds = (int)(tiles / G);
  const int64_t t0 = (int64_t)dp_rounds * G, tail = tiles - t0;
  const int64_t Q = (tail * nk + G - 1) / G;
  ea.red = part;
  hipLaunchKernelGGL(kern, dim3(G), dim3(NT), 0, st, X, Y, M, N, K, mtc, nk, dp_rounds, tail * nk,
                     Q, G / 8, ea);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((panel_fixup_kernel<BM, BN>), dim3((unsigned)tail), dim3(256), 0, st, part,
                     M, N, mtc, nk, t0, Q, ea);
  *used = true;
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_panel_sk(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* H,
                         int64_t ldh, int64_t s, IdxMap g, double* part, hipStream_t st) {
  EpiArgs ea;
  ea.out = H;
  ea.ldo = ldh;
  ea.s = s;
  ea.g = g;
  bool used = false;
  hipError_t e = hipSuccess;
  if (part) {
    const bool vec = vec_ok<double>(X, 2, M) && vec_ok<double>(Y, 2, N);
    switch (cfg) {  // the panel's small-tile configurations
      case GEMM_64x64:
        e = launch_sk<64, 64, 32, 2, 2>(X, Y, M, N, K, ea, part, vec, st, &used);
        break;
      case GEMM_64x64_K16:
        e = launch_sk<64, 64, 16, 2, 2>(X, Y, M, N, K, ea, part, vec, st, &used);
        break;
      default: break;
    }
  }
  if (e != hipSuccess || used) return e;
  return launch_gemm<double, EPI_PANEL>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

hipError_t gemm_partial(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, int splits,
                        double* out, hipStream_t st) {
  EpiArgs ea;
  ea.out = out;
  return launch_gemm<double, EPI_PARTIAL>(cfg, X, Y, M, N, K, splits, ea, st, nullptr);
}

}  // namespace ibmi
