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

hipError_t gemm_partial(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, int splits,
                        double* out, hipStream_t st) {
  EpiArgs ea;
  ea.out = out;
  return launch_gemm<double, EPI_PARTIAL>(cfg, X, Y, M, N, K, splits, ea, st, nullptr);
}

}  // namespace ibmi
