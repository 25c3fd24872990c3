// FP64 GEMM launches: residual (with optional store), sum of squares of a product, and the
// correction epilogue.
#include "gemm.h"

namespace ibmi {

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

hipError_t gemm_sumsq(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* red,
                      int64_t* n_red, hipStream_t st) {
  EpiArgs ea;
  ea.red = red;
  return launch_gemm<double, EPI_SUMSQ>(cfg, X, Y, M, N, K, 1, ea, st, n_red);
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

}  // namespace ibmi
