// FP32 GEMM launch of the FP32 update form.
#include "gemm.h"

namespace ibmi {

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
  // Rows klim .. of Y are zero in the column tiles that stop at klim, so rounding klim up
  // to whole K stages adds only zeros and keeps the loop branch-free.
  const int64_t bk = gemm_dims(cfg).bk;
  ea.klim = std::min(K, (klim + bk - 1) / bk * bk);
  return launch_gemm<float, EPI_SUBFROM>(cfg, X, Y, M, N, K, 1, ea, st, nullptr);
}

}  // namespace ibmi
