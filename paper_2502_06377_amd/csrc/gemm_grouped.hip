// Grouped (batched) FP64 GEMM launches.
#include "gemm.h"

namespace ibmi {

hipError_t gemm_grouped(GemmCfg cfg, int epi, const GemmTask* tasks, const int* tile_off,
                        int ntasks, int total_tiles, const int* active, bool vec, hipStream_t st) {
  if (ntasks <= 0 || total_tiles <= 0) return hipSuccess;
  switch (epi) {
    case EPI_STORE:
      return launch_grouped<double, EPI_STORE>(cfg, tasks, tile_off, ntasks, total_tiles, active,
                                               vec, st);
    case EPI_PANEL:
      return launch_grouped<double, EPI_PANEL>(cfg, tasks, tile_off, ntasks, total_tiles, active,
                                               vec, st);
    case EPI_PARTIAL:
      return launch_grouped<double, EPI_PARTIAL>(cfg, tasks, tile_off, ntasks, total_tiles,
                                                 active, vec, st);
    case EPI_RESID:
      return launch_grouped<double, EPI_RESID>(cfg, tasks, tile_off, ntasks, total_tiles, active,
                                               vec, st);
    default: return hipErrorInvalidValue;
  }
}

bool gemm_vec_ok(const GemmTask& t) {
  return vec_ok<double>(t.X, 2, t.M) && vec_ok<double>(t.Y, 2, t.N);
}

}  // namespace ibmi
