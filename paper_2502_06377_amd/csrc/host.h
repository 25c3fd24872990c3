// Host-side helpers shared by the single-matrix and batched drivers of libibmi.
#pragma once
#include <stdint.h>

#include <vector>

#include "kernels.h"

namespace ibmi {

// The default sets (multi-block overlapping partition; end sets m+h rows, interior m+2h).
void default_partition(int64_t p, int64_t b, int64_t ovl, std::vector<int64_t>& s,
                       std::vector<int64_t>& e);

// Tile configurations of the batched form's grouped launches (autotuned or defaults).
void batch_tuning(GemmCfg* panel, GemmCfg* diag, GemmCfg* resid);

}  // namespace ibmi
