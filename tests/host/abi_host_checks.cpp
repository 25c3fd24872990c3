// Host-only checks of the C ABI, built with AddressSanitizer and UBSan by
// tests/test_host_sanitizers.py: partitioner, workspace sizing and argument checks, none of
// which starts device work.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>
#include "ibmi.h"
static int fails = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)
int main() {
  // partition: sizes, edge cases, capacity handling
  for (int64_t p : {1, 2, 127, 128, 129, 576, 1000, 4096, 16384, 46400}) {
    for (int b : {1, 16, 128, 576}) {
      for (int ovl : {0, 1, 15, 64}) {
        if (ovl >= b) continue;
        int32_t n = -1;
        EXPECT(ibmi_partition(p, b, ovl, nullptr, 0, &n) == IBMI_OK && n >= 1);
        std::vector<int64_t> bo(2 * n + 2, -7);
        int32_t n2 = -1;
        EXPECT(ibmi_partition(p, b, ovl, bo.data(), n, &n2) == IBMI_OK && n2 == n);
        EXPECT(bo[2 * n] == -7 && bo[2 * n + 1] == -7);  // nothing written past capacity
        EXPECT(bo[0] == 0 && bo[2 * n - 1] == p);
        for (int k = 0; k < n; ++k) EXPECT(bo[2 * k] < bo[2 * k + 1]);
        if (n > 1) {
          int32_t n3 = -1;
          std::vector<int64_t> small(2, -7);
          (void)ibmi_partition(p, b, ovl, small.data(), 1, &n3);  // short buffer: at most 1 pair
        }
      }
    }
  }
  int32_t n = 0;
  EXPECT(ibmi_partition(0, 128, 0, nullptr, 0, &n) == IBMI_ERR_INVALID_ARG);
  EXPECT(ibmi_partition(100, 0, 0, nullptr, 0, &n) == IBMI_ERR_INVALID_ARG);
  EXPECT(ibmi_partition(100, 16, 16, nullptr, 0, &n) == IBMI_ERR_INVALID_ARG);
  EXPECT(ibmi_partition(100, 16, -1, nullptr, 0, &n) == IBMI_ERR_INVALID_ARG);
  // workspace sizes for every form and stop test, and invalid options
  for (int prec = 0; prec <= 3; ++prec)
    for (int stop = 0; stop <= 3; ++stop) {
      ibmi_options o{};
      o.p = 3000; o.block_rows = 576; o.overlap = 64; o.precision = (ibmi_precision)prec;
      o.init = IBMI_INIT_IDENTITY; o.stop = (ibmi_stop)stop; o.tol = 1e-10; o.lambda_min = 1e-3;
      o.max_sweeps = 10; o.stagnation_guard = 1;
      EXPECT(ibmi_workspace_bytes(&o) > 0);
    }
  ibmi_options bad{};
  bad.p = 100; bad.block_rows = 16; bad.tol = 0.0; bad.max_sweeps = 1;
  EXPECT(ibmi_workspace_bytes(&bad) == 0);
  EXPECT(ibmi_workspace_bytes(nullptr) == 0);
  // explicit bounds: gap, overlap order, out of range
  ibmi_options o{};
  o.p = 100; o.block_rows = 50; o.overlap = 0; o.tol = 1e-10; o.max_sweeps = 5;
  const int64_t gap[4] = {0, 40, 50, 100}, oob[4] = {0, 60, 50, 120}, ok[4] = {0, 60, 40, 100};
  o.bounds = gap; o.n_blocks = 2;
  EXPECT(ibmi_workspace_bytes(&o) == 0);
  o.bounds = oob;
  EXPECT(ibmi_workspace_bytes(&o) == 0);
  o.bounds = ok;
  EXPECT(ibmi_workspace_bytes(&o) > 0);
  // plan argument checks return before any device call
  o.bounds = nullptr; o.n_blocks = 0;
  const size_t need = ibmi_workspace_bytes(&o);
  ibmi_plan_t plan = nullptr;
  const double* fakeA = reinterpret_cast<const double*>(uintptr_t(1) << 40);
  void* fakeW = reinterpret_cast<void*>(uintptr_t(1) << 44);
  EXPECT(ibmi_plan(nullptr, &o, fakeA, 100, fakeW, need, nullptr) == IBMI_ERR_INVALID_ARG);
  EXPECT(ibmi_plan(&plan, &o, fakeA, 99, fakeW, need, nullptr) == IBMI_ERR_INVALID_ARG);
  EXPECT(ibmi_plan(&plan, &o, fakeA, 100, fakeW, need - 1, nullptr) == IBMI_ERR_OUT_OF_MEMORY);
  EXPECT(ibmi_plan(&plan, &o, fakeA, 100, (char*)fakeA + 800, need, nullptr) == IBMI_ERR_INVALID_ARG);
  EXPECT(plan == nullptr);
  for (int s = 0; s <= 6; ++s) EXPECT(ibmi_status_str((ibmi_status)s) != nullptr);
  // batched sizing and argument checks
  const int64_t ps[3] = {128, 300, 2048};
  ibmi_options bo{};
  bo.p = 0; bo.block_rows = 128; bo.overlap = 16; bo.tol = 1e-8; bo.max_sweeps = 500;
  EXPECT(ibmi_batch_workspace_bytes(3, ps, &bo) > 0);
  EXPECT(ibmi_batch_workspace_bytes(0, ps, &bo) == 0);
  std::printf(fails ? "host checks: %d failed\n" : "host checks: all passed\n", fails);
  return fails ? 1 : 0;
}
