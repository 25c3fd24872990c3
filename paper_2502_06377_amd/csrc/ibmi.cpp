// Host side of libibmi: partitioner, plan (block factors), sweep driver and the C ABI
// declared in include/ibmi.h.  All device work goes through the kernels in kernels.hip.
#include "ibmi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host.h"
#include "kernels.h"

using ibmi::BlockDesc;
using ibmi::GemmCfg;
using ibmi::SplitCfg;
using ibmi::IdxMap;
using ibmi::Opnd;

namespace {

constexpr int64_t kMaxBlockRows = 1024;  // LDS panel and register-slot limits of the factor kernels
constexpr size_t kAlign = 256;

thread_local int32_t g_last_failed_block = -1;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

#define IBMI_HIP(call)                          \
  do {                                          \
    if ((call) != hipSuccess) return IBMI_ERR_HIP; \
  } while (0)

}  // namespace

// The partition reading documented in ibmi.h (ibmi_partition).
void ibmi::default_partition(int64_t p, int64_t b, int64_t ovl, std::vector<int64_t>& s,
                             std::vector<int64_t>& e) {
  s.clear();
  e.clear();
  if (p <= b) {
    s.push_back(0);
    e.push_back(p);
    return;
  }
  const int64_t m = b - ovl;
  int64_t k_sets = (p + m - 1) / m;
  std::vector<int64_t> cs, ce;
  for (int64_t k = 0; k < k_sets; ++k) {
    cs.push_back(k * m);
    ce.push_back(std::min((k + 1) * m, p));
  }
  if (k_sets > 1 && ce.back() - cs.back() < ovl) {
    ce[k_sets - 2] = ce.back();
    cs.pop_back();
    ce.pop_back();
    --k_sets;
  }
  const int64_t hl = ovl / 2, hr = ovl - ovl / 2;
  for (int64_t k = 0; k < k_sets; ++k) {
    s.push_back(std::max<int64_t>(0, cs[k] - hl));
    e.push_back(std::min(p, ce[k] + hr));
  }
}

namespace {
using ibmi::default_partition;

// Validated sets of a plan (partitioner or explicit bounds).
ibmi_status make_sets(const ibmi_options* o, std::vector<int64_t>& s, std::vector<int64_t>& e) {
  if (!o || o->p < 1) return IBMI_ERR_INVALID_ARG;
  const int64_t p = o->p;
  if (o->bounds) {
    if (o->n_blocks < 1) return IBMI_ERR_INVALID_ARG;
    s.assign(o->n_blocks, 0);
    e.assign(o->n_blocks, 0);
    for (int k = 0; k < o->n_blocks; ++k) {
      s[k] = o->bounds[2 * k];
      e[k] = o->bounds[2 * k + 1];
    }
  } else {
    if (o->block_rows < 1 || o->overlap < 0 || o->overlap >= o->block_rows)
      return IBMI_ERR_INVALID_ARG;
    default_partition(p, o->block_rows, o->overlap, s, e);
  }
  // sorted by start, non-empty, inside [0,p), covering, each within the size limit
  int64_t covered_to = 0;
  for (size_t k = 0; k < s.size(); ++k) {
    if (s[k] < 0 || e[k] > p || s[k] >= e[k]) return IBMI_ERR_INVALID_ARG;
    if (k > 0 && s[k] < s[k - 1]) return IBMI_ERR_INVALID_ARG;
    if (e[k] - s[k] > kMaxBlockRows) return IBMI_ERR_INVALID_ARG;
    if (s[k] > covered_to) return IBMI_ERR_INVALID_ARG;
    covered_to = std::max(covered_to, e[k]);
  }
  if (covered_to != p) return IBMI_ERR_INVALID_ARG;
  if (o->init == IBMI_INIT_BLOCKDIAG_INV) {
    for (size_t k = 1; k < s.size(); ++k)
      if (s[k] < e[k - 1]) return IBMI_ERR_INVALID_ARG;
  }
  return IBMI_OK;
}

ibmi_status check_options(const ibmi_options* o) {
  if (!o) return IBMI_ERR_INVALID_ARG;
  if (!(o->tol > 0.0) || o->max_sweeps < 1 || o->fixed_sweeps < 0) return IBMI_ERR_INVALID_ARG;
  if (o->precision < IBMI_PREC_FP64 || o->precision > IBMI_PREC_BF16X6_UPDATE)
    return IBMI_ERR_INVALID_ARG;
  if (o->init < IBMI_INIT_IDENTITY || o->init > IBMI_INIT_GIVEN) return IBMI_ERR_INVALID_ARG;
  if (o->stop < IBMI_STOP_FRO || o->stop > IBMI_STOP_PAPER) return IBMI_ERR_INVALID_ARG;
  if (o->stop == IBMI_STOP_REL_BOUND && !(o->lambda_min > 0.0)) return IBMI_ERR_INVALID_ARG;
  return IBMI_OK;
}

GemmCfg env_cfg(const char* name, GemmCfg dflt) {
  const char* v = std::getenv(name);
  if (!v) return dflt;
  const int i = std::atoi(v);
  return (i >= 0 && i < ibmi::GEMM_CFG_COUNT) ? (GemmCfg)i : dflt;
}

// Defaults measured on MI355X at p = 16384 (sweep of all configurations): the panel 96x64
// tiles (six row tiles cover a 576-row set; 0.76 of the FP64 peak against 0.71 for 64x64),
// the diagonal product 64x64 tiles with many resident waves, the square residual the 8-wave
// 128x128 tile, the FP32 update 96x128 tiles (64x64 below p = 8192), the split-bfloat16
// update 8-wave 192x256 tiles (two terms; with three terms they would not fit in LDS) or
// 6-wave 192x128 tiles (three terms), K cut into chunks of 2048 (the three row tiles of a
// 576-row set times eight chunks fill the chip where whole-K tiles leave it half idle).
struct Tuning {
  GemmCfg panel = ibmi::GEMM_64x64_K16, diag = ibmi::GEMM_64x64_K16,
          resid = ibmi::GEMM_128x128_W8, plan = ibmi::GEMM_64x64_K16, upd32 = ibmi::GEMM_64x64,
          small = ibmi::GEMM_64x64_K16;
  int diag_splits = 0;  // 0 = automatic
  SplitCfg split = ibmi::SPLIT_192x256;  // split-bfloat16 update product, two terms
  SplitCfg split6 = ibmi::SPLIT_192x128; // the same with three terms
  int64_t split_kchunk = 2048;           // their K chunk (0: whole K per tile)
};

Tuning tuning_for(int64_t p) {
  Tuning t;
  if (p < 2048) {  // small matrices: more, smaller tiles
    t.resid = ibmi::GEMM_64x64_K16;
  }
  if (p >= 8192) {  // enough column tiles to fill the chip with the larger tiles
    t.panel = ibmi::GEMM_96x64_K16;
    t.upd32 = ibmi::GEMM_96x128;
  }
  t.upd32 = env_cfg("IBMI_CFG_UPD32", t.upd32);
  t.panel = env_cfg("IBMI_CFG_PANEL", t.panel);
  t.diag = env_cfg("IBMI_CFG_DIAG", t.diag);
  t.resid = env_cfg("IBMI_CFG_RESID", t.resid);
  t.plan = env_cfg("IBMI_CFG_PLAN", t.plan);
  if (const char* v = std::getenv("IBMI_DIAG_SPLITS")) t.diag_splits = std::max(1, std::atoi(v));
  if (const char* v = std::getenv("IBMI_CFG_SPLIT")) {
    const int i = std::atoi(v);
    if (i >= 0 && i < ibmi::SPLIT_CFG_COUNT) t.split = (SplitCfg)i;
  }
  if (const char* v = std::getenv("IBMI_CFG_SPLIT6")) {
    const int i = std::atoi(v);
    if (i >= 0 && i < ibmi::SPLIT_CFG_COUNT) t.split6 = (SplitCfg)i;
  }
  if (const char* v = std::getenv("IBMI_SPLIT_KCHUNK")) t.split_kchunk = std::max(0, std::atoi(v));
  return t;
}

}  // namespace

// Default tile configurations of the batched form's grouped launches (small matrices: small
// tiles, many resident waves); IBMI_CFG_* environment overrides apply as for single plans.
void ibmi::batch_tuning(GemmCfg* panel, GemmCfg* diag, GemmCfg* resid) {
  *panel = env_cfg("IBMI_CFG_PANEL", ibmi::GEMM_64x64_K16);
  *diag = env_cfg("IBMI_CFG_DIAG", ibmi::GEMM_64x64_K16);
  *resid = env_cfg("IBMI_CFG_RESID", ibmi::GEMM_64x64_K16);
}

namespace {

int diag_splits_for(int64_t b, int64_t c, GemmCfg cfg, int forced) {
  if (c <= 0) return 1;
  if (forced > 0) return (int)std::min<int64_t>(forced, std::max<int64_t>(1, c / 64));
  const int64_t tiles = ibmi::gemm_tiles(cfg, b, b);
  int64_t want = (512 + tiles - 1) / tiles;
  want = std::min<int64_t>(want, std::max<int64_t>(1, c / 512));
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, 32));
}

// Workspace layout (offsets in bytes from the workspace base).
struct Layout {
  size_t desc = 0, fac = 0, wt = 0, part = 0, red = 0, red2 = 0, scal = 0, status = 0, total = 0;
  // Correction (FP32 / split-bfloat16 update) forms only (zero size otherwise)
  size_t a32 = 0, dmat = 0, rt = 0, rkt = 0, delta = 0, tt = 0, spart = 0;
  int64_t ld32 = 0;  // row stride of the FP32 copies of A and D (multiple of 4)
  std::vector<BlockDesc> blocks;
  std::vector<int64_t> wt_off;  // doubles, relative to wt
  int64_t b_max = 0;
  int splits = 1;
  int64_t red_len = 0;
};

Layout make_layout(const ibmi_options* o, const std::vector<int64_t>& s,
                   const std::vector<int64_t>& e, const Tuning& t) {
  Layout L;
  const int64_t p = o->p;
  const int K = (int)s.size();
  int64_t fac = 0, wt = 0;
  for (int k = 0; k < K; ++k) {
    const int64_t b = e[k] - s[k], c = p - b;
    BlockDesc d{};
    d.s = s[k];
    d.b = b;
    d.l_off = fac;
    d.linv_off = fac + b * b;
    d.ainv_off = fac + 2 * b * b;
    fac += 3 * b * b;
    L.blocks.push_back(d);
    L.wt_off.push_back(wt);
    wt += c * b;
    L.b_max = std::max(L.b_max, b);
    L.splits = std::max(L.splits, diag_splits_for(b, c, t.diag, t.diag_splits));
  }
  L.red_len = std::max<int64_t>(ibmi::gemm_tiles(t.resid, p, p), 1);
  size_t off = 0;
  L.desc = off;
  off = align_up(off + K * sizeof(BlockDesc));
  L.fac = off;
  off = align_up(off + (size_t)fac * 8);
  L.wt = off;
  off = align_up(off + (size_t)wt * 8);
  L.part = off;
  off = align_up(off + (size_t)L.splits * L.b_max * L.b_max * 8);
  L.red = off;
  off = align_up(off + (size_t)L.red_len * 8);
  L.red2 = off;
  off = align_up(off + (size_t)1024 * 8);
  L.scal = off;
  off = align_up(off + 8 * 8);
  L.status = off;
  off = align_up(off + 4 * sizeof(int));
  if (o->precision != IBMI_PREC_FP64) {
    L.ld32 = (p + 3) / 4 * 4;
    const size_t pp = (size_t)p * L.ld32;
    const int64_t c_max = p - [&] {
      int64_t bmin = p;
      for (const auto& d : L.blocks) bmin = std::min(bmin, d.b);
      return bmin;
    }();
    L.a32 = off;
    off = align_up(off + pp * 4);
    L.dmat = off;
    off = align_up(off + pp * 4);
    L.rt = off;
    off = align_up(off + pp * 8);
    L.rkt = off;
    off = align_up(off + (size_t)L.b_max * p * 8);
    L.delta = off;
    off = align_up(off + (size_t)std::max<int64_t>(c_max, 1) * L.b_max * 8);
    L.tt = off;
    off = align_up(off + (size_t)L.b_max * L.b_max * 8);
    if (o->precision != IBMI_PREC_FP32_UPDATE) {
      const int64_t chunks = ibmi::split_max_chunks(p, t.split_kchunk);
      L.spart = off;
      if (chunks > 1) off = align_up(off + (size_t)chunks * L.b_max * p * 4);
    }
  } else if (o->stop == IBMI_STOP_REL_HR) {
    L.rt = off;  // R = I - A H of the last sweep, for the H R bound
    off = align_up(off + (size_t)p * p * 8);
  }
  L.total = off;
  return L;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

// HIP event pairs bracketing launches of one category, collected after a stream sync.
struct Timer {
  std::vector<hipEvent_t> free_ev;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double ms = 0.0, flops = 0.0;
  int64_t launches = 0;
  hipEvent_t get() {
    if (!free_ev.empty()) {
      hipEvent_t e = free_ev.back();
      free_ev.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void collect() {
    for (auto& pr : pending) {
      float t = 0.f;
      if (hipEventSynchronize(pr.second) == hipSuccess &&
          hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess)
        ms += t;
      free_ev.push_back(pr.first);
      free_ev.push_back(pr.second);
    }
    pending.clear();
  }
  ~Timer() {
    collect();
    for (hipEvent_t e : free_ev) (void)hipEventDestroy(e);
  }
};

struct ibmi_plan_s {
  ibmi_options o;
  ibmi_progress_fn progress = nullptr;
  void* progress_user = nullptr;
  bool profiling = false;
  Timer timers[3];
  std::vector<int64_t> s, e;
  int64_t p = 0;
  const double* A = nullptr;
  int64_t lda = 0;
  hipStream_t st = nullptr;
  char* work = nullptr;
  size_t work_bytes = 0;
  Layout L;
  Tuning t;
  double* fac() const { return (double*)(work + L.fac); }
  double* wt(int k) const { return (double*)(work + L.wt) + L.wt_off[k]; }
  double* ainv(int k) const { return fac() + L.blocks[k].ainv_off; }
  double* part() const { return (double*)(work + L.part); }
  double* red() const { return (double*)(work + L.red); }
  double* red2() const { return (double*)(work + L.red2); }
  double* scal() const { return (double*)(work + L.scal); }
  int* status() const { return (int*)(work + L.status); }
  BlockDesc* desc() const { return (BlockDesc*)(work + L.desc); }
  bool mixed() const { return o.precision != IBMI_PREC_FP64; }
  // bfloat16 terms per operand of the update product (0: plain FP32 products)
  int split_terms() const {
    return o.precision == IBMI_PREC_BF16X3_UPDATE ? 2
           : o.precision == IBMI_PREC_BF16X6_UPDATE ? 3 : 0;
  }
  float* spart() const { return (float*)(work + L.spart); }
  float* a32() const { return (float*)(work + L.a32); }
  float* dmat() const { return (float*)(work + L.dmat); }
  double* rt() const { return (double*)(work + L.rt); }
  double* rkt() const { return (double*)(work + L.rkt); }
  double* delta() const { return (double*)(work + L.delta); }
  double* tt() const { return (double*)(work + L.tt); }
};

extern "C" {

const char* ibmi_status_str(ibmi_status s) {
  switch (s) {
    case IBMI_OK: return "IBMI_OK";
    case IBMI_ERR_INVALID_ARG: return "IBMI_ERR_INVALID_ARG";
    case IBMI_ERR_NOT_SPD: return "IBMI_ERR_NOT_SPD";
    case IBMI_ERR_OUT_OF_MEMORY: return "IBMI_ERR_OUT_OF_MEMORY";
    case IBMI_ERR_HIP: return "IBMI_ERR_HIP";
    case IBMI_ERR_NONFINITE: return "IBMI_ERR_NONFINITE";
  }
  return "IBMI_UNKNOWN_STATUS";
}

ibmi_status ibmi_partition(int64_t p, int32_t block_rows, int32_t overlap, int64_t* bounds_out,
                           int32_t capacity, int32_t* n_out) {
  if (p < 1 || block_rows < 1 || overlap < 0 || overlap >= block_rows || !n_out)
    return IBMI_ERR_INVALID_ARG;
  std::vector<int64_t> s, e;
  default_partition(p, block_rows, overlap, s, e);
  *n_out = (int32_t)s.size();
  if (bounds_out) {
    const int n = std::min<int>(capacity, (int)s.size());
    for (int k = 0; k < n; ++k) {
      bounds_out[2 * k] = s[k];
      bounds_out[2 * k + 1] = e[k];
    }
  }
  return IBMI_OK;
}

size_t ibmi_workspace_bytes(const ibmi_options* opts) {
  if (check_options(opts) != IBMI_OK) return 0;
  std::vector<int64_t> s, e;
  if (make_sets(opts, s, e) != IBMI_OK) return 0;
  return make_layout(opts, s, e, tuning_for(opts->p)).total;
}

int32_t ibmi_plan_failed_block(void) { return g_last_failed_block; }

ibmi_status ibmi_plan(ibmi_plan_t* out, const ibmi_options* opts, const double* dA, int64_t lda,
                      void* dWork, size_t work_bytes, void* stream) {
  g_last_failed_block = -1;
  if (!out || !dA || !dWork) return IBMI_ERR_INVALID_ARG;
  ibmi_status rc = check_options(opts);
  if (rc != IBMI_OK) return rc;
  if (lda < opts->p || ((uintptr_t)dWork % kAlign) != 0) return IBMI_ERR_INVALID_ARG;
  auto* P = new ibmi_plan_s();
  P->o = *opts;
  P->o.bounds = nullptr;  // the plan keeps its own copy of the sets
  P->p = opts->p;
  P->A = dA;
  P->lda = lda;
  P->st = (hipStream_t)stream;
  P->t = tuning_for(P->p);
  rc = make_sets(opts, P->s, P->e);
  if (rc != IBMI_OK) {
    delete P;
    return rc;
  }
  P->L = make_layout(opts, P->s, P->e, P->t);
  if (work_bytes < P->L.total) {
    delete P;
    return IBMI_ERR_OUT_OF_MEMORY;
  }
  const size_t a_bytes = (size_t)((P->p - 1) * lda + P->p) * 8;
  if (ranges_overlap(dA, a_bytes, dWork, P->L.total)) {
    delete P;
    return IBMI_ERR_INVALID_ARG;
  }
  P->work = (char*)dWork;
  P->work_bytes = work_bytes;
  const int K = (int)P->s.size();
  hipStream_t st = P->st;
  auto fail = [&](ibmi_status r) {
    delete P;
    return r;
  };
  if (hipMemcpyAsync(P->desc(), P->L.blocks.data(), K * sizeof(BlockDesc), hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  if (ibmi::fill_int(P->status(), INT_MAX, 1, st) != hipSuccess) return fail(IBMI_ERR_HIP);
  if (ibmi::chol_factor(P->desc(), K, P->L.b_max, P->A, P->lda, P->fac(), P->status(), st) !=
      hipSuccess)
    return fail(IBMI_ERR_HIP);
  int status = INT_MAX;
  if (hipMemcpyAsync(&status, P->status(), sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  if (status != INT_MAX) {
    g_last_failed_block = status;
    return fail(IBMI_ERR_NOT_SPD);
  }
  if (ibmi::chol_linv(P->desc(), K, P->L.b_max, P->fac(), st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  for (int k = 0; k < K; ++k) {
    const BlockDesc& d = P->L.blocks[k];
    const int64_t b = d.b, c = P->p - b;
    double* linv = P->fac() + d.linv_off;
    double* tmp = P->fac() + d.l_off;  // the factor L is no longer needed
    Opnd Xl{linv, b, IdxMap{}, IdxMap{}};
    if (ibmi::gemm_store(P->t.plan, Xl, Xl, b, b, b, tmp, b, st) != hipSuccess)
      return fail(IBMI_ERR_HIP);
    if (ibmi::symmetrize_block(tmp, P->ainv(k), b, st) != hipSuccess) return fail(IBMI_ERR_HIP);
    if (c > 0) {
      const IdxMap g{0, d.s, b};
      Opnd Xa{P->A, P->lda, IdxMap{d.s, INT64_MAX, 0}, g};
      Opnd Yi{P->ainv(k), b, IdxMap{}, IdxMap{}};
      if (ibmi::gemm_store(P->t.plan, Xa, Yi, c, b, b, P->wt(k), b, st) != hipSuccess)
        return fail(IBMI_ERR_HIP);
    }
  }
  if (P->mixed() && ibmi::to_f32(P->A, P->lda, P->a32(), P->L.ld32, P->p, st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(IBMI_ERR_HIP);
  *out = P;
  return IBMI_OK;
}

ibmi_status ibmi_plan_blocks(ibmi_plan_t plan, int32_t* n_blocks, int64_t* bounds) {
  if (!plan || !n_blocks) return IBMI_ERR_INVALID_ARG;
  *n_blocks = (int32_t)plan->s.size();
  if (bounds)
    for (size_t k = 0; k < plan->s.size(); ++k) {
      bounds[2 * k] = plan->s[k];
      bounds[2 * k + 1] = plan->e[k];
    }
  return IBMI_OK;
}

static ibmi_status check_h(ibmi_plan_t plan, const double* dH, int64_t ldh) {
  if (!plan || !dH || ldh < plan->p) return IBMI_ERR_INVALID_ARG;
  const size_t h_bytes = (size_t)((plan->p - 1) * ldh + plan->p) * 8;
  const size_t a_bytes = (size_t)((plan->p - 1) * plan->lda + plan->p) * 8;
  if (ranges_overlap(dH, h_bytes, plan->A, a_bytes) ||
      ranges_overlap(dH, h_bytes, plan->work, plan->L.total))
    return IBMI_ERR_INVALID_ARG;
  return IBMI_OK;
}

// Starts an event-bracketed region of category cat when profiling; returns the end event.
static hipEvent_t prof_begin(ibmi_plan_t P, int cat) {
  if (!P->profiling) return nullptr;
  Timer& t = P->timers[cat];
  hipEvent_t a = t.get(), b = t.get();
  if (!a || !b) return nullptr;
  (void)hipEventRecord(a, P->st);
  t.pending.push_back({a, b});
  return b;
}
static void prof_end(ibmi_plan_t P, int cat, hipEvent_t end, double flops) {
  if (!end) return;
  (void)hipEventRecord(end, P->st);
  P->timers[cat].launches += 1;
  P->timers[cat].flops += flops;
}

static ibmi_status block_step(ibmi_plan_t P, double* dH, int64_t ldh, int k) {
  const BlockDesc& d = P->L.blocks[k];
  const int64_t s = d.s, b = d.b, c = P->p - b;
  hipStream_t st = P->st;
  if (c == 0) {
    IBMI_HIP(ibmi::copy_block(P->ainv(k), b, dH, ldh, s, st));
    return IBMI_OK;
  }
  const IdxMap g{0, s, b};
  Opnd Xw{P->wt(k), b, IdxMap{}, IdxMap{}};
  Opnd Yp{dH, ldh, g, g};
  hipEvent_t ev = prof_begin(P, 0);
  IBMI_HIP(ibmi::gemm_panel(P->t.panel, Xw, Yp, b, c, c, dH, ldh, s, g, st));
  prof_end(P, 0, ev, 2.0 * b * (double)c * c);
  const int splits = diag_splits_for(b, c, P->t.diag, P->t.diag_splits);
  Opnd Yd{dH, ldh, g, IdxMap{s, INT64_MAX, 0}};
  ev = prof_begin(P, 1);
  IBMI_HIP(ibmi::gemm_partial(P->t.diag, Xw, Yd, b, b, c, splits, P->part(), st));
  IBMI_HIP(ibmi::diag_finalize(P->ainv(k), P->part(), splits, b, dH, ldh, s, st));
  prof_end(P, 1, ev, 2.0 * (double)b * b * c);
  return IBMI_OK;
}

static ibmi_status residual_sq(ibmi_plan_t P, const double* dH, int64_t ldh, bool want_h,
                               double* res_sq, double* h_sq, double* store);

// One set of a low-precision update (correction) form.  On entry rt holds R_s^T = I - A H_s
// for the H at the start of the sweep and dmat holds D = H - H_s in FP32; u is the end of the
// union of the sets already updated in this sweep (D vanishes outside rows/columns [0,u)).
//   RkT   = R_s^T[I,:] - A[:,I]^T D       (FP32 or split-bfloat16 matrix cores, FP32 sums)
//   Delta = R[I^c,I] A_I^{-1}             H[I^c,I] += Delta, mirrored; D likewise
//   T     = R[I,I] - Delta^T A[I^c,I]     (split-K, fixed-order sum)
//   H[I,I] += sym(T A_I^{-1});  D[I,I] likewise
static ibmi_status block_step_mixed(ibmi_plan_t P, double* dH, int64_t ldh, int k, int64_t u) {
  const BlockDesc& d = P->L.blocks[k];
  const int64_t s = d.s, b = d.b, c = P->p - b, p = P->p;
  hipStream_t st = P->st;
  if (c == 0) {
    IBMI_HIP(ibmi::copy_block(P->ainv(k), b, dH, ldh, s, st));
    return IBMI_OK;
  }
  const IdxMap g{0, s, b};
  hipEvent_t ev = prof_begin(P, 0);
  const int64_t ld32 = P->L.ld32;
  if (const int terms = P->split_terms()) {
    // A and D are symmetric: rows s.. of A and the rows of D are the operands.
    IBMI_HIP(ibmi::gemm_split_subfrom(terms == 2 ? P->t.split : P->t.split6, terms, P->a32(),
                                      ld32, s, P->dmat(), ld32, b,
                                      p, p, u, u, P->t.split_kchunk, P->rt(), p, s, P->rkt(), p,
                                      P->spart(), st));
  } else {
    Opnd Xa32{(const double*)P->a32(), ld32, IdxMap{}, IdxMap{s, INT64_MAX, 0}};
    Opnd Yd32{(const double*)P->dmat(), ld32, IdxMap{}, IdxMap{}};
    IBMI_HIP(ibmi::gemm_f32_subfrom(P->t.upd32, Xa32, Yd32, b, p, p, u, u, P->rt(), p, s,
                                    P->rkt(), p, st));
  }
  prof_end(P, 0, ev, 2.0 * (double)b * ((double)u * p + (double)(p - u) * u));
  ev = prof_begin(P, 1);
  Opnd Xr{P->rkt(), p, IdxMap{}, g};
  Opnd Yi{P->ainv(k), b, IdxMap{}, IdxMap{}};
  IBMI_HIP(ibmi::gemm_corr(P->t.plan, Xr, Yi, c, b, b, P->delta(), b, dH, ldh, P->dmat(), ld32, s,
                           g, st));
  const int splits = diag_splits_for(b, c, P->t.diag, P->t.diag_splits);
  Opnd Xd{P->delta(), b, IdxMap{}, IdxMap{}};
  Opnd Ya{P->A, P->lda, g, IdxMap{s, INT64_MAX, 0}};
  IBMI_HIP(ibmi::gemm_partial(P->t.diag, Xd, Ya, b, b, c, splits, P->part(), st));
  IBMI_HIP(ibmi::corr_diag(P->rkt(), p, s, P->part(), splits, b, P->tt(), st));
  Opnd Xt{P->tt(), b, IdxMap{}, IdxMap{}};
  // (R[I,I] - Delta^T A[I^c,I]) A_I^{-1}, split over K like the diagonal product (the split
  // buffer is free again once corr_diag has read it): 81 tiles alone leave most CUs idle.
  const int s2 = std::min<int>(P->L.splits, (int)std::max<int64_t>(1, b / 64));
  IBMI_HIP(ibmi::gemm_partial(P->t.small, Xt, Yi, b, b, b, s2, P->part(), st));
  IBMI_HIP(ibmi::corr_apply(P->part(), s2, b, dH, ldh, P->dmat(), ld32, s, st));
  prof_end(P, 1, ev, 4.0 * (double)b * b * c + 2.0 * (double)b * b * b);
  return IBMI_OK;
}

// One full sweep of the plan's form followed by the residual; restart recomputes the
// starting residual of the low-precision update forms from H.
static ibmi_status sweep_once(ibmi_plan_t P, double* dH, int64_t ldh, bool restart, bool want_h,
                              double* res_sq, double* h_sq) {
  const int K = (int)P->s.size();
  if (!P->mixed()) {
    for (int k = 0; k < K; ++k) {
      ibmi_status rc = block_step(P, dH, ldh, k);
      if (rc != IBMI_OK) return rc;
    }
    return residual_sq(P, dH, ldh, want_h, res_sq, h_sq,
                       P->o.stop == IBMI_STOP_REL_HR ? P->rt() : nullptr);
  }
  const int64_t p = P->p;
  if (restart) {
    double ignore = 0.0;
    ibmi_status rc = residual_sq(P, dH, ldh, false, &ignore, nullptr, P->rt());
    if (rc != IBMI_OK) return rc;
  }
  IBMI_HIP(ibmi::zero_f32(P->dmat(), p * P->L.ld32, P->st));
  int64_t u = 0;
  for (int k = 0; k < K; ++k) {
    ibmi_status rc = block_step_mixed(P, dH, ldh, k, u);
    if (rc != IBMI_OK) return rc;
    u = std::max(u, P->e[k]);
  }
  return residual_sq(P, dH, ldh, want_h, res_sq, h_sq, P->rt());
}

ibmi_status ibmi_sweep(ibmi_plan_t plan, double* dH, int64_t ldh, int32_t restart,
                       double* residual) {
  ibmi_status rc = check_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  double r2 = 0.0;
  rc = sweep_once(plan, dH, ldh, restart != 0, false, &r2, nullptr);
  if (rc != IBMI_OK) return rc;
  if (residual) *residual = std::sqrt(r2);
  return std::isfinite(r2) ? IBMI_OK : IBMI_ERR_NONFINITE;
}

ibmi_status ibmi_block_step(ibmi_plan_t plan, double* dH, int64_t ldh, int32_t k) {
  ibmi_status rc = check_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  if (k < 0 || k >= (int32_t)plan->s.size()) return IBMI_ERR_INVALID_ARG;
  return block_step(plan, dH, ldh, k);
}

ibmi_status ibmi_init_h(ibmi_plan_t plan, double* dH, int64_t ldh) {
  ibmi_status rc = check_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  if (plan->o.init == IBMI_INIT_IDENTITY) {
    IBMI_HIP(ibmi::fill_identity(dH, ldh, plan->p, 1.0, plan->st));
  } else if (plan->o.init == IBMI_INIT_BLOCKDIAG_INV) {
    IBMI_HIP(ibmi::fill_identity(dH, ldh, plan->p, 0.0, plan->st));
    for (size_t k = 0; k < plan->s.size(); ++k)
      IBMI_HIP(ibmi::copy_block(plan->ainv((int)k), plan->L.blocks[k].b, dH, ldh, plan->s[k],
                                plan->st));
  }
  return IBMI_OK;
}

// Enqueue ||I - A H||_F^2 (scal[0]) and, if wanted, ||H||_F^2 (scal[1]); then read both.
static ibmi_status residual_sq(ibmi_plan_t P, const double* dH, int64_t ldh, bool want_h,
                               double* res_sq, double* h_sq, double* store) {
  hipStream_t st = P->st;
  Opnd Xa{P->A, P->lda, IdxMap{}, IdxMap{}};
  Opnd Yh{dH, ldh, IdxMap{}, IdxMap{}};
  int64_t n_red = 0;
  hipEvent_t ev = prof_begin(P, 2);
  IBMI_HIP(ibmi::gemm_resid(P->t.resid, Xa, Yh, P->p, P->p, P->p, P->red(), &n_red, store,
                            P->p, st));
  IBMI_HIP(ibmi::reduce_sum(P->red(), n_red, P->scal(), st));
  prof_end(P, 2, ev, 2.0 * (double)P->p * P->p * P->p);
  if (want_h) {
    int64_t n2 = 0;
    IBMI_HIP(ibmi::sumsq(dH, ldh, P->p, P->red2(), &n2, st));
    IBMI_HIP(ibmi::reduce_sum(P->red2(), n2, P->scal() + 1, st));
  }
  double host[2] = {0.0, 0.0};
  IBMI_HIP(hipMemcpyAsync(host, P->scal(), sizeof(host), hipMemcpyDeviceToHost, st));
  IBMI_HIP(hipStreamSynchronize(st));
  if (P->profiling)
    for (Timer& t : P->timers) t.collect();
  *res_sq = host[0];
  if (h_sq) *h_sq = host[1];
  return IBMI_OK;
}

// ||(H A)[I_K, I_K^c]||_F^2 for the last set: rows s.. of H (H symmetric, so the product's
// row operand is H's columns s..) times A's columns on the two-segment complement.
static ibmi_status paper_sq(ibmi_plan_t P, const double* dH, int64_t ldh, double* out) {
  hipStream_t st = P->st;
  const int K = (int)P->s.size();
  const BlockDesc& d = P->L.blocks[K - 1];
  const int64_t c = P->p - d.b;
  if (c == 0) {
    *out = 0.0;
    return IBMI_OK;
  }
  Opnd Xh{dH, ldh, IdxMap{}, IdxMap{d.s, INT64_MAX, 0}};
  Opnd Ya{P->A, P->lda, IdxMap{}, IdxMap{0, d.s, d.b}};
  int64_t n_red = 0;
  IBMI_HIP(ibmi::gemm_sumsq(P->t.resid, Xh, Ya, d.b, c, P->p, P->red(), &n_red, st));
  IBMI_HIP(ibmi::reduce_sum(P->red(), n_red, P->scal() + 3, st));
  IBMI_HIP(hipMemcpyAsync(out, P->scal() + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  IBMI_HIP(hipStreamSynchronize(st));
  return IBMI_OK;
}

// ||H R||_F^2 with R = I - A H as stored by the last residual evaluation (H symmetric, so
// the product's row operand H^T is H itself).
static ibmi_status hr_sq(ibmi_plan_t P, const double* dH, int64_t ldh, double* out) {
  hipStream_t st = P->st;
  Opnd Xh{dH, ldh, IdxMap{}, IdxMap{}};
  Opnd Yr{P->rt(), P->p, IdxMap{}, IdxMap{}};
  int64_t n_red = 0;
  IBMI_HIP(ibmi::gemm_sumsq(P->t.resid, Xh, Yr, P->p, P->p, P->p, P->red(), &n_red, st));
  IBMI_HIP(ibmi::reduce_sum(P->red(), n_red, P->scal() + 2, st));
  IBMI_HIP(hipMemcpyAsync(out, P->scal() + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  IBMI_HIP(hipStreamSynchronize(st));
  return IBMI_OK;
}

ibmi_status ibmi_residual(ibmi_plan_t plan, const double* dH, int64_t ldh, double* out) {
  ibmi_status rc = check_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  if (!out) return IBMI_ERR_INVALID_ARG;
  double r2 = 0.0;
  rc = residual_sq(plan, dH, ldh, false, &r2, nullptr, nullptr);
  if (rc != IBMI_OK) return rc;
  *out = std::sqrt(r2);
  return IBMI_OK;
}

ibmi_status ibmi_solve(ibmi_plan_t plan, double* dH, int64_t ldh, ibmi_info* info,
                       double* history) {
  ibmi_status rc = check_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  if (!info) return IBMI_ERR_INVALID_ARG;
  const ibmi_options& o = plan->o;
  *info = ibmi_info{0, 0, -1, 0, 0.0, 0.0, 0, 0};
  rc = ibmi_init_h(plan, dH, ldh);
  if (rc != IBMI_OK) return rc;
  const int limit = o.fixed_sweeps > 0 ? o.fixed_sweeps : o.max_sweeps;
  const bool want_h = o.stop != IBMI_STOP_FRO;
  double best = INFINITY;
  int since_best = 0;
  double ratio = -1.0, rho_eval = 0.0;  // REL_HR: last bound / ||R||_F, and that ||R||_F
  while (true) {
    double r2 = 0.0, h2 = 0.0;
    rc = sweep_once(plan, dH, ldh, info->sweeps == 0, want_h, &r2, &h2);
    if (rc != IBMI_OK) return rc;
    info->sweeps += 1;
    const double rho = std::sqrt(r2);
    info->residual = rho;
    if (!std::isfinite(rho)) return IBMI_ERR_NONFINITE;
    if (history) history[info->sweeps - 1] = rho;
    double sv = rho;
    if (o.stop == IBMI_STOP_REL_BOUND) {
      sv = rho / (o.lambda_min * std::sqrt(h2));
    } else if (o.stop == IBMI_STOP_PAPER) {
      double e2 = 0.0;
      rc = paper_sq(plan, dH, ldh, &e2);
      if (rc != IBMI_OK) return rc;
      sv = std::sqrt(e2);
    } else if (o.stop == IBMI_STOP_REL_HR) {
      const bool last = o.fixed_sweeps > 0 && info->sweeps >= limit;
      const bool due = rho < 1.0 && (ratio < 0.0 || ratio * rho < o.tol || rho < 0.1 * rho_eval);
      if (due || last) {
        sv = INFINITY;
        if (rho < 1.0) {
          double hr2 = 0.0;
          rc = hr_sq(plan, dH, ldh, &hr2);
          if (rc != IBMI_OK) return rc;
          const double x = std::sqrt(hr2) / ((1.0 - rho) * std::sqrt(h2));
          if (x < 1.0) sv = x / (1.0 - x);
        }
        ratio = rho > 0.0 ? sv / rho : 0.0;
        rho_eval = rho;
        info->evaluations += 1;
      } else {
        sv = ratio >= 0.0 ? ratio * rho : INFINITY;
      }
    }
    info->stop_value = sv;
    // Stagnation guard, in the units of the stop test.
    if (sv < 0.99 * best) {
      best = sv;
      since_best = 0;
    } else {
      ++since_best;
    }
    if (plan->progress && plan->progress(info->sweeps, rho, sv, plan->progress_user) != 0) {
      info->cancelled = 1;
      info->converged = o.fixed_sweeps > 0 ? 0 : (sv < o.tol);
      break;
    }
    if (o.fixed_sweeps > 0) {
      if (info->sweeps >= limit) {
        info->converged = sv < o.tol;
        break;
      }
      continue;
    }
    if (sv < o.tol) {
      info->converged = 1;
      break;
    }
    if (info->sweeps >= limit) break;
    if (o.stagnation_guard && best < 100.0 * o.tol && since_best >= ibmi::kGuardSweeps) {
      info->floor_limited = 1;
      break;
    }
  }
  return IBMI_OK;
}

ibmi_status ibmi_set_progress(ibmi_plan_t plan, ibmi_progress_fn fn, void* user) {
  if (!plan) return IBMI_ERR_INVALID_ARG;
  plan->progress = fn;
  plan->progress_user = user;
  return IBMI_OK;
}

ibmi_status ibmi_set_profiling(ibmi_plan_t plan, int32_t on) {
  if (!plan) return IBMI_ERR_INVALID_ARG;
  plan->profiling = on != 0;
  return IBMI_OK;
}

ibmi_status ibmi_kernel_times(ibmi_plan_t plan, double* ms, int64_t* launches, double* flops) {
  if (!plan) return IBMI_ERR_INVALID_ARG;
  IBMI_HIP(hipStreamSynchronize(plan->st));
  for (int i = 0; i < 3; ++i) {
    Timer& t = plan->timers[i];
    t.collect();
    if (ms) ms[i] = t.ms;
    if (launches) launches[i] = t.launches;
    if (flops) flops[i] = t.flops;
    t.ms = 0.0;
    t.flops = 0.0;
    t.launches = 0;
  }
  return IBMI_OK;
}

ibmi_status ibmi_plan_destroy(ibmi_plan_t plan) {
  if (!plan) return IBMI_ERR_INVALID_ARG;
  delete plan;
  return IBMI_OK;
}

}  // extern "C"
