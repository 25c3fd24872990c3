// Batched form of libibmi: many independent SPD matrices of uneven order solved together.
//
// Every sweep of every matrix runs in one captured HIP graph: for each set index j, one
// grouped launch of the panel products of set j of all matrices that have one, one grouped
// split-K diagonal launch and one grouped finalisation; then one grouped residual launch,
// a per-matrix reduction and a check kernel that marks converged (or capped) matrices
// inactive on the device.  Inactive matrices are skipped by every later kernel, so the graph
// can be replayed until no matrix is active without the host looking at each one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"
#include "ibmi.h"
#include "kernels.h"

using namespace ibmi;

namespace {

constexpr size_t kAlignB = 256;
size_t up(size_t x) { return (x + kAlignB - 1) / kAlignB * kAlignB; }

#define BHIP(call)                                   \
  do {                                               \
    if ((call) != hipSuccess) return IBMI_ERR_HIP;   \
  } while (0)

// One grouped launch: its tasks (host copy), where they live on the device, and shape.
struct Group {
  std::vector<GemmTask> tasks;
  std::vector<int> tile_off;  // ntasks + 1
  size_t d_tasks = 0, d_off = 0;  // workspace offsets
  int epi = 0;
  GemmCfg cfg = GEMM_64x64_K16;
  bool vec = false;
};

struct FinGroup {
  std::vector<FinTask> tasks;
  size_t d_tasks = 0;
};

}  // namespace

struct ibmi_batch_s {
  int n = 0;
  ibmi_options o;
  std::vector<int64_t> p, lda;
  std::vector<const double*> A;
  hipStream_t st = nullptr;
  char* work = nullptr;
  size_t total = 0;
  // blocks of all matrices
  std::vector<BlockDesc> blocks;
  std::vector<int> blk0, nblk;
  std::vector<int64_t> wt_off;  // doubles from wt region, per block
  int kmax = 0;
  // regions
  size_t r_desc = 0, r_fac = 0, r_wt = 0, r_part = 0, r_red = 0, r_state = 0, r_tasks = 0,
         r_status = 0, r_redoff = 0, r_active = 0;
  size_t part_doubles = 0, red_doubles = 0, task_bytes = 0;
  // tuning
  GemmCfg cfg_panel = GEMM_64x64_K16, cfg_diag = GEMM_64x64_K16, cfg_resid = GEMM_64x64_K16;
  // per-solve tables
  std::vector<Group> panel, diag, resid;  // panel/diag per set index j; resid has one entry
  std::vector<FinGroup> fin;
  std::vector<int> red_off;  // per matrix offsets of residual partial sums (n + 1)
  std::vector<double*> H;
  std::vector<int64_t> ldh;
  bool tables_ready = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double* fac() const { return (double*)(work + r_fac); }
  double* wt() const { return (double*)(work + r_wt); }
  double* part() const { return (double*)(work + r_part); }
  double* red() const { return (double*)(work + r_red); }
  BatchState* state() const { return (BatchState*)(work + r_state); }
  int* active() const { return (int*)(work + r_active); }  // n flags, count, ticket
  int* status() const { return (int*)(work + r_status); }
  int* redoff() const { return (int*)(work + r_redoff); }
  ~ibmi_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

// Split-K factor of a batch's diagonal product b x b x c: enough workgroups per task that
// the grouped launch fills the chip, but chunks of at least 256 columns.
int batch_splits(int64_t b, int64_t c) {
  if (c <= 0) return 1;
  const int64_t tiles = ((b + 63) / 64) * ((b + 63) / 64);
  int64_t s = std::max<int64_t>(1, (64 + tiles - 1) / tiles);
  s = std::min<int64_t>(s, std::max<int64_t>(1, c / 256));
  return (int)std::min<int64_t>(s, 16);
}

// Residual partial sums: one per tile, sized for the smallest tile any configuration uses.
int64_t batch_tiles_sum(const ibmi_batch_s* B) {
  int64_t t = 0;
  for (int i = 0; i < B->n; ++i) t += ((B->p[i] + 31) / 32) * ((B->p[i] + 63) / 64);
  return t;
}

// Fills the sets of every matrix and the workspace layout; returns INVALID_ARG on bad input.
ibmi_status batch_layout(ibmi_batch_s* B) {
  const int64_t br = B->o.block_rows, ov = B->o.overlap;
  if (br < 1 || ov < 0 || ov >= br || br > 1024) return IBMI_ERR_INVALID_ARG;
  B->blocks.clear();
  B->blk0.assign(B->n, 0);
  B->nblk.assign(B->n, 0);
  B->wt_off.clear();
  int64_t fac = 0, wt = 0;
  size_t part = 0;
  B->kmax = 0;
  std::vector<size_t> part_per_step;
  for (int i = 0; i < B->n; ++i) {
    if (B->p[i] < 1) return IBMI_ERR_INVALID_ARG;
    std::vector<int64_t> s, e;
    default_partition(B->p[i], br, ov, s, e);
    B->blk0[i] = (int)B->blocks.size();
    B->nblk[i] = (int)s.size();
    B->kmax = std::max(B->kmax, (int)s.size());
    if (part_per_step.size() < s.size()) part_per_step.resize(s.size(), 0);
    for (size_t k = 0; k < s.size(); ++k) {
      BlockDesc d;
      d.s = s[k];
      d.b = e[k] - s[k];
      d.l_off = fac;
      d.linv_off = fac + d.b * d.b;
      d.ainv_off = fac + 2 * d.b * d.b;
      d.a = B->A.empty() ? nullptr : B->A[i];
      d.lda = B->lda.empty() ? 0 : B->lda[i];
      fac += 3 * d.b * d.b;
      B->blocks.push_back(d);
      B->wt_off.push_back(wt);
      const int64_t c = B->p[i] - d.b;
      wt += c * d.b;
      part_per_step[k] += (size_t)batch_splits(d.b, c) * d.b * d.b;
    }
  }
  for (size_t v : part_per_step) part = std::max(part, v);
  B->part_doubles = std::max<size_t>(part, 1);
  B->red_doubles = (size_t)std::max<int64_t>(batch_tiles_sum(B), 1);
  const size_t nb = B->blocks.size();
  // task tables: per set index, panel + diag GEMM tasks and finalisation tasks, plus the
  // residual tasks and the plan-time tasks (reused region)
  const size_t max_tasks = 3 * nb + 3 * (size_t)B->n + 16;
  B->task_bytes = max_tasks * (sizeof(GemmTask) + sizeof(FinTask) + 2 * sizeof(int)) +
                  (size_t)(4 * B->kmax + 16) * 2 * kAlignB;
  size_t off = 0;
  B->r_desc = off;
  off = up(off + nb * sizeof(BlockDesc));
  B->r_fac = off;
  off = up(off + (size_t)fac * 8);
  B->r_wt = off;
  off = up(off + (size_t)wt * 8);
  B->r_part = off;
  off = up(off + B->part_doubles * 8);
  B->r_red = off;
  off = up(off + B->red_doubles * 8);
  B->r_redoff = off;
  off = up(off + (B->n + 1) * sizeof(int));
  B->r_state = off;
  off = up(off + (B->n + 1) * sizeof(BatchState));
  B->r_active = off;
  off = up(off + (B->n + 2) * sizeof(int));
  B->r_status = off;
  off = up(off + 4 * sizeof(int));
  B->r_tasks = off;
  off = up(off + B->task_bytes);
  B->total = off;
  return IBMI_OK;
}

void set_shape(GemmTask& t, GemmCfg cfg, int splits) {
  const GemmDims d = gemm_dims(cfg);
  t.mtc = (int)((t.M + d.bm - 1) / d.bm);
  t.ntc = (int)((t.N + d.bn - 1) / d.bn);
  t.splits = std::max(1, splits);
  t.kchunk = t.splits > 1 ? (t.K + t.splits - 1) / t.splits : std::max<int64_t>(t.K, 1);
}

void finish_group(Group& g) {
  g.tile_off.assign(g.tasks.size() + 1, 0);
  for (size_t t = 0; t < g.tasks.size(); ++t)
    g.tile_off[t + 1] = g.tile_off[t] + g.tasks[t].mtc * g.tasks[t].ntc * g.tasks[t].splits;
  g.vec = true;
  for (const GemmTask& t : g.tasks) g.vec = g.vec && gemm_vec_ok(t);
}

// Copies a group's tasks and prefix sums into the task region at *cursor.
ibmi_status upload_group(ibmi_batch_s* B, Group& g, size_t* cursor) {
  if (g.tasks.empty()) return IBMI_OK;
  const size_t tb = g.tasks.size() * sizeof(GemmTask), ob = g.tile_off.size() * sizeof(int);
  if (*cursor + up(tb) + up(ob) > B->task_bytes) return IBMI_ERR_OUT_OF_MEMORY;
  g.d_tasks = B->r_tasks + *cursor;
  *cursor += up(tb);
  g.d_off = B->r_tasks + *cursor;
  *cursor += up(ob);
  BHIP(hipMemcpyAsync(B->work + g.d_tasks, g.tasks.data(), tb, hipMemcpyHostToDevice, B->st));
  BHIP(hipMemcpyAsync(B->work + g.d_off, g.tile_off.data(), ob, hipMemcpyHostToDevice, B->st));
  return IBMI_OK;
}

hipError_t launch_group(ibmi_batch_s* B, const Group& g, const int* active) {
  if (g.tasks.empty()) return hipSuccess;
  return gemm_grouped(g.cfg, g.epi, (const GemmTask*)(B->work + g.d_tasks),
                      (const int*)(B->work + g.d_off), (int)g.tasks.size(), g.tile_off.back(),
                      active, g.vec, B->st);
}

// The plan-time products of every set: A_I^{-1} = L^{-T} L^{-1}, then W^T = A[I^c,I] A_I^{-1}.
ibmi_status batch_factor_products(ibmi_batch_s* B) {
  Group g1, g2;
  FinGroup sym;
  g1.epi = g2.epi = EPI_STORE;
  g1.cfg = g2.cfg = GEMM_64x64_K16;
  for (size_t k = 0; k < B->blocks.size(); ++k) {
    const BlockDesc& d = B->blocks[k];
    double* linv = B->fac() + d.linv_off;
    double* tmp = B->fac() + d.l_off;
    GemmTask t{};
    t.X = Opnd{linv, d.b, IdxMap{}, IdxMap{}};
    t.Y = t.X;
    t.M = t.N = t.K = d.b;
    t.ea.out = tmp;
    t.ea.ldo = d.b;
    set_shape(t, g1.cfg, 1);
    g1.tasks.push_back(t);
    FinTask f{};
    f.x = tmp;
    f.out = B->fac() + d.ainv_off;
    f.b = d.b;
    sym.tasks.push_back(f);
  }
  int mat = 0;
  for (size_t k = 0; k < B->blocks.size(); ++k) {
    while (mat + 1 < B->n && (int)k >= B->blk0[mat + 1]) ++mat;
    const BlockDesc& d = B->blocks[k];
    const int64_t c = B->p[mat] - d.b;
    if (c == 0) continue;
    GemmTask t{};
    const IdxMap g{0, d.s, d.b};
    t.X = Opnd{B->A[mat], B->lda[mat], IdxMap{d.s, INT64_MAX, 0}, g};
    t.Y = Opnd{B->fac() + d.ainv_off, d.b, IdxMap{}, IdxMap{}};
    t.M = c;
    t.N = d.b;
    t.K = d.b;
    t.ea.out = B->wt() + B->wt_off[k];
    t.ea.ldo = d.b;
    set_shape(t, g2.cfg, 1);
    g2.tasks.push_back(t);
  }
  finish_group(g1);
  finish_group(g2);
  size_t cur = 0;
  ibmi_status rc = upload_group(B, g1, &cur);
  if (rc != IBMI_OK) return rc;
  rc = upload_group(B, g2, &cur);
  if (rc != IBMI_OK) return rc;
  sym.d_tasks = B->r_tasks + cur;
  BHIP(hipMemcpyAsync(B->work + sym.d_tasks, sym.tasks.data(), sym.tasks.size() * sizeof(FinTask),
                      hipMemcpyHostToDevice, B->st));
  BHIP(launch_group(B, g1, nullptr));
  BHIP(symmetrize_grouped((const FinTask*)(B->work + sym.d_tasks), (int)sym.tasks.size(), B->st));
  BHIP(launch_group(B, g2, nullptr));
  BHIP(hipStreamSynchronize(B->st));  // the host task copies must outlive the uploads
  return IBMI_OK;
}

// Task tables of one sweep for the current H pointers.
ibmi_status build_tables(ibmi_batch_s* B) {
  B->panel.assign(B->kmax, Group{});
  B->diag.assign(B->kmax, Group{});
  B->fin.assign(B->kmax, FinGroup{});
  B->resid.assign(1, Group{});
  size_t part_cursor = 0;
  for (int j = 0; j < B->kmax; ++j) {
    Group& gp = B->panel[j];
    Group& gd = B->diag[j];
    gp.epi = EPI_PANEL;
    gd.epi = EPI_PARTIAL;
    gp.cfg = B->cfg_panel;
    gd.cfg = B->cfg_diag;
    part_cursor = 0;
    for (int i = 0; i < B->n; ++i) {
      if (j >= B->nblk[i]) continue;
      const int k = B->blk0[i] + j;
      const BlockDesc& d = B->blocks[k];
      const int64_t c = B->p[i] - d.b;
      double* H = B->H[i];
      const int64_t ldh = B->ldh[i];
      FinTask f{};
      f.x = B->fac() + d.ainv_off;  // A_I^{-1}
      f.b = d.b;
      f.out = H;
      f.ldo = ldh;
      f.s = d.s;
      f.mat = i;
      f.splits = 0;
      if (c > 0) {
        const IdxMap g{0, d.s, d.b};
        GemmTask t{};
        t.X = Opnd{B->wt() + B->wt_off[k], d.b, IdxMap{}, IdxMap{}};
        t.Y = Opnd{H, ldh, g, g};
        t.M = d.b;
        t.N = c;
        t.K = c;
        t.mat = i;
        t.ea.out = H;
        t.ea.ldo = ldh;
        t.ea.s = d.s;
        t.ea.g = g;
        set_shape(t, gp.cfg, 1);
        gp.tasks.push_back(t);
        GemmTask u{};
        u.X = t.X;
        u.Y = Opnd{H, ldh, g, IdxMap{d.s, INT64_MAX, 0}};
        u.M = d.b;
        u.N = d.b;
        u.K = c;
        u.mat = i;
        const int splits = batch_splits(d.b, c);
        u.ea.out = B->part() + part_cursor;
        set_shape(u, gd.cfg, splits);
        gd.tasks.push_back(u);
        f.part = B->part() + part_cursor;
        f.splits = splits;
        part_cursor += (size_t)splits * d.b * d.b;
      }
      B->fin[j].tasks.push_back(f);
    }
    if (part_cursor > B->part_doubles) return IBMI_ERR_OUT_OF_MEMORY;
    finish_group(gp);
    finish_group(gd);
  }
  Group& gr = B->resid[0];
  gr.epi = EPI_RESID;
  gr.cfg = B->cfg_resid;
  B->red_off.assign(B->n + 1, 0);
  for (int i = 0; i < B->n; ++i) {
    GemmTask t{};
    t.X = Opnd{B->A[i], B->lda[i], IdxMap{}, IdxMap{}};
    t.Y = Opnd{B->H[i], B->ldh[i], IdxMap{}, IdxMap{}};
    t.M = t.N = t.K = B->p[i];
    t.mat = i;
    t.ea.red = B->red() + B->red_off[i];
    set_shape(t, gr.cfg, 1);
    B->red_off[i + 1] = B->red_off[i] + t.mtc * t.ntc;
    gr.tasks.push_back(t);
  }
  finish_group(gr);
  size_t cur = 0;
  for (int j = 0; j < B->kmax; ++j) {
    ibmi_status rc = upload_group(B, B->panel[j], &cur);
    if (rc != IBMI_OK) return rc;
    rc = upload_group(B, B->diag[j], &cur);
    if (rc != IBMI_OK) return rc;
    FinGroup& fg = B->fin[j];
    const size_t fb = fg.tasks.size() * sizeof(FinTask);
    if (cur + up(fb) > B->task_bytes) return IBMI_ERR_OUT_OF_MEMORY;
    fg.d_tasks = B->r_tasks + cur;
    cur += up(fb);
    BHIP(hipMemcpyAsync(B->work + fg.d_tasks, fg.tasks.data(), fb, hipMemcpyHostToDevice, B->st));
  }
  ibmi_status rc = upload_group(B, gr, &cur);
  if (rc != IBMI_OK) return rc;
  BHIP(hipMemcpyAsync(B->redoff(), B->red_off.data(), (B->n + 1) * sizeof(int),
                      hipMemcpyHostToDevice, B->st));
  BHIP(hipStreamSynchronize(B->st));
  B->tables_ready = true;
  return IBMI_OK;
}

// Enqueues one sweep of every active matrix, its residual and the device-side stop test.
hipError_t enqueue_sweep(ibmi_batch_s* B) {
  const int* act = B->active();
  for (int j = 0; j < B->kmax; ++j) {
    hipError_t e = launch_group(B, B->panel[j], act);
    if (e != hipSuccess) return e;
    e = launch_group(B, B->diag[j], act);
    if (e != hipSuccess) return e;
    e = diag_finalize_grouped((const FinTask*)(B->work + B->fin[j].d_tasks),
                              (int)B->fin[j].tasks.size(), act, B->st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_group(B, B->resid[0], act);
  if (e != hipSuccess) return e;
  return batch_check(B->red(), B->redoff(), B->n, B->active(), B->state(), B->o.tol,
                     B->o.max_sweeps, B->o.stagnation_guard, B->st);
}

// Task tables for dH (rebuilt when pointers or tuning change) and the captured sweep graph.
ibmi_status prepare(ibmi_batch_s* B, double* const* dH, const int64_t* ldh) {
  bool same = B->tables_ready && (int)B->H.size() == B->n;
  for (int i = 0; i < B->n; ++i) {
    if (!dH[i] || ldh[i] < B->p[i]) return IBMI_ERR_INVALID_ARG;
    if (same && (B->H[i] != dH[i] || B->ldh[i] != ldh[i])) same = false;
  }
  if (same && B->exec) return IBMI_OK;
  B->H.assign(dH, dH + B->n);
  B->ldh.assign(ldh, ldh + B->n);
  ibmi_status rc = build_tables(B);
  if (rc != IBMI_OK) return rc;
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  BHIP(hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_sweep(B);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(B->st, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return IBMI_ERR_HIP;
  }
  B->graph = g;
  BHIP(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  return IBMI_OK;
}

ibmi_status start(ibmi_batch_s* B) {
  for (int i = 0; i < B->n; ++i) BHIP(fill_identity(B->H[i], B->ldh[i], B->p[i], 1.0, B->st));
  BHIP(batch_reset(B->active(), B->state(), B->n, B->st));
  return IBMI_OK;
}

}  // namespace

extern "C" {

size_t ibmi_batch_workspace_bytes(int32_t n, const int64_t* p, const ibmi_options* opts) {
  if (n < 1 || !p || !opts) return 0;
  ibmi_batch_s B;
  B.n = n;
  B.o = *opts;
  B.p.assign(p, p + n);
  if (batch_layout(&B) != IBMI_OK) return 0;
  return B.total;
}

ibmi_status ibmi_batch_plan(ibmi_batch_t* out, int32_t n, const int64_t* p,
                            const double* const* dA, const int64_t* lda, const ibmi_options* opts,
                            void* dWork, size_t work_bytes, void* stream) {
  if (!out || n < 1 || !p || !dA || !lda || !opts || !dWork) return IBMI_ERR_INVALID_ARG;
  if (!(opts->tol > 0.0) || opts->max_sweeps < 1 || opts->precision != IBMI_PREC_FP64 ||
      opts->init != IBMI_INIT_IDENTITY || opts->stop != IBMI_STOP_FRO)
    return IBMI_ERR_INVALID_ARG;
  if (((uintptr_t)dWork % kAlignB) != 0) return IBMI_ERR_INVALID_ARG;
  auto* B = new ibmi_batch_s();
  B->n = n;
  B->o = *opts;
  B->o.bounds = nullptr;
  B->p.assign(p, p + n);
  B->lda.assign(lda, lda + n);
  B->A.assign(dA, dA + n);
  B->st = (hipStream_t)stream;
  for (int i = 0; i < n; ++i)
    if (!dA[i] || lda[i] < p[i]) {
      delete B;
      return IBMI_ERR_INVALID_ARG;
    }
  batch_tuning(&B->cfg_panel, &B->cfg_diag, &B->cfg_resid);
  ibmi_status rc = batch_layout(B);
  if (rc != IBMI_OK || work_bytes < B->total) {
    delete B;
    return rc != IBMI_OK ? rc : IBMI_ERR_OUT_OF_MEMORY;
  }
  B->work = (char*)dWork;
  auto fail = [&](ibmi_status r) {
    delete B;
    return r;
  };
  const int nb = (int)B->blocks.size();
  int64_t bmax = 0;
  for (const BlockDesc& d : B->blocks) bmax = std::max(bmax, d.b);
  if (hipMemcpyAsync(B->work + B->r_desc, B->blocks.data(), nb * sizeof(BlockDesc),
                     hipMemcpyHostToDevice, B->st) != hipSuccess ||
      fill_int(B->status(), INT_MAX, 1, B->st) != hipSuccess ||
      chol_factor((const BlockDesc*)(B->work + B->r_desc), nb, bmax, nullptr, 0, B->fac(),
                  B->status(), B->st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  int status = INT_MAX;
  if (hipMemcpyAsync(&status, B->status(), sizeof(int), hipMemcpyDeviceToHost, B->st) !=
          hipSuccess ||
      hipStreamSynchronize(B->st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  if (status != INT_MAX) return fail(IBMI_ERR_NOT_SPD);
  if (chol_linv((const BlockDesc*)(B->work + B->r_desc), nb, bmax, B->fac(), B->st) != hipSuccess)
    return fail(IBMI_ERR_HIP);
  rc = batch_factor_products(B);
  if (rc != IBMI_OK) return fail(rc);
  *out = B;
  return IBMI_OK;
}

ibmi_status ibmi_batch_solve(ibmi_batch_t B, double* const* dH, const int64_t* ldh,
                             ibmi_info* infos) {
  if (!B || !dH || !ldh || !infos) return IBMI_ERR_INVALID_ARG;
  ibmi_status prc = prepare(B, dH, ldh);
  if (prc != IBMI_OK) return prc;
  prc = start(B);
  if (prc != IBMI_OK) return prc;
  const int replays_per_check = 4;
  int n_active = B->n;
  int launched = 0;
  while (n_active > 0 && launched < B->o.max_sweeps) {
    for (int r = 0; r < replays_per_check && launched < B->o.max_sweeps; ++r, ++launched)
      BHIP(hipGraphLaunch(B->exec, B->st));
    BHIP(hipMemcpyAsync(&n_active, B->active() + B->n, sizeof(int), hipMemcpyDeviceToHost,
                        B->st));
    BHIP(hipStreamSynchronize(B->st));
  }
  std::vector<BatchState> hs(B->n);
  BHIP(hipMemcpyAsync(hs.data(), B->state(), B->n * sizeof(BatchState), hipMemcpyDeviceToHost,
                      B->st));
  BHIP(hipStreamSynchronize(B->st));
  ibmi_status rc = IBMI_OK;
  for (int i = 0; i < B->n; ++i) {
    infos[i].sweeps = hs[i].sweeps;
    infos[i].converged = hs[i].converged;
    infos[i].failed_block = -1;
    infos[i].floor_limited = hs[i].floor_limited;
    infos[i].residual = hs[i].residual;
    infos[i].stop_value = hs[i].residual;
    infos[i].cancelled = 0;
    infos[i].evaluations = 0;
    if (!std::isfinite(hs[i].residual)) rc = IBMI_ERR_NONFINITE;
  }
  return rc;
}

ibmi_status ibmi_batch_set_tuning(ibmi_batch_t B, int32_t panel, int32_t diag, int32_t resid) {
  if (!B) return IBMI_ERR_INVALID_ARG;
  for (int32_t c : {panel, diag, resid})
    if (c < 0 || c >= GEMM_CFG_COUNT) return IBMI_ERR_INVALID_ARG;
  B->cfg_panel = (GemmCfg)panel;
  B->cfg_diag = (GemmCfg)diag;
  B->cfg_resid = (GemmCfg)resid;
  B->tables_ready = false;
  return IBMI_OK;
}

ibmi_status ibmi_batch_get_tuning(ibmi_batch_t B, int32_t* cfg3) {
  if (!B || !cfg3) return IBMI_ERR_INVALID_ARG;
  cfg3[0] = B->cfg_panel;
  cfg3[1] = B->cfg_diag;
  cfg3[2] = B->cfg_resid;
  return IBMI_OK;
}

ibmi_status ibmi_batch_autotune(ibmi_batch_t B, double* const* dH, const int64_t* ldh,
                                int32_t reps, int32_t* best_cfg3, double* best_ms) {
  if (!B || !dH || !ldh || reps < 1) return IBMI_ERR_INVALID_ARG;
  static const int cand[][3] = {{GEMM_64x64_K16, GEMM_64x64_K16, GEMM_64x64_K16},
                                {GEMM_64x64, GEMM_64x64, GEMM_64x64},
                                {GEMM_32x64_W1, GEMM_32x64_W1, GEMM_64x64_K16},
                                {GEMM_64x64_W1, GEMM_64x64_W1, GEMM_64x64_W1},
                                {GEMM_64x64_K16, GEMM_64x64_K16, GEMM_128x128_W8},
                                {GEMM_64x128_K16, GEMM_64x64_K16, GEMM_64x128_K16},
                                {GEMM_64x64_W2, GEMM_64x64_W2, GEMM_64x64_K16}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return IBMI_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return IBMI_ERR_HIP;
  }
  double best = 1e300;
  int bi = 0;
  ibmi_status rc = IBMI_OK;
  for (int c = 0; c < (int)(sizeof(cand) / sizeof(cand[0])); ++c) {
    rc = ibmi_batch_set_tuning(B, cand[c][0], cand[c][1], cand[c][2]);
    if (rc == IBMI_OK) rc = prepare(B, dH, ldh);
    if (rc == IBMI_OK) rc = start(B);
    if (rc != IBMI_OK) break;
    if (hipGraphLaunch(B->exec, B->st) != hipSuccess ||  // warm-up replay
        hipEventRecord(e0, B->st) != hipSuccess) {
      rc = IBMI_ERR_HIP;
      break;
    }
    for (int r = 0; r < reps; ++r)
      if (hipGraphLaunch(B->exec, B->st) != hipSuccess) rc = IBMI_ERR_HIP;
    float ms = 0.f;
    if (rc != IBMI_OK || hipEventRecord(e1, B->st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = IBMI_ERR_HIP;
      break;
    }
    if (ms / reps < best) {
      best = ms / reps;
      bi = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != IBMI_OK) return rc;
  rc = ibmi_batch_set_tuning(B, cand[bi][0], cand[bi][1], cand[bi][2]);
  if (best_cfg3) ibmi_batch_get_tuning(B, best_cfg3);
  if (best_ms) *best_ms = best;
  return rc;
}

ibmi_status ibmi_batch_destroy(ibmi_batch_t B) {
  if (!B) return IBMI_ERR_INVALID_ARG;
  delete B;
  return IBMI_OK;
}

}  // extern "C"
