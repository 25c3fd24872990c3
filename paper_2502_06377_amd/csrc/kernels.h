// Internal interface between the host driver (ibmi.cpp) and the gfx950 kernels
// (kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibmi {

// Index map j -> base + j + (j >= cut ? skip : 0).  Covers the identity (base 0, no cut),
// a contiguous range I = [s, e) (base s) and a complement I^c = [0,s) u [e,p)
// (base 0, cut s, skip e - s) without materialising index arrays or permutations.
struct IdxMap {
  int64_t base = 0, cut = INT64_MAX, skip = 0;
  __host__ __device__ __forceinline__ int64_t operator()(int64_t j) const {
    return base + j + (j >= cut ? skip : 0);
  }
};

// Operand of the FP64 GEMM below: element (k, x) is ptr[r(k) * ld + c(x)].
struct Opnd {
  const double* ptr;
  int64_t ld;
  IdxMap r, c;
};

// Descriptor of one diagonal set I_k = [s, s + b) and where its factors live.
struct BlockDesc {
  int64_t s, b;
  int64_t l_off;      // b*b: Cholesky factor, lower = L, strict upper = L^T
  int64_t linv_off;   // b*b: L^{-1} (lower triangle, zeros above)
  int64_t ainv_off;   // b*b: A_I^{-1}, bitwise symmetric
  const double* a;    // the set's matrix (batched plans; single plans pass A to the kernel)
  int64_t lda;
};

// Epilogue kinds of the MFMA GEMM and their arguments.
enum {
  EPI_STORE = 0,        // out[m][n] = C
  EPI_PANEL = 1,        // H[s+m][g(n)] = H[g(n)][s+m] = -C
  EPI_PARTIAL = 2,      // out[z][m][n] = C over K chunk z
  EPI_RESID = 3,        // red[slot] = sum over the tile of (delta_mn - C)^2
  EPI_RESID_STORE = 4,  // out[m][n] = delta_mn - C and red[slot] = sum of its squares
  EPI_SUBFROM = 5,      // out[m][n] = src[(s+m)][n] - C
  EPI_CORR = 6,         // correction of H[I^c,I] and D (low-precision update forms)
  EPI_SUMSQ = 7         // red[slot] = sum over the tile of C^2
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

// One product of a grouped (batched) launch.
struct GemmTask {
  Opnd X, Y;
  int64_t M, N, K, kchunk;
  int32_t mtc, ntc, splits, mat;
  EpiArgs ea;
};

// Elementwise b x b task: diagonal finalisation (x = A_I^{-1}, part = split-K partials,
// out = H at rows/cols [s, s+b)) or symmetrisation (out = (x + x^T)/2, b x b).
struct FinTask {
  const double* x;
  const double* part;
  double* out;
  int64_t b, ldo, s;
  int32_t splits, mat;
};

// Stagnation guard: sweeps in a row without a 1% improvement of the best stop value that
// end a solve at its floor (long enough that the sweep-to-sweep noise of a slowly converging
// iteration does not end it early).
constexpr int kGuardSweeps = 16;

// Per-matrix state of a batched solve.
struct BatchState {
  int32_t sweeps, converged, floor_limited, since_best;
  double residual;
  double best;
};

// Tile configurations of the MFMA GEMM: workgroup tile, waves, and the number of
// independent 16x16 accumulation chains each wave carries.
enum GemmCfg {
  GEMM_64x64 = 0,       // 2x2 waves of 32x32 ( 4 chains), BK 32
  GEMM_64x64_K16 = 1,   // 2x2 waves of 32x32 ( 4 chains), BK 16
  GEMM_128x128_W8 = 2,  // 2x4 waves of 64x32 ( 8 chains), BK 16
  GEMM_96x128_W8 = 3,   // 2x4 waves of 48x32 ( 6 chains), BK 32
  GEMM_96x64_K16 = 4,   // 2x2 waves of 48x32 ( 6 chains), BK 16
  GEMM_64x128_K16 = 5,  // 2x2 waves of 32x64 ( 8 chains), BK 16
  GEMM_64x64_W1 = 6,    // 1 wave of 64x64    (16 chains), BK 16
  GEMM_32x64_W1 = 7,    // 1 wave of 32x64    ( 8 chains), BK 16
  GEMM_64x64_W2 = 8,    // 2x1 waves of 32x64 ( 8 chains), BK 32
  GEMM_96x128 = 9,      // 2x2 waves of 48x64 (12 chains), BK 32
  GEMM_192x96 = 10,     // 2x2 waves of 96x48 (18 chains), BK 16
  GEMM_CFG_COUNT = 11
};
struct GemmDims {
  int bm, bn, bk;
};
GemmDims gemm_dims(GemmCfg c);
int64_t gemm_tiles(GemmCfg cfg, int64_t M, int64_t N);

// C[m][n] = sum_{k in [k0, k0 + K)} X(k, m) * Y(k, n), for m < M, n < N.
// Epilogues:
//   store   : out[m * ldo + n] = C                                        (splits = 1)
//   panel   : H[(s+m)*ldh + g(n)] = -C and H[g(n)*ldh + s+m] = -C          (splits = 1)
//   partial : out[z * M * N + m * N + n] = C over K chunk z                (split-K)
//   resid   : partial sums of (delta_mn - C)^2 per workgroup -> red[]      (splits = 1)
hipError_t gemm_store(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                      double* out, int64_t ldo, hipStream_t st);
hipError_t gemm_panel(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                      double* H, int64_t ldh, int64_t s, IdxMap g, hipStream_t st);
hipError_t gemm_partial(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                        int splits, double* out, hipStream_t st);
// Writes one partial sum of (delta_mn - C)^2 per tile to red (gemm_tiles of them) and their
// count to *n_red; when out is non-null also stores delta_mn - C to out[m * ldo + n].
hipError_t gemm_resid(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                      double* red, int64_t* n_red, double* out, int64_t ldo, hipStream_t st);
// Writes one partial sum of C[m][n]^2 per tile to red (gemm_tiles of them), count to *n_red.
hipError_t gemm_sumsq(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K, double* red,
                      int64_t* n_red, hipStream_t st);
// FP32 operands, FP32 accumulation: out[m][n] = src[(s+m)*lds + n] - C[m][n].  Column tiles
// starting at n0 >= ncut only sum k < klim (the rest of the operand is known to be zero).
hipError_t gemm_f32_subfrom(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                            int64_t ncut, int64_t klim, const double* src, int64_t lds,
                            int64_t s, double* out, int64_t ldo, hipStream_t st);
// Delta = C (m over I^c via g, n over I): stores Delta[m][n] to delta and adds it to
// H[g(m)][s+n] (mirrored to H[s+n][g(m)]) and, rounded to FP32, to D likewise.
hipError_t gemm_corr(GemmCfg cfg, Opnd X, Opnd Y, int64_t M, int64_t N, int64_t K,
                     double* delta, int64_t ld_delta, double* H, int64_t ldh, float* D,
                     int64_t ldd, int64_t s, IdxMap g, hipStream_t st);
// Split-bfloat16 form of the same update (terms = 2: bf16x3, terms = 3: bf16x6):
// out[m][n] = src[(s+m)*lds + n] - sum_k X[(xrow0+m)*ldx + k] * Y[n*ldy + k] for m < M,
// n < N, k < K (k < klim for column tiles starting at or after ncut).  K is cut into chunks
// of kchunk (0: one chunk); with more than one chunk per tile the FP32 partial products go to
// part (split_max_chunks(K, kchunk) * M * N floats) and a second kernel sums them in order.
// X, Y 16-byte aligned, ldx and ldy multiples of 4.
enum SplitCfg {
  SPLIT_128x128 = 0,  // 2x2 waves of 64x64
  SPLIT_64x128 = 1,   // 1x2 waves of 64x64
  SPLIT_96x128 = 2,   // 2x2 waves of 48x64
  SPLIT_192x128 = 3,  // 3x2 waves of 64x64
  SPLIT_144x128 = 4,  // 3x2 waves of 48x64
  SPLIT_64x64 = 5,    // 1 wave of 64x64
  SPLIT_192x256 = 6,  // 2x4 waves of 96x64
  SPLIT_CFG_COUNT = 7
};
struct SplitDims {
  int bm, bn, bk;
};
SplitDims split_dims(SplitCfg c);
int64_t split_max_chunks(int64_t K, int64_t kchunk);
hipError_t gemm_split_subfrom(SplitCfg cfg, int terms, const float* X, int64_t ldx,
                              int64_t xrow0, const float* Y, int64_t ldy, int64_t M, int64_t N,
                              int64_t K, int64_t ncut, int64_t klim, int64_t kchunk,
                              const double* src, int64_t lds, int64_t s, double* out,
                              int64_t ldo, float* part, hipStream_t st);
// out (p x ldo) = FP32 copy of A (p x p, row stride lda).
hipError_t to_f32(const double* a, int64_t lda, float* out, int64_t ldo, int64_t p,
                  hipStream_t st);
hipError_t zero_f32(float* x, int64_t n, hipStream_t st);
hipError_t corr_diag(const double* rkt, int64_t ldr, int64_t s, const double* part, int splits,
                     int64_t b, double* tt, hipStream_t st);
// X = sum of `splits` partial b x b products (fixed order); H[s+i][s+j] += (X[i][j] +
// X[j][i]) / 2 and the same increment, rounded to FP32, into D.
hipError_t corr_apply(const double* part, int splits, int64_t b, double* H, int64_t ldh, float* D,
                      int64_t ldd, int64_t s, hipStream_t st);

// Grouped launch of tasks[0..ntasks) (tile prefix sums in tile_off, total_tiles workgroups);
// tasks of matrices with active[mat] == 0 are skipped when active is non-null.
hipError_t gemm_grouped(GemmCfg cfg, int epi, const GemmTask* tasks, const int* tile_off,
                        int ntasks, int total_tiles, const int* active, bool vec, hipStream_t st);
// Whether the fast 16-byte load path is valid for both operands of a task.
bool gemm_vec_ok(const GemmTask& t);
hipError_t symmetrize_grouped(const FinTask* tasks, int ntasks, hipStream_t st);
hipError_t diag_finalize_grouped(const FinTask* tasks, int ntasks, const int* active,
                                 hipStream_t st);
// After a batched sweep: per-matrix residual from its tile partial sums (fixed order), then
// the stop test; active[i] = 0 once matrix i converged or reached max_sweeps; active[n] =
// number still active.
hipError_t batch_check(const double* red, const int* red_off, int n, int* active,
                       BatchState* state, double tol, int max_sweeps, int guard,
                       hipStream_t st);
hipError_t batch_reset(int* active, BatchState* state, int n, hipStream_t st);

// Block factors (one launch for all sets of a plan).
// A may be null: each set then reads its own matrix from its descriptor (batched plans).
hipError_t chol_factor(const BlockDesc* d_desc, int n_blocks, int64_t b_max, const double* A,
                       int64_t lda, double* fac, int* d_status, hipStream_t st);
hipError_t chol_linv(const BlockDesc* d_desc, int n_blocks, int64_t b_max, double* fac,
                     hipStream_t st);
hipError_t symmetrize_block(const double* x, double* out, int64_t b, hipStream_t st);

// H[I,I] = A_I^{-1} - (G + G^T)/2 with G = sum of `splits` partial b x b products.
hipError_t diag_finalize(const double* ainv, const double* partial, int splits, int64_t b,
                         double* H, int64_t ldh, int64_t s, hipStream_t st);

// H = I, or H = 0 followed by copy_block for each set.
hipError_t fill_identity(double* H, int64_t ldh, int64_t p, double diag, hipStream_t st);
hipError_t copy_block(const double* src, int64_t b, double* H, int64_t ldh, int64_t s,
                      hipStream_t st);

// Sum of squares of H's entries, one partial per workgroup into red (returns count).
hipError_t sumsq(const double* H, int64_t ldh, int64_t p, double* red, int64_t* n_red,
                 hipStream_t st);
// out[0] = sum red[0..n) in a fixed order (single workgroup).
hipError_t reduce_sum(const double* red, int64_t n, double* out, hipStream_t st);
hipError_t fill_int(int* p, int v, int n, hipStream_t st);

}  // namespace ibmi
