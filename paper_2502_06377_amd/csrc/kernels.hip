// gfx950 (CDNA4) kernels of the IBMI library other than the GEMMs: block factors (Cholesky,
// L^{-1}; once per plan), diagonal finalisation, initialisation, reductions, the helpers of
// the low-precision update forms and the batched-form bookkeeping.  The GEMM templates live in gemm.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "gemm.h"
#include "kernels.h"

namespace ibmi {
// ---------------------------------------------------------------------------------------
// Cholesky factor of every diagonal block, one workgroup (16 waves) per set.
// Right-looking, panels of NB columns held in LDS (row stride NB+1 to spread banks):
// factor the panel, write it back as L (lower) and L^T (strict upper, so that row i of the
// upper part is column i of L and reads stay contiguous), then update the trailing lower
// triangle.  A non-positive or non-finite pivot records the set index (atomicMin) and stops.
// ---------------------------------------------------------------------------------------
constexpr int CH_NB = 16;
constexpr int CH_THREADS = 1024;

__global__ void __launch_bounds__(CH_THREADS)
chol_factor_kernel(const BlockDesc* desc, const double* A, int64_t lda, double* fac,
                   int* status) {
  extern __shared__ double Ps[];  // rows x (CH_NB + 1)
  constexpr int LDP = CH_NB + 1;
  const BlockDesc bd = desc[blockIdx.x];
  const int b = (int)bd.b;
  const int64_t s = bd.s;
  double* L = fac + bd.l_off;
  if (!A) {
    A = bd.a;
    lda = bd.lda;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = CH_THREADS / 64;

  for (int64_t e = tid; e < (int64_t)b * b; e += CH_THREADS) {
    const int64_t i = e / b, j = e % b;
    L[e] = A[(s + i) * lda + s + j];
  }
  __syncthreads();

  for (int jb = 0; jb < b; jb += CH_NB) {
    const int nb = mn32(CH_NB, b - jb);
    const int rows = b - jb;
    for (int e = tid; e < rows * nb; e += CH_THREADS) {
      const int r = e / nb, c = e % nb;
      Ps[r * LDP + c] = L[(int64_t)(jb + r) * b + jb + c];
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      const double piv = Ps[c * LDP + c];
      if (!(piv > 0.0) || !(piv < INFINITY)) {  // uniform: every thread read the same value
        if (tid == 0) atomicMin(status, (int)blockIdx.x);
        return;
      }
      const double l = sqrt(piv);
      __syncthreads();
      for (int r = c + tid; r < rows; r += CH_THREADS)
        Ps[r * LDP + c] = (r == c) ? l : Ps[r * LDP + c] / l;
      __syncthreads();
      const int w = nb - c - 1;
      if (w > 0) {
        for (int e = tid; e < rows * w; e += CH_THREADS) {
          const int r = e / w, d = c + 1 + e % w;
          if (r >= d) Ps[r * LDP + d] -= Ps[r * LDP + c] * Ps[d * LDP + c];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * nb; e += CH_THREADS) {
      const int r = e / nb, c = e % nb;
      if (r >= c) {
        const double v = Ps[r * LDP + c];
        L[(int64_t)(jb + r) * b + jb + c] = v;
        if (r > c) L[(int64_t)(jb + c) * b + jb + r] = v;
      }
    }
    // trailing update of the lower triangle: rows/cols >= nb (panel-relative)
    for (int i = nb + wave; i < rows; i += NW) {
      double* Lrow = L + (int64_t)(jb + i) * b + jb;
      for (int j = nb + lane; j <= i; j += 64) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < CH_NB; ++t)
          if (t < nb) acc += Ps[i * LDP + t] * Ps[j * LDP + t];
        Lrow[j] -= acc;
      }
    }
    __syncthreads();
  }
}

// L^{-1} by forward substitution, one wave per pair of columns (no LDS, no barriers).
// Column j of L^{-1} is y with L y = e_j; lane l keeps y[l + 64u] in registers.  The row of
// L is read contiguously (t < i selects the lower part).  Writes L^{-1} row-major, zeros
// above the diagonal.
constexpr int LINV_SLOTS = 16;  // b <= 1024

__global__ void __launch_bounds__(64) chol_linv_kernel(const BlockDesc* desc, double* fac) {
  const BlockDesc bd = desc[blockIdx.y];
  const int b = (int)bd.b;
  const int j0 = blockIdx.x * 2;
  if (j0 >= b) return;
  const int j1 = j0 + 1;
  const double* L = fac + bd.l_off;
  double* Linv = fac + bd.linv_off;
  const int lane = threadIdx.x;
  const int nu = (b + 63) / 64;
  double y0[LINV_SLOTS], y1[LINV_SLOTS];
#pragma unroll
  for (int u = 0; u < LINV_SLOTS; ++u) y0[u] = y1[u] = 0.0;
  for (int i = j0; i < b; ++i) {
    const double* Li = L + (int64_t)i * b;
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int u = 0; u < LINV_SLOTS; ++u) {
      const int t = lane + 64 * u;
      if (u < nu && t < i) {
        const double l = Li[t];
        p0 += l * y0[u];
        p1 += l * y1[u];
      }
    }
    p0 = wave_sum(p0);
    p1 = wave_sum(p1);
    const double lii = Li[i];
    const double v0 = ((i == j0 ? 1.0 : 0.0) - p0) / lii;
    const double v1 = i >= j1 ? ((i == j1 ? 1.0 : 0.0) - p1) / lii : 0.0;
    const int ou = i >> 6, ol = i & 63;
#pragma unroll
    for (int u = 0; u < LINV_SLOTS; ++u)
      if (u == ou && lane == ol) {
        y0[u] = v0;
        y1[u] = v1;
      }
  }
#pragma unroll
  for (int u = 0; u < LINV_SLOTS; ++u) {
    const int t = lane + 64 * u;
    if (u < nu && t < b) {
      Linv[(int64_t)t * b + j0] = y0[u];
      if (j1 < b) Linv[(int64_t)t * b + j1] = y1[u];
    }
  }
}

hipError_t chol_factor(const BlockDesc* d_desc, int n_blocks, int64_t b_max, const double* A,
                       int64_t lda, double* fac, int* d_status, hipStream_t st) {
  // The dynamic-LDS limit is a per-kernel attribute shared by every plan in the process, so it
  // is raised once, to what the largest allowed set (1024 rows) needs, and never lowered:
  // plans built concurrently on other threads cannot shrink it under each other.
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute((const void*)chol_factor_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(1024 * (CH_NB + 1) * sizeof(double)));
  });
  if (attr != hipSuccess) return attr;
  const size_t lds = (size_t)b_max * (CH_NB + 1) * sizeof(double);
  hipLaunchKernelGGL(chol_factor_kernel, dim3(n_blocks), dim3(CH_THREADS), lds, st, d_desc, A,
                     lda, fac, d_status);
  return hipGetLastError();
}

hipError_t chol_linv(const BlockDesc* d_desc, int n_blocks, int64_t b_max, double* fac,
                     hipStream_t st) {
  hipLaunchKernelGGL(chol_linv_kernel, dim3((unsigned)((b_max + 1) / 2), n_blocks), dim3(64), 0,
                     st, d_desc, fac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Small elementwise kernels.
// ---------------------------------------------------------------------------------------
__global__ void symmetrize_kernel(const double* x, double* out, int64_t b) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    out[e] = 0.5 * (x[e] + x[j * b + i]);
  }
}

hipError_t symmetrize_block(const double* x, double* out, int64_t b, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(grid), dim3(256), 0, st, x, out, b);
  return hipGetLastError();
}

// H[I,I] = A_I^{-1} - (G + G^T)/2; G[m][n] = sum_z partial[z][m][n] in z order.  Both
// (m,n) and (n,m) use the same sums, so the block is bitwise symmetric.
__global__ void diag_finalize_kernel(const double* ainv, const double* part, int splits,
                                     int64_t b, double* H, int64_t ldh, int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double gij = 0.0, gji = 0.0;
    for (int z = 0; z < splits; ++z) {
      gij += part[z * n + i * b + j];
      gji += part[z * n + j * b + i];
    }
    H[(s + i) * ldh + s + j] = ainv[e] - 0.5 * (gij + gji);
  }
}

hipError_t diag_finalize(const double* ainv, const double* partial, int splits, int64_t b,
                         double* H, int64_t ldh, int64_t s, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(diag_finalize_kernel, dim3(grid), dim3(256), 0, st, ainv, partial, splits,
                     b, H, ldh, s);
  return hipGetLastError();
}

__global__ void fill_identity_kernel(double* H, int64_t ldh, int64_t p, double diag) {
  const int64_t n = p * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / p, j = e % p;
    H[i * ldh + j] = (i == j) ? diag : 0.0;
  }
}

hipError_t fill_identity(double* H, int64_t ldh, int64_t p, double diag, hipStream_t st) {
  const int64_t n = p * p;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_identity_kernel, dim3(grid), dim3(256), 0, st, H, ldh, p, diag);
  return hipGetLastError();
}

__global__ void copy_block_kernel(const double* src, int64_t b, double* H, int64_t ldh,
                                  int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    H[(s + i) * ldh + s + j] = src[e];
  }
}

hipError_t copy_block(const double* src, int64_t b, double* H, int64_t ldh, int64_t s,
                      hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(copy_block_kernel, dim3(grid), dim3(256), 0, st, src, b, H, ldh, s);
  return hipGetLastError();
}

// Sum of squares with a fixed grid: workgroup g takes rows g, g + G, ... in order.
constexpr int SUMSQ_GRID = 1024;
__global__ void __launch_bounds__(256) sumsq_kernel(const double* H, int64_t ldh, int64_t p,
                                                    double* red) {
  __shared__ double ws[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x; i < p; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < p; j += blockDim.x) {
      const double v = H[i * ldh + j];
      acc += v * v;
    }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) red[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

hipError_t sumsq(const double* H, int64_t ldh, int64_t p, double* red, int64_t* n_red,
                 hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(SUMSQ_GRID), dim3(256), 0, st, H, ldh, p, red);
  *n_red = SUMSQ_GRID;
  return hipGetLastError();
}

__global__ void __launch_bounds__(1024) reduce_sum_kernel(const double* red, int64_t n,
                                                          double* out) {
  __shared__ double ws[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += red[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += ws[w];
    out[0] = t;
  }
}

hipError_t reduce_sum(const double* red, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, red, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Helpers of the low-precision update (correction) forms.
// ---------------------------------------------------------------------------------------
__global__ void to_f32_kernel(const double* a, int64_t lda, float* out, int64_t ldo, int64_t p) {
  const int64_t n = p * ldo;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ldo, j = e % ldo;
    out[e] = j < p ? (float)a[i * lda + j] : 0.0f;
  }
}

hipError_t to_f32(const double* a, int64_t lda, float* out, int64_t ldo, int64_t p,
                  hipStream_t st) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(8192), dim3(256), 0, st, a, lda, out, ldo, p);
  return hipGetLastError();
}

__global__ void zero_f32_kernel(float* x, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

hipError_t zero_f32(float* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_f32_kernel, dim3(8192), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

// TT[i][j] = RkT[i][s + j] - sum_z P[z][j][i]   (i, j < b): the transpose of
// T = R[I,I] - Delta^T A[I^c,I], with R[I,I] read from the current residual columns.
__global__ void corr_diag_kernel(const double* rkt, int64_t ldr, int64_t s, const double* part,
                                 int splits, int64_t b, double* tt) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double g = 0.0;
    for (int z = 0; z < splits; ++z) g += part[z * n + j * b + i];
    tt[e] = rkt[i * ldr + s + j] - g;
  }
}

hipError_t corr_diag(const double* rkt, int64_t ldr, int64_t s, const double* part, int splits,
                     int64_t b, double* tt, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(corr_diag_kernel, dim3(grid), dim3(256), 0, st, rkt, ldr, s, part, splits,
                     b, tt);
  return hipGetLastError();
}

// X = sum of the split-K partials in order; H[s+i][s+j] += (X[i][j] + X[j][i]) / 2 and the
// same increment (rounded) into D.  Both sums run in the same order, so the increment, and H,
// stay bitwise symmetric.
__global__ void corr_apply_kernel(const double* part, int splits, int64_t b, double* H,
                                  int64_t ldh, float* D, int64_t ldd, int64_t s) {
  const int64_t n = b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double xij = 0.0, xji = 0.0;
    for (int z = 0; z < splits; ++z) {
      xij += part[z * n + e];
      xji += part[z * n + j * b + i];
    }
    const double inc = 0.5 * (xij + xji);
    H[(s + i) * ldh + s + j] += inc;
    D[(s + i) * ldd + s + j] += (float)inc;
  }
}

hipError_t corr_apply(const double* part, int splits, int64_t b, double* H, int64_t ldh, float* D,
                      int64_t ldd, int64_t s, hipStream_t st) {
  const int64_t n = b * b;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(corr_apply_kernel, dim3(grid), dim3(256), 0, st, part, splits, b, H, ldh, D,
                     ldd, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Batched-form helpers: one workgroup per task (b <= 1024), tasks of inactive matrices skip.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) symmetrize_grouped_kernel(const FinTask* tasks) {
  const FinTask t = tasks[blockIdx.x];
  const int64_t n = t.b * t.b;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t i = e / t.b, j = e % t.b;
    t.out[e] = 0.5 * (t.x[e] + t.x[j * t.b + i]);
  }
}

hipError_t symmetrize_grouped(const FinTask* tasks, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(symmetrize_grouped_kernel, dim3(ntasks), dim3(256), 0, st, tasks);
  return hipGetLastError();
}

// H[s+i][s+j] = x[i][j] - (G + G^T)/2 with G the fixed-order sum of `splits` partials.
__global__ void __launch_bounds__(256) diag_finalize_grouped_kernel(const FinTask* tasks,
                                                                    const int* active) {
  const FinTask t = tasks[blockIdx.x];
  if (active && !active[t.mat]) return;
  const int64_t b = t.b, n = b * b;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t i = e / b, j = e % b;
    double gij = 0.0, gji = 0.0;
    for (int z = 0; z < t.splits; ++z) {
      gij += t.part[z * n + i * b + j];
      gji += t.part[z * n + j * b + i];
    }
    t.out[(t.s + i) * t.ldo + t.s + j] = t.x[e] - 0.5 * (gij + gji);
  }
}

hipError_t diag_finalize_grouped(const FinTask* tasks, int ntasks, const int* active,
                                 hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_finalize_grouped_kernel, dim3(ntasks), dim3(256), 0, st, tasks,
                     active);
  return hipGetLastError();
}

// One workgroup per matrix sums its residual partials in a fixed order and applies the stop
// test; the last workgroup to finish (atomic ticket) counts the matrices still active.
__global__ void __launch_bounds__(256) batch_check_kernel(const double* red, const int* red_off,
                                                          int n, int* active, BatchState* state,
                                                          double tol, int max_sweeps, int guard,
                                                          int* ticket) {
  __shared__ double ws[4];
  __shared__ int last;
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int64_t t = red_off[i] + threadIdx.x; t < red_off[i + 1]; t += blockDim.x) acc += red[t];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (active[i]) {
      BatchState s = state[i];
      const double rho = sqrt(ws[0] + ws[1] + ws[2] + ws[3]);
      s.sweeps += 1;
      s.residual = rho;
      bool stop = false;
      if (!(rho < INFINITY)) stop = true;           // NaN or Inf: stop, host reports it
      else if (rho < tol) {
        s.converged = 1;
        stop = true;
      } else if (s.sweeps >= max_sweeps) {
        stop = true;
      } else {
        if (rho < 0.99 * s.best) {
          s.best = rho;
          s.since_best = 0;
        } else {
          s.since_best += 1;
        }
        if (guard && s.best < 100.0 * tol && s.since_best >= kGuardSweeps) {
          s.floor_limited = 1;
          stop = true;
        }
      }
      state[i] = s;
      if (stop) active[i] = 0;
    }
    __threadfence();
    last = (atomicAdd(ticket, 1) == n - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    int cnt = 0;
    for (int k = 0; k < n; ++k) cnt += __atomic_load_n(&active[k], __ATOMIC_RELAXED);
    active[n] = cnt;
    *ticket = 0;
  }
}

hipError_t batch_check(const double* red, const int* red_off, int n, int* active,
                       BatchState* state, double tol, int max_sweeps, int guard, hipStream_t st) {
  hipLaunchKernelGGL(batch_check_kernel, dim3(n), dim3(256), 0, st, red, red_off, n, active,
                     state, tol, max_sweeps, guard, active + n + 1);
  return hipGetLastError();
}

__global__ void batch_reset_kernel(int* active, BatchState* state, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    active[i] = 1;
    BatchState s;
    s.sweeps = s.converged = s.floor_limited = s.since_best = 0;
    s.residual = 0.0;
    s.best = INFINITY;
    state[i] = s;
  }
  if (i == 0) {
    active[n] = n;
    active[n + 1] = 0;
  }
}

hipError_t batch_reset(int* active, BatchState* state, int n, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, st, active, state,
                     n);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace ibmi
