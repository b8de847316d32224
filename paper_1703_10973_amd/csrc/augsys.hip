// Section 4.1 (eq aug_ex): the n-sized preconditioner equation W~ x = b, W~ = tau I + U U^T
// (eq tIUUt), through the symmetric indefinite augmented system
//
//     [ tau I          sqrt(tau) U ] [x]   [b]
//     [ sqrt(tau) U^T     -tau I   ] [y] = [0],
//
// factored by LU with partial pivoting (a backward-stable method; the paper names LDL^T with
// threshold pivoting).  Its second row gives y = U^T x / sqrt(tau) and its first then reads
// W~ x = b.  Eliminating x first without pivoting would repeat the steps of eq wsmf, whose backward
// error grows like u kappa(W~) = u (tau + ||U||^2) / tau as tau shrinks; the pivoted factorization
// keeps it at the rounding level.  The matrix is dense, (n + k)^2 doubles, and the solve takes
// O((n + k)^3) work where eq wsmf takes O(n k^2): a stable solve of the preconditioner equation
// beside the SMW route, not a replacement for it.
//
// One column j of the factorization is two launches: a single workgroup finds the pivot (the
// first row of largest magnitude, as LAPACK's idamax), swaps the rows (all columns, and the
// right-hand side with them) and forms the multipliers below the diagonal; then the trailing
// block takes its rank-1 update.  The two triangular solves run in one workgroup with the
// right-hand side in LDS.
#include <cmath>
#include <cstring>

#include "internal.h"

namespace lrsdp {
namespace {

constexpr int kAT = 256;       // threads of the pivot kernel and of the updates
constexpr int kSolveT = 1024;  // threads of the triangular solves
constexpr int kAugMax = 16384; // n + k at most (the right-hand side lives in LDS: 128 KB)

__global__ void k_aug_build(int n, int k, double tau, const double* __restrict__ Ut,
                            double* __restrict__ K, const double* __restrict__ b,
                            double* __restrict__ r) {
  const int N = n + k;
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)N * N) return;
  const int i = (int)(idx / N), j = (int)(idx - (size_t)i * N);
  const double st = sqrt(tau);
  double v = 0.0;
  if (i < n && j < n) v = (i == j) ? tau : 0.0;
  else if (i < n) v = st * Ut[(size_t)(j - n) * n + i];        // sqrt(tau) U
  else if (j < n) v = st * Ut[(size_t)(i - n) * n + j];        // sqrt(tau) U^T
  else v = (i == j) ? -tau : 0.0;
  K[idx] = v;
  if (j == 0) r[i] = (i < n) ? b[i] : 0.0;
}

// column j: pivot row p = the first i >= j of largest |K[i][j]|; swap rows j and p (and r);
// K[i][j] /= K[j][j] below the diagonal.  A pivot that is zero or not finite sets *flag.
__global__ __launch_bounds__(kAT) void k_aug_pivot(int N, int j, double* __restrict__ K,
                                                   double* __restrict__ r, int* __restrict__ flag) {
  __shared__ double sv[kAT];
  __shared__ int si[kAT];
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = N;
  for (int i = j + t; i < N; i += kAT) {
    const double a = fabs(K[(size_t)i * N + j]);
    if (a > best) {  // rows ascend per thread: the first maximum is kept
      best = a;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int h = kAT / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double ov = sv[t + h];
      const int oi = si[t + h];
      if (ov > sv[t] || (ov == sv[t] && oi < si[t])) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  const double pv = sv[0];
  if (!(pv > 0.0) || !isfinite(pv) || p >= N) {  // singular or not finite
    if (t == 0) *flag = 1;
    return;
  }
  if (p != j) {
    for (int c = t; c < N; c += kAT) {
      const double a = K[(size_t)j * N + c];
      K[(size_t)j * N + c] = K[(size_t)p * N + c];
      K[(size_t)p * N + c] = a;
    }
    if (t == 0) {
      const double a = r[j];
      r[j] = r[p];
      r[p] = a;
    }
  }
  __syncthreads();
  const double inv = 1.0 / K[(size_t)j * N + j];
  for (int i = j + 1 + t; i < N; i += kAT) K[(size_t)i * N + j] *= inv;
}

// K[i][c] -= K[i][j] K[j][c] for i, c in (j, N)
__global__ __launch_bounds__(kAT) void k_aug_update(int N, int j, double* __restrict__ K) {
  const int w = N - j - 1;
  const size_t e = blockIdx.x * (size_t)kAT + threadIdx.x;
  if (e >= (size_t)w * w) return;
  const int i = j + 1 + (int)(e / w), c = j + 1 + (int)(e - (e / w) * w);
  K[(size_t)i * N + c] -= K[(size_t)i * N + j] * K[(size_t)j * N + c];
}

// L U z = r (L unit lower, U upper, both in K), then x = z[0, n)
__global__ __launch_bounds__(kSolveT) void k_aug_solve(int N, int n, const double* __restrict__ K,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ x) {
  extern __shared__ double z[];
  const int t = threadIdx.x;
  for (int i = t; i < N; i += kSolveT) z[i] = r[i];
  __syncthreads();
  for (int j = 0; j < N; ++j) {  // forward: z_i -= L[i][j] z_j, i > j
    const double zj = z[j];
    for (int i = j + 1 + t; i < N; i += kSolveT) z[i] -= K[(size_t)i * N + j] * zj;
    __syncthreads();
  }
  for (int j = N - 1; j >= 0; --j) {  // backward: z_j /= U[j][j]; z_i -= U[i][j] z_j, i < j
    if (t == 0) z[j] /= K[(size_t)j * N + j];
    __syncthreads();
    const double zj = z[j];
    for (int i = t; i < j; i += kSolveT) z[i] -= K[(size_t)i * N + j] * zj;
    __syncthreads();
  }
  for (int i = t; i < n; i += kSolveT) x[i] = z[i];
}

}  // namespace

// lrsdp_aug_wtilde_solve on ctx's device (the caller has made it current)
int aug_wtilde_solve(lrsdp_ctx* ctx, int n, int k, double tau, const double* Ut, const double* b,
                     double* x) {
  if (!ctx || !Ut || !b || !x || n < 1 || k < 1 || !(tau > 0.0) || !std::isfinite(tau) ||
      (int64_t)n + k > kAugMax)
    return LRSDP_ERR_INVALID_ARG;
  hipStream_t s = ctx->stream;
  const int N = n + k;
  double* K = nullptr;
  double* r = nullptr;
  int* flag = nullptr;
  int rc = dev_alloc_n(ctx, &K, (size_t)N * N);
  if (rc == LRSDP_OK) rc = dev_alloc_n(ctx, &r, (size_t)N);
  if (rc == LRSDP_OK) rc = dev_alloc_n(ctx, &flag, (size_t)1);
  auto body = [&]() -> int {
    LRSDP_TRY(rc);
    LRSDP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_aug_build<<<grid_for((int64_t)N * N, 256), 256, 0, s>>>(n, k, tau, Ut, K, b, r);
    for (int j = 0; j < N; ++j) {
      k_aug_pivot<<<1, kAT, 0, s>>>(N, j, K, r, flag);
      const int64_t w = N - j - 1;
      if (w > 0)
        k_aug_update<<<(unsigned)((w * w + kAT - 1) / kAT), kAT, 0, s>>>(N, j, K);
    }
    k_aug_solve<<<1, kSolveT, (size_t)N * sizeof(double), s>>>(N, n, K, r, x);
    LRSDP_HIP(hipGetLastError());
    int h = 0;
    LRSDP_HIP(hipMemcpyAsync(&ctx->h_pinned[43], flag, sizeof(int), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipStreamSynchronize(s));
    std::memcpy(&h, &ctx->h_pinned[43], sizeof(int));
    return h ? LRSDP_ERR_INVALID_ARG : LRSDP_OK;
  };
  const int brc = body();
  (void)hipStreamSynchronize(s);
  if (flag) dev_free(ctx, flag, sizeof(int));
  if (r) dev_free(ctx, r, (size_t)N * sizeof(double));
  if (K) dev_free(ctx, K, (size_t)N * N * sizeof(double));
  return brc;
}

}  // namespace lrsdp
