// The interior-point method around the Hessian equation (Section 2), on the device.
//
// Infeasible primal-dual path following on  min C . X  s.t.  A_i . X = b_i,  X PSD  (eq SDP)
// and its dual (eq SDD), with the Nesterov-Todd scaling of Section 2.2: W is the positive
// definite matrix with W S W = X.  Each iteration reduces the Newton system to the Hessian
// equation  H dy = b - sigma mu A(S^{-1}) + A(W R_d W),  R_d = C - S - sum y_i A_i,
// H = A^T (W kron W) A (eqs hesseqn1, hesseqn2), which Algorithm 1 solves on the device (a
// rank-k factor of W, then PCG).  Then dS = R_d - sum dy_i A_i and
// dX = sigma mu S^{-1} - X - W dS W (Todd, Toh and Tutuncu, SIAM J. Optim. 1998), and X and
// (y, S) each move a fixed fraction of the way to the boundary of the cone.
//
// Every matrix step runs here:
//   - W from Cholesky factors and a matrix square root.  With S = L L^T and G = L^T X L,
//     W = L^{-T} G^{1/2} L^{-1} gives W S W = L^{-T} G L^{-1} = X.  The eigenvalues of G are
//     those of X S, all of the order of mu near the central path, so G is well conditioned
//     and its square root comes from the coupled Newton-Schulz iteration (three FP64 MFMA
//     GEMMs per step) rather than from an eigendecomposition;
//   - S^{-1} = L^{-T} L^{-1} (one GEMM; the Cholesky factor and its inverse come from the
//     recursive factorization of the setup);
//   - the step to the boundary from the smallest eigenvalue of L_X^{-1} dX L_X^{-T} (and of
//     L^{-1} dS L^{-T}), and the rank estimate from the largest eigenvalues of W, by Lanczos with
//     full reorthogonalization (GEMVs on the device, the small tridiagonal problem bisected on
//     the host), or by the eigen step's Householder tridiagonalization where Lanczos stops short;
//   - A(X), sum y_i A_i, the residuals and inner products: gathers, scatters and reductions
//     with a fixed summation order.
// The host keeps the loop and reads a few scalars per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "dense.h"
#include "eig.h"

namespace lrsdp {
namespace {

constexpr int kT = 256;
constexpr int kG = 256;  // partial sums per reduction

// ---------------------------------------------------------------- elementwise kernels
// M = a I (n x n, full storage)
__global__ void k_scaled_eye(int n, double a, double* M) {
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
       i += (size_t)gridDim.x * blockDim.x)
    M[i] = (i % (n + 1) == 0) ? a : 0.0;
}

// Rd = C - S, with C = I when C is null
__global__ void k_c_minus(int n, const double* C, const double* S, double* Rd) {
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
       i += (size_t)gridDim.x * blockDim.x) {
    const double c = C ? C[i] : ((i % (n + 1) == 0) ? 1.0 : 0.0);
    Rd[i] = c - S[i];
  }
}

// M += scale sum_i v_i A_i.  A_i has val_i at (a_i, b_i) and (b_i, a_i); the pairs are
// distinct, so no two constraints write one entry.
__global__ void k_add_At(int m, int n, const int32_t* a, const int32_t* b, const double* val,
                         const double* v, double scale, double* M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double t = scale * val[i] * v[i];
  const int ai = a[i], bi = b[i];
  M[(size_t)ai * n + bi] += t;
  if (ai != bi) M[(size_t)bi * n + ai] += t;
}

// out_i = base_i + scale (A_i . X) (base may be null: 0, and may alias out), X symmetric
__global__ void k_gather_A(int m, int n, const int32_t* a, const int32_t* b, const double* coef,
                           const double* X, const double* base, double scale, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double t = scale * (coef[i] * X[(size_t)a[i] * n + b[i]]);
  out[i] = base ? base[i] + t : t;
}

// X = sym(X + alpha D) (D may be null: X = sym(X)); thread per pair i <= j
__global__ void k_sym_axpy(int n, double* X, double alpha, const double* D) {
  const size_t nn = (size_t)n * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < nn;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
    if (i > j) continue;
    const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
    double u = X[ij], w = X[ji];
    if (D) {
      u += alpha * D[ij];
      w += alpha * D[ji];
    }
    const double v = 0.5 * (u + w);
    X[ij] = v;
    X[ji] = v;
  }
}

// dX = sm Si - X - T
__global__ void k_dx(int n, double sm, const double* Si, const double* X, const double* T,
                     double* dX) {
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
       i += (size_t)gridDim.x * blockDim.x)
    dX[i] = sm * Si[i] - X[i] - T[i];
}

// Newton-Schulz: T = (3 I - P) / 2
__global__ void k_ns_t(int n, const double* P, double* T) {
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn;
       i += (size_t)gridDim.x * blockDim.x)
    T[i] = ((i % (n + 1) == 0) ? 1.5 : 0.0) - 0.5 * P[i];
}

// dst = a src
__global__ void k_scale(size_t len, double a, const double* src, double* dst) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = a * src[i];
}

// y += a d (length m)
__global__ void k_axpy(int m, double a, const double* d, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y[i] = fma(a, d[i], y[i]);
}

// y = y + ylo (the double-double answer of the Hessian solve, rounded once)
__global__ void k_round_pair(int m, double* y, const double* ylo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y[i] = y[i] + ylo[i];
}

__global__ void k_zero_int(int count, int* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// *flag = 1 when M (n x n) is not M[0][0] I (every writer stores the same value)
__global__ void k_not_scaled_eye(int n, const double* M, int* flag) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const size_t i = idx / n, j = idx - i * n;
  if (M[idx] != (i == j ? M[0] : 0.0)) *flag = 1;
}

// ---------------------------------------------------------------- Lanczos
// h[i] = V[i] . w for the rows i < R of V (R x n, row-major): one wavefront per row
__global__ __launch_bounds__(256) void k_rows_dot(int R, int n, const double* __restrict__ V,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ h) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const double* v = V + (size_t)row * n;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s = fma(v[c], w[c], s);
  s = wave_sum(s);
  if (lane == 0) h[row] = s;
}

// w -= V^T h over the rows i < R;  *alpha += h[R - 1] (the projection on the newest vector)
__global__ void k_sub_vt(int R, int n, const double* __restrict__ V, const double* __restrict__ h,
                         double* __restrict__ w, double* __restrict__ alpha) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) {
    double t = w[p];
    for (int i = 0; i < R; ++i) t = fma(-V[(size_t)i * n + p], h[i], t);
    w[p] = t;
  }
  if (p == 0) *alpha += h[R - 1];
}

__global__ void k_fill(int len, double x, double* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = x;
}

// v = w / sqrt(nn) (the next Lanczos vector), beta = sqrt(nn)
__global__ void k_lanczos_next(int n, const double* __restrict__ nn, const double* __restrict__ w,
                               double* __restrict__ v, double* __restrict__ beta) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const double b = sqrt(*nn);
  if (p < n) v[p] = b > 0.0 ? w[p] / b : 0.0;
  if (p == 0) *beta = b;
}

// a fixed start vector with no structure the matrices share: v_p = 1 + frac(p golden ratio)
__global__ void k_lanczos_start(int n, double* v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) {
    const double x = p * 0.6180339887498949;
    v[p] = 1.0 + (x - floor(x));
  }
}

// ---------------------------------------------------------------- reductions
// Kinds of the per-element term of a sum over len elements.
enum : int { kDot = 0, kEyeDev = 1, kStartRatio = 2, kTrace = 3 };

// part[blockIdx.x] = this block's share of the sum (grid-stride, fixed grid, so the order
// of every sum depends only on len):
//   kDot:        x_i y_i;
//   kEyeDev:     (delta_ij - x_ij)^2 over an n x n matrix (len = n^2, y unused);
//   kStartRatio: max over i of (1 + |x_i|) / (1 + sqrt(1 / y_i)) (y = 1 / (A^T A)_ii);
//   kTrace:      the diagonal x_ii of an n x n matrix (len = n^2, y unused).
__global__ __launch_bounds__(kT) void k_reduce_part(int kind, size_t len, int n, const double* x,
                                                    const double* y, double* part) {
  __shared__ double red[kT / kWave];
  __shared__ double mx[kT];
  double s = 0.0, hi = 0.0;
  for (size_t i = blockIdx.x * (size_t)kT + threadIdx.x; i < len; i += (size_t)gridDim.x * kT) {
    if (kind == kDot) {
      s = fma(x[i], y[i], s);
    } else if (kind == kEyeDev) {
      const double d = ((i % (n + 1) == 0) ? 1.0 : 0.0) - x[i];
      s = fma(d, d, s);
    } else if (kind == kTrace) {
      if (i % (n + 1) == 0) s += x[i];
    } else {
      hi = fmax(hi, (1.0 + fabs(x[i])) / (1.0 + sqrt(1.0 / y[i])));
    }
  }
  if (kind == kStartRatio) {
    mx[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
      double h = 0.0;
      for (int t = 0; t < kT; ++t) h = fmax(h, mx[t]);
      part[blockIdx.x] = h;
    }
    return;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = the sum (or the max, kStartRatio) of part[0..G) in index order
__global__ void k_reduce_fin(int kind, int G, const double* part, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s = (kind == kStartRatio) ? fmax(s, part[g]) : s + part[g];
  *out = s;
}

int reduce_grid(size_t len) {
  return (int)std::max<size_t>(1, std::min<size_t>(kG, (len + kT - 1) / kT));
}

// slots of sc
enum : int { kXS = 0, kRp2 = 1, kRd2 = 2, kCX = 3, kBy = 4, kB2 = 5, kC2 = 6, kRatio = 7,
             kGF = 8, kNS = 9, kLz = 10, kXdS = 11, kdXS = 12, kdXdS = 13, kSlots = 14 };

// The i-th smallest eigenvalue (0-based) of the symmetric tridiagonal matrix with diagonal a and
// off-diagonal b (j x j), by bisection on the Sturm count to the rounding level.
double tri_eig(const std::vector<double>& a, const std::vector<double>& b, int j, int i) {
  double lo = a[0], hi = a[0];
  for (int q = 0; q < j; ++q) {
    const double r = (q > 0 ? std::fabs(b[q - 1]) : 0.0) + (q + 1 < j ? std::fabs(b[q]) : 0.0);
    lo = std::min(lo, a[q] - r);
    hi = std::max(hi, a[q] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  auto below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double d = 1.0;
    for (int q = 0; q < j; ++q) {
      d = a[q] - x - (q > 0 ? b[q - 1] * b[q - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300 * (scale > 0.0 ? scale : 1.0);
      if (d < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 4e-16 * scale; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) > i) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- the iteration's state
struct Ipm {
  lrsdp_problem* P = nullptr;
  lrsdp_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  int n = 0, m = 0, kmax = 1;
  bool householder = false;  // the steps from the Householder eigen step only
  size_t nn = 0;
  // n x n
  double *Rd = nullptr, *W = nullptr, *Si = nullptr, *Lb = nullptr, *Li = nullptr,
         *Lxi = nullptr, *G = nullptr, *Y = nullptr, *Y2 = nullptr, *Z = nullptr,
         *Z2 = nullptr, *Pm = nullptr, *T1 = nullptr, *T2 = nullptr, *dX = nullptr,
         *dS = nullptr, *Mx = nullptr, *Lx = nullptr, *Xb = nullptr, *Sb = nullptr;  // Xb,
  // m                                                     // Sb, yb: the best iterate so far
  double *rhs = nullptr, *dy = nullptr, *dylo = nullptr, *rp = nullptr, *yb = nullptr;
  // scratch
  double *ptmp = nullptr, *part = nullptr, *sc = nullptr, *lam = nullptr, *vl = nullptr;
  void* ews = nullptr;
  int* flag = nullptr;
  size_t ptmp_n = 0, ews_bytes = 0;
  // Lanczos: basis (lz_max x n), work vector, projections, alpha and beta per step
  int lz_max = 0;
  double *lzV = nullptr, *lzw = nullptr, *lzh = nullptr, *lza = nullptr, *lzb = nullptr;
  double* lz_host = nullptr;  // pinned: alpha (lz_max) then beta (lz_max)

  int reduce(int kind, size_t len, const double* x, const double* y, int slot) {
    const int g = reduce_grid(len);
    k_reduce_part<<<g, kT, 0, s>>>(kind, len, n, x, y, part + (size_t)slot * kG);
    k_reduce_fin<<<1, 64, 0, s>>>(kind, g, part + (size_t)slot * kG, sc + slot);
    LRSDP_HIP(hipGetLastError());
    return LRSDP_OK;
  }
  int read(int count, double* h) {
    LRSDP_HIP(hipMemcpyAsync(ctx->h_pinned, sc, count * sizeof(double), hipMemcpyDeviceToHost,
                             s));
    LRSDP_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) h[i] = ctx->h_pinned[i];
    return LRSDP_OK;
  }
  // C = alpha op(A) op(B) + beta C, n x n operands
  int mm(const double* A, bool tA, const double* B, bool tB, double* C, unsigned flags,
         double alpha = 1.0, double beta = 0.0) {
    GemmArgs g;
    g.M = g.N = g.K = n;
    g.A = A;
    g.lda = n;
    g.transA = tA;
    g.B = B;
    g.ldb = n;
    g.transB = tB;
    g.C = C;
    g.ldc = n;
    g.alpha = alpha;
    g.beta = beta;
    g.flags = flags;
    return gemm(g, s);
  }
  // whether M is c I (then every eigenvalue is c = M[0][0])
  int scaled_eye(const double* M, bool* yes, double* c) {
    k_zero_int<<<1, 64, 0, s>>>(1, flag + 1);
    k_not_scaled_eye<<<grid_for((int64_t)nn, 256), 256, 0, s>>>(n, M, flag + 1);
    LRSDP_HIP(hipGetLastError());
    LRSDP_HIP(hipMemcpyAsync(&ctx->h_pinned[41], flag + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipMemcpyAsync(&ctx->h_pinned[42], M, sizeof(double), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipStreamSynchronize(s));
    int h = 0;
    std::memcpy(&h, &ctx->h_pinned[41], sizeof(int));
    *yes = h == 0;
    *c = ctx->h_pinned[42];
    return LRSDP_OK;
  }
  // Cholesky of M (copied into Lm, which receives L when keep_L) and its inverse into Linv
  // (lower; the upper part outside the 64-aligned diagonal blocks is left undefined, and no
  // product below reads it).  Returns 1 in *bad when a pivot was not positive.
  int chol_inv(const double* M, double* Lm, double* Linv, bool keep_L, int* bad) {
    LRSDP_HIP(hipMemcpyAsync(Lm, M, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    k_zero_int<<<1, 64, 0, s>>>(1, flag);
    LRSDP_TRY(potrf_inv(Lm, n, n, Linv, n, flag, ptmp, keep_L, s));
    int h = 0;
    LRSDP_HIP(hipMemcpyAsync(&ctx->h_pinned[40], flag, sizeof(int), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipStreamSynchronize(s));
    std::memcpy(&h, &ctx->h_pinned[40], sizeof(int));
    *bad = h;
    return LRSDP_OK;
  }
  // Extreme eigenvalues of the symmetric M (n x n) by Lanczos with full reorthogonalization
  // (classical Gram-Schmidt twice per step) from a fixed start vector: lo receives the nlo
  // smallest Ritz values, hi the nhi largest (largest first).  OK once those Ritz values change
  // by at most rtol (relative to their scale) over 8 steps, or after n steps (where the Ritz
  // values are the eigenvalues); NOT_CONVERGED at lz_max steps or when the Krylov space closes
  // early (it may then miss part of the spectrum), and the caller takes the Householder path.
  int lanczos(const double* M, int nlo, double* lo, int nhi, double* hi, double rtol,
              int* steps) {
    const int g = grid_for(n, kT);
    const int jmax = std::min(n, lz_max);
    k_lanczos_start<<<g, kT, 0, s>>>(n, lzV);
    LRSDP_TRY(reduce(kDot, n, lzV, lzV, kLz));
    k_lanczos_next<<<g, kT, 0, s>>>(n, sc + kLz, lzV, lzV, lzb + lz_max);  // v_0 = start / |start|
    k_fill<<<grid_for(lz_max, kT), kT, 0, s>>>(lz_max, 0.0, lza);
    std::vector<double> a, b, prev_lo(nlo, 0.0), prev_hi(nhi, 0.0);
    int done_steps = 0;
    bool converged = false;
    for (int j = 0; j < jmax; ++j) {
      const double* v = lzV + (size_t)j * n;
      LRSDP_TRY(gemv(M, n, n, v, lzw, s));
      for (int pass = 0; pass < 2; ++pass) {  // w -= V V^T w over the basis so far
        k_rows_dot<<<(j + 1 + 3) / 4, 256, 0, s>>>(j + 1, n, lzV, lzw, lzh);
        k_sub_vt<<<g, kT, 0, s>>>(j + 1, n, lzV, lzh, lzw, lza + j);
      }
      LRSDP_TRY(reduce(kDot, n, lzw, lzw, kLz));
      double* next = (j + 1 < jmax) ? lzV + (size_t)(j + 1) * n : lzw;
      k_lanczos_next<<<g, kT, 0, s>>>(n, sc + kLz, lzw, next, lzb + j);
      LRSDP_HIP(hipGetLastError());
      const int jj = j + 1;
      if (jj % 8 != 0 && jj < jmax) continue;
      // T_jj: diagonal alpha_0..alpha_{jj-1}, off-diagonal beta_0..beta_{jj-2}
      LRSDP_HIP(hipMemcpyAsync(lz_host, lza, jj * sizeof(double), hipMemcpyDeviceToHost, s));
      LRSDP_HIP(hipMemcpyAsync(lz_host + lz_max, lzb, jj * sizeof(double),
                               hipMemcpyDeviceToHost, s));
      LRSDP_HIP(hipStreamSynchronize(s));
      a.assign(lz_host, lz_host + jj);
      b.assign(lz_host + lz_max, lz_host + lz_max + jj);
      double big = 0.0;
      for (int q = 0; q < jj; ++q) big = std::max({big, std::fabs(a[q]), std::fabs(b[q])});
      for (int q = 0; q + 1 < jj; ++q)
        if (!(std::fabs(b[q]) > 1e-13 * big)) return LRSDP_NOT_CONVERGED;  // invariant subspace:
                                                                          // the caller falls back
      std::vector<double> cur_lo(nlo, 0.0), cur_hi(nhi, 0.0);
      for (int q = 0; q < nlo && q < jj; ++q) cur_lo[q] = tri_eig(a, b, jj, q);
      for (int q = 0; q < nhi && q < jj; ++q) cur_hi[q] = tri_eig(a, b, jj, jj - 1 - q);
      double scale = 0.0;
      for (double x : cur_lo) scale = std::max(scale, std::fabs(x));
      for (double x : cur_hi) scale = std::max(scale, std::fabs(x));
      bool same = jj >= 16;
      for (int q = 0; q < nlo; ++q) same = same && std::fabs(cur_lo[q] - prev_lo[q]) <= rtol * scale;
      for (int q = 0; q < nhi; ++q) same = same && std::fabs(cur_hi[q] - prev_hi[q]) <= rtol * scale;
      prev_lo = cur_lo;
      prev_hi = cur_hi;
      done_steps = jj;
      if (same) {
        converged = true;
        break;
      }
    }
    if (done_steps == n) converged = true;  // the Ritz values are the eigenvalues
    for (int q = 0; q < nlo; ++q) lo[q] = prev_lo[q];
    for (int q = 0; q < nhi; ++q) hi[q] = prev_hi[q];
    *steps = done_steps;
    return converged ? LRSDP_OK : LRSDP_NOT_CONVERGED;
  }
  // largest step t in (0, inf] with M + t D PSD, M = L L^T with Linv = L^{-1}:
  // -1 / lambda_min(L^{-1} D L^{-T}), inf when that eigenvalue is >= 0
  int max_step(const double* Linv, const double* D, double* out) {
    LRSDP_TRY(mm(Linv, false, D, false, T1, kKToRow));   // L^{-1} D
    LRSDP_TRY(mm(T1, false, Linv, true, Mx, kKToCol | kLowerOut));  // (L^{-1} D) L^{-T}
    LRSDP_TRY(mirror_lower(Mx, n, n, s));
    double h[1];
    int steps = 0;
    const int lrc = householder ? LRSDP_NOT_CONVERGED : lanczos(Mx, 1, h, 0, nullptr, 1e-11, &steps);
    if (lrc < 0) return lrc;
    if (lrc != LRSDP_OK) {  // Householder tridiagonalization and Sturm bisection
      LRSDP_TRY(eig_top_and_min(Mx, n, 1, ews, lam, vl, s));
      LRSDP_HIP(hipMemcpyAsync(ctx->h_pinned, lam, sizeof(double), hipMemcpyDeviceToHost, s));
      LRSDP_HIP(hipStreamSynchronize(s));
      h[0] = ctx->h_pinned[0];
    }
    *out = (h[0] >= 0.0) ? INFINITY : -1.0 / h[0];
    return LRSDP_OK;
  }
};

double* ctx_pinned(const Ipm& I) { return I.ctx->h_pinned; }

// Hessian-solve statuses whose answer still serves as an inexact Newton direction: the last
// iterate of a solve that stopped short of its tolerance or broke down from rounding
bool inexact_ok(int st) {
  return st == LRSDP_NOT_CONVERGED || st == LRSDP_ERR_STAGNATED ||
         st == LRSDP_ERR_INDEFINITE_PRECOND;
}



int ipm_alloc(Ipm& I) {
  const size_t nn = I.nn, m = I.m;
  double** mats[] = {&I.Rd, &I.W, &I.Si, &I.Lb, &I.Li, &I.Lxi, &I.G, &I.Y, &I.Y2, &I.Z,
                     &I.Z2, &I.Pm, &I.T1, &I.T2, &I.dX, &I.dS, &I.Mx, &I.Lx, &I.Xb, &I.Sb};
  for (double** p : mats) LRSDP_TRY(dev_alloc_n(I.ctx, p, nn));
  double** vecs[] = {&I.rhs, &I.dy, &I.dylo, &I.rp, &I.yb};
  for (double** p : vecs) LRSDP_TRY(dev_alloc_n(I.ctx, p, m));
  I.ptmp_n = std::max<size_t>(1, potrf_inv_tmp_doubles(I.n));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.ptmp, I.ptmp_n));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.part, (size_t)kSlots * kG));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.sc, (size_t)kSlots));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lam, (size_t)I.kmax + 4));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.vl, (size_t)(I.kmax + 2) * I.n));
  I.ews_bytes = std::max(eig_workspace_bytes(I.n, 1), eig_workspace_bytes(I.n, I.kmax + 1));
  LRSDP_TRY(dev_alloc(I.ctx, &I.ews, I.ews_bytes));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.flag, (size_t)4));
  I.lz_max = std::min(I.n, 320);
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lzV, (size_t)I.lz_max * I.n));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lzw, (size_t)I.n));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lzh, (size_t)I.lz_max));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lza, (size_t)I.lz_max));
  LRSDP_TRY(dev_alloc_n(I.ctx, &I.lzb, (size_t)I.lz_max + 1));
  if (hipHostMalloc(reinterpret_cast<void**>(&I.lz_host), 2 * (size_t)I.lz_max * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    I.lz_host = nullptr;
    return LRSDP_ERR_DEVICE;
  }
  return LRSDP_OK;
}

void ipm_free(Ipm& I) {
  const size_t nn = I.nn, m = I.m;
  double* mats[] = {I.Rd, I.W, I.Si, I.Lb, I.Li, I.Lxi, I.G, I.Y, I.Y2, I.Z,
                    I.Z2, I.Pm, I.T1, I.T2, I.dX, I.dS, I.Mx, I.Lx, I.Xb, I.Sb};
  for (double* p : mats) dev_free(I.ctx, p, nn * sizeof(double));
  double* vecs[] = {I.rhs, I.dy, I.dylo, I.rp, I.yb};
  for (double* p : vecs) dev_free(I.ctx, p, m * sizeof(double));
  dev_free(I.ctx, I.ptmp, I.ptmp_n * sizeof(double));
  dev_free(I.ctx, I.part, (size_t)kSlots * kG * sizeof(double));
  dev_free(I.ctx, I.sc, (size_t)kSlots * sizeof(double));
  dev_free(I.ctx, I.lam, ((size_t)I.kmax + 4) * sizeof(double));
  dev_free(I.ctx, I.vl, (size_t)(I.kmax + 2) * I.n * sizeof(double));
  dev_free(I.ctx, I.ews, I.ews_bytes);
  dev_free(I.ctx, I.flag, 4 * sizeof(int));
  dev_free(I.ctx, I.lzV, (size_t)I.lz_max * I.n * sizeof(double));
  dev_free(I.ctx, I.lzw, (size_t)I.n * sizeof(double));
  dev_free(I.ctx, I.lzh, (size_t)I.lz_max * sizeof(double));
  dev_free(I.ctx, I.lza, (size_t)I.lz_max * sizeof(double));
  dev_free(I.ctx, I.lzb, ((size_t)I.lz_max + 1) * sizeof(double));
  if (I.lz_host) (void)hipHostFree(I.lz_host);
}

// W (n x n) with W S W = X, and S^{-1}, from S = L L^T (Li = L^{-1}, Lb = L) and the
// coupled Newton-Schulz iteration on G / c, c >= lambda_max(G):  T = (3 I - Z Y) / 2,
// Y <- Y T, Z <- T Z, so that Y -> (G / c)^{1/2} and Z -> (G / c)^{-1/2}.
int nt_scaling(Ipm& I, const double* X, int max_ns, double ns_tol, int* ns_iters,
               double* resid) {
  const int n = I.n;
  hipStream_t s = I.s;
  const int eg = grid_for((int64_t)I.nn, kT, 4096);
  // G and the powers of G / ||G||_F are symmetric: each computes its lower triangle and
  // mirrors it
  LRSDP_TRY(I.mm(X, false, I.Lb, false, I.T1, kKFromCol));                 // X L (L lower)
  LRSDP_TRY(I.mm(I.Lb, true, I.T1, false, I.G, kKFromRow | kLowerOut));   // L^T X L
  LRSDP_TRY(mirror_lower(I.G, n, n, s));
  LRSDP_TRY(I.reduce(kDot, I.nn, I.G, I.G, kGF));
  double h[kSlots];
  LRSDP_TRY(I.read(kSlots, h));
  const double cf = std::sqrt(h[kGF]);
  if (!(cf > 0.0) || !std::isfinite(cf)) return LRSDP_ERR_DEVICE;
  // The iteration takes each eigenvalue x of G / c to 1 when 0 < x < 3, the smallest the
  // slowest, so c should be a close upper bound of lambda_max(G).  G is positive definite, so
  // lambda_max <= (sum lambda_i^8)^{1/8} = ||G^4||_F^{1/4}, which exceeds it by at most n^{1/8}
  // (||G||_F by up to sqrt(n), reached when G is a multiple of I, as on the central path).
  k_scale<<<eg, kT, 0, s>>>(I.nn, 1.0 / cf, I.G, I.Y);                     // G / ||G||_F
  LRSDP_TRY(I.mm(I.Y, false, I.Y, false, I.Pm, kLowerOut));
  LRSDP_TRY(mirror_lower(I.Pm, n, n, s));
  LRSDP_TRY(I.mm(I.Pm, false, I.Pm, false, I.Z, kLowerOut));
  LRSDP_TRY(mirror_lower(I.Z, n, n, s));
  LRSDP_TRY(I.reduce(kDot, I.nn, I.Z, I.Z, kGF));
  LRSDP_TRY(I.read(kSlots, h));
  const double c = cf * std::min(1.0, std::pow(h[kGF], 0.125));
  if (!(c > 0.0) || !std::isfinite(c)) return LRSDP_ERR_DEVICE;
  k_scale<<<eg, kT, 0, s>>>(I.nn, 1.0 / c, I.G, I.Y);
  k_scaled_eye<<<eg, kT, 0, s>>>(n, 1.0, I.Z);
  int it = 0;
  bool done = false;
  // (the products of the loop are symmetric only in exact arithmetic: symmetrizing them, by
  // averaging or by mirroring one triangle, breaks the coupling of Y and Z, and the iteration
  // then diverges once the residual nears 1e-9; the loop keeps the full products)
  for (; it < max_ns && !done; ++it) {
    LRSDP_TRY(I.mm(I.Z, false, I.Y, false, I.Pm, 0));
    LRSDP_TRY(I.reduce(kEyeDev, I.nn, I.Pm, nullptr, kNS));
    k_ns_t<<<eg, kT, 0, s>>>(n, I.Pm, I.T1);
    LRSDP_TRY(I.mm(I.Y, false, I.T1, false, I.Y2, 0));
    LRSDP_TRY(I.mm(I.T1, false, I.Z, false, I.Z2, 0));
    std::swap(I.Y, I.Y2);
    std::swap(I.Z, I.Z2);
    LRSDP_TRY(I.read(kSlots, h));
    // ||I - Z Y||_F of the step just taken; the update squares it (quadratic phase)
    const double r = std::sqrt(h[kNS]);
    *resid = r;
    if (!std::isfinite(r)) break;
    done = r <= ns_tol;
  }
  *ns_iters = it;
  if (!done) return LRSDP_ERR_IPM;
  // G^{1/2} = sqrt(c) Y;  W = L^{-T} G^{1/2} L^{-1};  S^{-1} = L^{-T} L^{-1} (symmetric:
  // lower triangles, mirrored)
  k_sym_axpy<<<eg, kT, 0, s>>>(n, I.Y, 0.0, nullptr);
  LRSDP_TRY(I.mm(I.Y, false, I.Li, false, I.T1, kKFromCol, std::sqrt(c)));
  LRSDP_TRY(I.mm(I.Li, true, I.T1, false, I.W, kKFromRow | kLowerOut));
  LRSDP_TRY(mirror_lower(I.W, n, n, s));
  LRSDP_TRY(I.mm(I.Li, true, I.Li, false, I.Si, kKFromRow | kKFromCol | kLowerOut));
  LRSDP_TRY(mirror_lower(I.Si, n, n, s));
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

}  // namespace

int ipm_run(lrsdp_problem* P, const double* bvec, const double* C, const lrsdp_ipm_opts& o,
            double* X, double* y, double* S, lrsdp_ipm_info* info, lrsdp_ipm_record* recs,
            int max_recs) {
  auto t_start = std::chrono::steady_clock::now();
  Ipm I;
  I.P = P;
  I.ctx = P->ctx;
  I.s = P->ctx->stream;
  I.n = P->n;
  I.m = P->m;
  I.nn = (size_t)I.n * I.n;
  I.kmax = o.k;
  I.householder = o.householder_eig != 0;
  hipStream_t s = I.s;
  const int n = I.n, m = I.m;
  int rc = ipm_alloc(I);
  lrsdp_ipm_info inf{};
  inf.status = LRSDP_NOT_CONVERGED;
  inf.best_iter = -1;
  double best_merit = INFINITY;
  bool have_best = false;
  const int eg = grid_for((int64_t)I.nn, kT, 4096);
  const int vg = grid_for(m, kT);
  auto body = [&]() -> int {
    LRSDP_TRY(rc);
    // starting point (the usual scaled identities): X = xi I, S = eta I, y = 0
    LRSDP_TRY(I.reduce(kDot, m, bvec, bvec, kB2));
    LRSDP_TRY(I.reduce(kStartRatio, m, bvec, P->ginv, kRatio));
    if (C) LRSDP_TRY(I.reduce(kDot, I.nn, C, C, kC2));
    double h[kSlots];
    LRSDP_TRY(I.read(kSlots, h));
    const double nb = std::sqrt(h[kB2]);
    const double nc = C ? std::sqrt(h[kC2]) : std::sqrt((double)n);
    const double xi = std::max({10.0, std::sqrt((double)n), n * h[kRatio]});
    const double eta = std::max({10.0, std::sqrt((double)n), 1.0 + nc});
    if (!o.warm_start) {
      k_scaled_eye<<<eg, kT, 0, s>>>(n, xi, X);
      k_scaled_eye<<<eg, kT, 0, s>>>(n, eta, S);
      LRSDP_HIP(hipMemsetAsync(y, 0, (size_t)m * sizeof(double), s));
    }
    LRSDP_HIP(hipGetLastError());
    // the factors of the current iterate: S = Lb Lb^T with Li = Lb^{-1}, X's inverse factor
    // Lxi (then kept from each step's update, which factors the new iterate to accept it)
    {
      int bad = 0;
      inf.fail_stage = 1;
      LRSDP_TRY(I.chol_inv(S, I.Lb, I.Li, true, &bad));
      if (bad) return LRSDP_ERR_IPM;
      LRSDP_TRY(I.chol_inv(X, I.Lx, I.Lxi, false, &bad));
      if (bad) return LRSDP_ERR_IPM;
      inf.fail_stage = 0;
    }
    lrsdp_opts so = o.solve;
    double mu0 = 0.0;
    double stall_ref = INFINITY;
    int stall = 0;
    for (int it = 0; it <= o.max_iter; ++it) {
      auto t_it = std::chrono::steady_clock::now();
      // residuals and the duality measure
      k_c_minus<<<eg, kT, 0, s>>>(n, C, S, I.Rd);
      k_add_At<<<vg, kT, 0, s>>>(m, n, P->a, P->b, P->val, y, -1.0, I.Rd);
      k_gather_A<<<vg, kT, 0, s>>>(m, n, P->a, P->b, P->coef, X, bvec, -1.0, I.rp);
      LRSDP_TRY(I.reduce(kDot, I.nn, X, S, kXS));
      LRSDP_TRY(I.reduce(kDot, m, I.rp, I.rp, kRp2));
      LRSDP_TRY(I.reduce(kDot, I.nn, I.Rd, I.Rd, kRd2));
      if (C) LRSDP_TRY(I.reduce(kDot, I.nn, C, X, kCX));
      else LRSDP_TRY(I.reduce(kTrace, I.nn, X, nullptr, kCX));  // C = I: C . X = tr X
      LRSDP_TRY(I.reduce(kDot, m, bvec, y, kBy));
      LRSDP_TRY(I.read(kSlots, h));
      const double xs = h[kXS];
      const double mu = xs / n;
      if (it == 0) mu0 = mu;
      const double pinf = std::sqrt(h[kRp2]) / (1.0 + nb);
      const double dinf = std::sqrt(h[kRd2]) / (1.0 + nc);
      const double gap = xs / (1.0 + std::fabs(h[kCX]) + std::fabs(h[kBy]));
      inf.iters = it;
      if (!std::isfinite(mu) || !std::isfinite(pinf) || !std::isfinite(dinf))
        return LRSDP_ERR_DEVICE;
      const double merit = std::max({pinf, dinf, gap});
      if (merit < best_merit) {  // keep the best iterate (returned unless one meets tol)
        best_merit = merit;
        inf.best_iter = it;
        inf.mu = mu;
        inf.pinf = pinf;
        inf.dinf = dinf;
        inf.gap = gap;
        inf.primal_obj = h[kCX];
        inf.dual_obj = h[kBy];
        LRSDP_HIP(hipMemcpyAsync(I.Xb, X, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        LRSDP_HIP(hipMemcpyAsync(I.Sb, S, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        LRSDP_HIP(hipMemcpyAsync(I.yb, y, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice,
                                 s));
        have_best = true;
      }
      if (merit <= o.tol) {
        inf.status = LRSDP_OK;
        return LRSDP_OK;
      }
      if (it == o.max_iter) return LRSDP_OK;  // NOT_CONVERGED
      // stalled: no step in the last stall_iters took the measure below 0.9 of its best (once
      // W is ill-conditioned enough, FP64 directions stop making progress)
      if (merit < 0.9 * stall_ref) {
        stall_ref = merit;
        stall = 0;
      } else if (o.stall_iters > 0 && ++stall >= o.stall_iters) {
        inf.stalled = 1;
        return LRSDP_OK;  // NOT_CONVERGED
      }
      lrsdp_ipm_record rec{};
      rec.mu = mu;
      rec.pinf = pinf;
      rec.dinf = dinf;
      rec.gap = gap;
      // Nesterov-Todd scaling W and S^{-1} from S = L L^T
      auto t_sc = std::chrono::steady_clock::now();
      int ns = 0;
      const int nrc = nt_scaling(I, X, o.max_ns_iter, o.ns_tol, &ns, &inf.ns_resid);
      if (nrc == LRSDP_ERR_IPM) inf.fail_stage = 2;
      LRSDP_TRY(nrc);
      rec.ns_iters = ns;
      LRSDP_HIP(hipStreamSynchronize(s));
      rec.scaling_ms = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t_sc).count();
      // the affine part of the right-hand side, b + A(W R_d W); the centering term
      // -sigma mu A(S^{-1}) is added once sigma is known
      LRSDP_TRY(I.mm(I.W, false, I.Rd, false, I.T1, 0));
      LRSDP_TRY(I.mm(I.T1, false, I.W, false, I.T2, kLowerOut));
      LRSDP_TRY(mirror_lower(I.T2, n, n, s));
      k_gather_A<<<vg, kT, 0, s>>>(m, n, P->a, P->b, P->coef, I.T2, bvec, 1.0, I.rhs);
      LRSDP_HIP(hipGetLastError());
      // the rank of the split: fixed, or (rank_eta > 0) the largest i <= k with
      // lambda_i(W) >= eta lambda_{i+1}(W), at least 1 (Section 5)
      int k = o.k;
      auto t_rank = std::chrono::steady_clock::now();
      if (o.rank_eta > 0.0) {
        // lam_top[i - 1] = lambda_i(W), the k + 1 largest
        double lam_top[17];
        int steps = 0;
        // the first iterate from the default start has W = c I (X and S multiples of I): every
        // eigenvalue is c, which Lanczos cannot see (its Krylov space closes at once)
        bool flat = false;
        double c = 0.0;
        if (it == 0) LRSDP_TRY(I.scaled_eye(I.W, &flat, &c));
        if (flat)
          for (int i = 0; i <= o.k; ++i) lam_top[i] = c;
        const int lrc = flat ? LRSDP_OK
                        : o.householder_eig
                            ? LRSDP_NOT_CONVERGED
                            : I.lanczos(I.W, 0, nullptr, o.k + 1, lam_top, 1e-8, &steps);
        if (lrc < 0) return lrc;
        if (lrc != LRSDP_OK) {  // Householder path: hl[1 .. k+1] are the k+1 largest ascending
          LRSDP_TRY(eig_top_and_min(I.W, n, o.k + 1, I.ews, I.lam, I.vl, s));
          LRSDP_HIP(hipMemcpyAsync(ctx_pinned(I), I.lam, (o.k + 2) * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
          LRSDP_HIP(hipStreamSynchronize(s));
          for (int i = 1; i <= o.k + 1; ++i) lam_top[i - 1] = ctx_pinned(I)[o.k + 2 - i];
        }
        k = 1;
        for (int i = 1; i <= o.k; ++i)
          if (lam_top[i - 1] >= o.rank_eta * lam_top[i]) k = i;
      }
      rec.k = k;
      rec.rank_ms = std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t_rank).count();
      // the solve's tolerance: fixed, or (pcg_eps_mu > 0) in proportion to mu relative to the
      // start, between pcg_eps and 1e-3 (Section 4.2: the ratio of eps to mu is kept)
      so.eps = o.pcg_eps;
      if (o.pcg_eps_mu > 0.0) so.eps = std::min(1e-3, std::max(o.pcg_eps, o.pcg_eps_mu * mu / mu0));
      rec.eps = so.eps;
      // H dy = rhs by Algorithm 1: a rank-k factor of W, then PCG (refined in double-double
      // when W's spectral gap calls for it).  A solve that stops short of eps (NOT_CONVERGED,
      // STAGNATED) still gives the step its best iterate, as an inexact Newton direction.
      lrsdp_factor* F = nullptr;
      int frc = lrsdp_factor_create(P, I.W, k, &so, &F);
      if (frc < 0) return frc;
      rec.factor_ms = F->setup_ms;
      // the direction for the current right-hand side: dy (rounded from its double-double
      // pair), dS = R_d - sum dy_i A_i, dX = c S^{-1} - X - W dS W (c = sigma mu), and the
      // largest steps to the boundary (X = L_X L_X^T, S = L L^T)
      double steps_ms = 0.0;  // the steps to the boundary of the step's own direction
      auto direction = [&](double c, lrsdp_info* si, double* tp, double* td) -> int {
        const int src = lrsdp_solve(F, I.rhs, I.dy, I.dylo, &so, si);
        if (src < 0 && !inexact_ok(src)) return src;
        k_round_pair<<<vg, kT, 0, s>>>(m, I.dy, I.dylo);
        LRSDP_HIP(hipMemcpyAsync(I.dS, I.Rd, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        k_add_At<<<vg, kT, 0, s>>>(m, n, P->a, P->b, P->val, I.dy, -1.0, I.dS);
        LRSDP_TRY(I.mm(I.W, false, I.dS, false, I.T1, 0));
        LRSDP_TRY(I.mm(I.T1, false, I.W, false, I.T2, kLowerOut));
        LRSDP_TRY(mirror_lower(I.T2, n, n, s));
        k_dx<<<eg, kT, 0, s>>>(n, c, I.Si, X, I.T2, I.dX);
        k_sym_axpy<<<eg, kT, 0, s>>>(n, I.dX, 0.0, nullptr);
        LRSDP_HIP(hipGetLastError());
        const auto t0 = std::chrono::steady_clock::now();
        LRSDP_TRY(I.max_step(I.Lxi, I.dX, tp));
        LRSDP_TRY(I.max_step(I.Li, I.dS, td));
        steps_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                       .count();
        return src;
      };
      auto fin = [&](int rc2) {
        lrsdp_factor_destroy(F);
        return rc2;
      };
      // the centering: fixed, or Mehrotra's rule from the affine direction (sigma = 0) and the
      // duality measure its full steps (at most 1) reach,
      //   n mu_aff = X.S + a_d X.dS + a_p dX.S + a_p a_d dX.dS
      double sg = o.sigma;
      double tp = 0.0, td = 0.0;
      if (o.predictor) {
        auto t_pr = std::chrono::steady_clock::now();
        lrsdp_info pi{};
        const int prc = direction(0.0, &pi, &tp, &td);
        if (prc < 0 && !inexact_ok(prc)) return fin(prc);
        int drc = I.reduce(kDot, I.nn, X, I.dS, kXdS);
        if (drc == LRSDP_OK) drc = I.reduce(kDot, I.nn, I.dX, S, kdXS);
        if (drc == LRSDP_OK) drc = I.reduce(kDot, I.nn, I.dX, I.dS, kdXdS);
        if (drc == LRSDP_OK) drc = I.read(kSlots, h);
        if (drc != LRSDP_OK) return fin(drc);
        const double pa = std::min(1.0, tp), da = std::min(1.0, td);
        const double mu_aff = (xs + da * h[kXdS] + pa * h[kdXS] + pa * da * h[kdXdS]) / n;
        const double r = std::max(0.0, mu_aff / mu);
        sg = std::min(1.0, std::max(o.sigma, r * r * r));
        rec.pred_pcg_iters = pi.iters;
        inf.pcg_iters_total += pi.iters;
        rec.pred_ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t_pr).count();
      }
      rec.sigma = sg;
      // rhs = b - sigma mu A(S^{-1}) + A(W R_d W)
      k_gather_A<<<vg, kT, 0, s>>>(m, n, P->a, P->b, P->coef, I.Si, I.rhs, -sg * mu, I.rhs);
      lrsdp_info si{};
      const int src = direction(sg * mu, &si, &tp, &td);
      rec.solve_status = src;
      if (src < 0 && !inexact_ok(src)) return fin(src);
      fin(0);
      rec.pcg_iters = si.iters;
      rec.outer_iters = si.outer_iters;
      rec.solve_ms = si.solve_ms;
      rec.relres = si.relres;
      inf.pcg_iters_total += si.iters;
      // the update: X + a_p dX and S + a_d dS, each accepted once its Cholesky factorization
      // succeeds (the factors are the next step's); near the accuracy FP64 allows, a step
      // computed to 0.9 of the boundary can still leave an iterate that does not factor, and
      // the step is then shortened by 0.8 (at most 10 times)
      const auto t_up = std::chrono::steady_clock::now();
      double ap = std::min(1.0, o.frac * tp), ad = std::min(1.0, o.frac * td);
      int backtracks = 0;
      auto accept = [&](double* M, const double* D, double* Mn, double* Lm, double* Linv,
                        bool keep_L, double* a) -> int {
        for (int tries = 0;; ++tries) {
          LRSDP_HIP(hipMemcpyAsync(Mn, M, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
          k_sym_axpy<<<eg, kT, 0, s>>>(n, Mn, *a, D);
          LRSDP_HIP(hipGetLastError());
          int b2 = 0;
          LRSDP_TRY(I.chol_inv(Mn, Lm, Linv, keep_L, &b2));
          if (!b2) break;
          if (tries == 10) {
            inf.fail_stage = 3;
            return LRSDP_ERR_IPM;
          }
          *a *= 0.8;
          ++backtracks;
        }
        LRSDP_HIP(hipMemcpyAsync(M, Mn, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        return LRSDP_OK;
      };
      LRSDP_TRY(accept(X, I.dX, I.G, I.Lx, I.Lxi, false, &ap));
      LRSDP_TRY(accept(S, I.dS, I.Pm, I.Lb, I.Li, true, &ad));
      k_axpy<<<vg, kT, 0, s>>>(m, ad, I.dy, y);
      LRSDP_HIP(hipGetLastError());
      LRSDP_HIP(hipStreamSynchronize(s));
      rec.alpha_p = ap;
      rec.alpha_d = ad;
      rec.backtracks = backtracks;
      rec.steps_ms = steps_ms + std::chrono::duration<double, std::milli>(
                                    std::chrono::steady_clock::now() - t_up).count();
      rec.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_it)
                   .count();
      if (recs && it < max_recs) recs[it] = rec;
      inf.records = it + 1;
    }
    return LRSDP_OK;
  };
  rc = body();
  // a numerical breakdown after the first step ends the method at its best iterate
  const bool numerical = rc == LRSDP_ERR_IPM || rc == LRSDP_ERR_CHOL_Z || rc == LRSDP_ERR_CHOL_S ||
                         rc == LRSDP_ERR_NOT_PD_W || rc == LRSDP_ERR_EIG ||
                         rc == LRSDP_ERR_INDEFINITE_PRECOND;
  if (numerical && inf.fail_stage != 1 && have_best && inf.iters >= 1) {
    inf.stalled = 2;
    inf.last_error = rc;
    rc = LRSDP_OK;
  }
  if (inf.status != LRSDP_OK && have_best && inf.best_iter != inf.iters) {
    (void)hipMemcpyAsync(X, I.Xb, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(S, I.Sb, I.nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(y, I.yb, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  (void)hipStreamSynchronize(s);
  ipm_free(I);
  inf.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
               .count();
  if (rc < 0) inf.status = rc;
  if (info) *info = inf;
  return rc < 0 ? rc : inf.status;
}

}  // namespace lrsdp
