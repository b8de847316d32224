// Step A1, GEMM-based: the k largest eigenpairs of W by subspace iteration with
// Rayleigh-Ritz, and tau from the trace.
//
// Algorithm 1 step 1a only consumes tau and (V_l, Lambda_l).  Section 3.1 allows any tau
// with lambda_min(Lambda_s) <= tau < lambda_max(Lambda_s); the mean of the n - k smallest
// eigenvalues, (tr W - sum Lambda_l) / (n - k), lies in that range, leaves kappa(W0) (and
// so the bound of Lemma Htilde) unchanged, and needs no small eigenvalue.  Near the end of
// an interior-point run W has the Theta(1/mu) gap of Proposition Weig, so a block of
// b = k vectors converges at the rate lambda_{k+1} / lambda_k = O(mu) per sweep, each sweep
// one W-times-block product (W read once).  The block is not oversampled: W X for vectors
// beyond the k dominant directions is O(mu) against O(1), which leaves the Gram matrix of
// the Cholesky QR numerically singular at small mu.  Without a gap the iteration stalls
// and the caller falls back to the Householder path (eig.hip).
//
// One sweep (basis X: b orthonormal rows of length n):
//   T = X W;  B = X T^T;  B = Q Theta Q^T (Jacobi);  X <- Q^T X, T <- Q^T T  (Ritz pairs)
//   residuals ||T_i - theta_i X_i|| of the k largest; stop once all are at the FP64
//   rounding level of the product (64 u theta_max sqrt(n)), so the pairs are as accurate
//   as a dense eigensolver's
//   X <- orth(T W) by Cholesky QR, twice, after row normalization (each sweep applies W^2).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.h"
#include "eig.h"

namespace lrsdp {
namespace {

constexpr int BMAX = 16;

// G[i][j] = X_i . Y_j, one wavefront per entry (b x b entries).
__global__ __launch_bounds__(64) void k_gram(int b, int n, const double* X, const double* Y,
                                             double* G) {
  const int i = blockIdx.x / b, j = blockIdx.x % b, lane = threadIdx.x;
  double s = 0.0;
  for (int q = lane; q < n; q += 64) s = fma(X[(size_t)i * n + q], Y[(size_t)j * n + q], s);
  s = wave_sum(s);
  if (lane == 0) G[i * b + j] = s;
}

// Cholesky G = L L^T of the B x B Gram matrix (B <= 16, row pitch ldg) and L^{-1} into Linv
// (row pitch ldl), by one wavefront: lane i holds row i; pivots and column values come by
// cross-lane reads.  B is a template parameter so that every register index is fixed at
// compile time.  A non-positive pivot sets *flag.
template <int B>
__device__ __forceinline__ void chol_inv_wave(const double* G, int ldg, double* Linv, int ldl,
                                              int* flag) {
  const int i = threadIdx.x & 63;
  double a[B], y[B];
#pragma unroll
  for (int c = 0; c < B; ++c) {
    a[c] = (i < B && c <= i) ? G[i * ldg + c] : (i == c ? 1.0 : 0.0);
    y[c] = (i == c) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int j = 0; j < B; ++j) {
    double piv = __shfl(a[j], j);
    if (!(piv > 0.0)) {
      if (i == 0) atomicOr(flag, 1);
      piv = 1.0;
    }
    const double inv = 1.0 / sqrt(piv);
    const double l = (i >= j) ? a[j] * inv : 0.0;  // column j of L
    a[j] = l;
#pragma unroll
    for (int c = j + 1; c < B; ++c) {
      const double lc = __shfl(l, c);
      if (i >= c) a[c] = fma(-l, lc, a[c]);
    }
    // forward substitution on the identity: row j of L^{-1} is y_j / l_jj
#pragma unroll
    for (int c = 0; c <= j; ++c) {
      const double yj = __shfl(y[c], j) * inv;
      if (i == j) y[c] = yj;
      else if (i > j) y[c] = fma(-l, yj, y[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < B; ++c)
    if (i < B) Linv[i * ldl + c] = (c <= i) ? y[c] : 0.0;
}

template <int B>
__global__ __launch_bounds__(64) void k_small_chol_inv(const double* G, double* Linv, int* flag) {
  chol_inv_wave<B>(G, B, Linv, 64, flag);
}

void small_chol_inv(int b, const double* G, double* Linv, int* flag, hipStream_t s) {
  switch (b) {
#define LRSDP_SC(B) \
  case B:           \
    k_small_chol_inv<B><<<1, 64, 0, s>>>(G, Linv, flag); \
    break;
    LRSDP_SC(1) LRSDP_SC(2) LRSDP_SC(3) LRSDP_SC(4) LRSDP_SC(5) LRSDP_SC(6) LRSDP_SC(7)
    LRSDP_SC(8) LRSDP_SC(9) LRSDP_SC(10) LRSDP_SC(11) LRSDP_SC(12) LRSDP_SC(13) LRSDP_SC(14)
    LRSDP_SC(15) LRSDP_SC(16)
#undef LRSDP_SC
  }
}

// Scale each row of T to unit length (one wavefront per row).
__global__ __launch_bounds__(64) void k_row_normalize(int n, double* T) {
  const int i = blockIdx.x, lane = threadIdx.x;
  double* t = T + (size_t)i * n;
  double s = 0.0;
  for (int q = lane; q < n; q += 64) s = fma(t[q], t[q], s);
  s = wave_sum(s);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int q = lane; q < n; q += 64) t[q] *= inv;
}

// X[i][q] = sum_{j <= i} Linv[i][j] T[j][q]   (Linv: 64 x 64 block, lower)
__global__ void k_lower_apply(int b, int n, const double* Linv, const double* T, double* X) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)b * n) return;
  const int i = (int)(idx / n), q = (int)(idx - (size_t)i * n);
  double s = 0.0;
  for (int j = 0; j <= i; ++j) s = fma(Linv[i * 64 + j], T[(size_t)j * n + q], s);
  X[idx] = s;
}

// out[i][q] = sum_j Q[j][i] X[j][q]  (rows of out are the Ritz vectors)
__global__ void k_rotate(int b, int n, const double* Q, const double* X, double* out) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)b * n) return;
  const int i = (int)(idx / n), q = (int)(idx - (size_t)i * n);
  double s = 0.0;
  for (int j = 0; j < b; ++j) s = fma(Q[j * b + i], X[(size_t)j * n + q], s);
  out[idx] = s;
}

// res[i] = ||T_i - theta_i X_i|| (one wavefront per row)
__global__ __launch_bounds__(64) void k_ritz_residual(int n, const double* T, const double* X,
                                                      const double* theta, double* res) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const double th = theta[i];
  double s = 0.0;
  for (int q = lane; q < n; q += 64) {
    const double r = T[(size_t)i * n + q] - th * X[(size_t)i * n + q];
    s = fma(r, r, s);
  }
  s = wave_sum(s);
  if (lane == 0) res[i] = sqrt(s);
}

// Orders the LDS accesses of one wavefront's lanes (the only wavefront taking part).
#define LRSDP_WAVE_SYNC()                                   \
  do {                                                      \
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  \
    __builtin_amdgcn_wave_barrier();                        \
  } while (0)

// Cyclic Jacobi on the symmetric b x b matrix sym(B) = (B + B^T) / 2 (b <= 16, row pitch ldb):
// sym(B) = Q diag(theta) Q^T, theta ascending.  Run by one wavefront (lane j owns column j of
// the working copies A, V in LDS; cs: two doubles of LDS).
__device__ void jacobi_wave(int b, const double* Bin, int ldb, double* Q, double* theta,
                            double (*A)[BMAX + 1], double (*V)[BMAX + 1], double* cs) {
  const int t = threadIdx.x & 63;
  for (int e = t; e < BMAX * BMAX; e += 64) {
    const int r = e / BMAX, c = e % BMAX;
    A[r][c] = (r < b && c < b) ? 0.5 * (Bin[r * ldb + c] + Bin[c * ldb + r]) : 0.0;
    V[r][c] = (r == c) ? 1.0 : 0.0;
  }
  LRSDP_WAVE_SYNC();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, nrm = 0.0;
    for (int e = t; e < b * b; e += 64) {
      const int r = e / b, c = e % b;
      const double v = A[r][c] * A[r][c];
      nrm += v;
      if (r != c) off += v;
    }
    off = wave_sum(off);
    nrm = wave_sum(nrm);
    if (off <= 1e-32 * nrm) break;
    for (int p = 0; p < b - 1; ++p)
      for (int q = p + 1; q < b; ++q) {
        if (t == 0) {
          const double apq = A[p][q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double theta_r = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double tt = (theta_r >= 0.0 ? 1.0 : -1.0) /
                              (fabs(theta_r) + sqrt(1.0 + theta_r * theta_r));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        LRSDP_WAVE_SYNC();
        const double c = cs[0], s = cs[1];
        if (t < b) {  // columns p, q of A and V
          const double ap = A[t][p], aq = A[t][q];
          A[t][p] = c * ap - s * aq;
          A[t][q] = s * ap + c * aq;
          const double vp = V[t][p], vq = V[t][q];
          V[t][p] = c * vp - s * vq;
          V[t][q] = s * vp + c * vq;
        }
        LRSDP_WAVE_SYNC();
        if (t < b) {  // rows p, q of A
          const double ap = A[p][t], aq = A[q][t];
          A[p][t] = c * ap - s * aq;
          A[q][t] = s * ap + c * aq;
        }
        LRSDP_WAVE_SYNC();
      }
  }
  if (t == 0) {  // ascending order (selection sort of the columns)
    int ord[BMAX];
    for (int i = 0; i < b; ++i) ord[i] = i;
    for (int i = 0; i < b; ++i)
      for (int j = i + 1; j < b; ++j)
        if (A[ord[j]][ord[j]] < A[ord[i]][ord[i]]) {
          const int tmp = ord[i];
          ord[i] = ord[j];
          ord[j] = tmp;
        }
    for (int i = 0; i < b; ++i) {
      theta[i] = A[ord[i]][ord[i]];
      for (int r = 0; r < b; ++r) Q[r * b + i] = V[r][ord[i]];
    }
  }
  LRSDP_WAVE_SYNC();
}

__global__ __launch_bounds__(64) void k_jacobi(int b, const double* Bin, double* Q,
                                               double* theta) {
  __shared__ double A[BMAX][BMAX + 1];
  __shared__ double V[BMAX][BMAX + 1];
  __shared__ double cs[2];
  jacobi_wave(b, Bin, b, Q, theta, A, V, cs);
}

// ---------------------------------------------------------------- fused sweep kernels
// When b n doubles fit the LDS budget, one workgroup holds the whole block and a sweep
// takes two launches besides the products with W: Rayleigh-Ritz (Gram, Jacobi, rotation,
// residuals) and the orthonormalization (row scaling, Cholesky QR twice).
constexpr int kFT = 512;                   // threads of the fused kernels
constexpr size_t kFusedLds = 96 * 1024;    // their dynamic LDS budget (Rayleigh-Ritz: 2 b n)

// v[0..16) summed over the workgroup into out[0..16) (LDS); red: kFT / 64 x 16 doubles.
__device__ __forceinline__ void wg_sum16(double (&v)[16], double* red, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const double sm = wave_sum(v[m]);
    if (lane == 0) red[w * 16 + m] = sm;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    double sm = 0.0;
    for (int ww = 0; ww < kFT / 64; ++ww) sm += red[ww * 16 + threadIdx.x];
    out[threadIdx.x] = sm;
  }
  __syncthreads();
}

// G[i][j] = sum_q A[i][q] C[j][q], i, j < B (row pitch 16); SYM: the lower triangle, mirrored.
template <int B, bool SYM>
__device__ void wg_gram(int n, const double* A, const double* C, double* red, double* ch,
                        double* G) {
  constexpr int NE = SYM ? B * (B + 1) / 2 : B * B;
  for (int c0 = 0; c0 < NE; c0 += 16) {
    double v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = 0.0;
    for (int q = threadIdx.x; q < n; q += kFT) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int e = c0 + m;
        if (e < NE) {
          int i, j;
          if (SYM) {
            i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            while (i * (i + 1) / 2 > e) --i;
            j = e - i * (i + 1) / 2;
          } else {
            i = e / B;
            j = e - i * B;
          }
          v[m] = fma(A[i * n + q], C[j * n + q], v[m]);
        }
      }
    }
    wg_sum16(v, red, ch);
    if (threadIdx.x < 16 && c0 + threadIdx.x < NE) {
      const int e = c0 + threadIdx.x;
      int i, j;
      if (SYM) {
        i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        j = e - i * (i + 1) / 2;
      } else {
        i = e / B;
        j = e - i * B;
      }
      G[i * 16 + j] = ch[threadIdx.x];
      if (SYM) G[j * 16 + i] = ch[threadIdx.x];
    }
    __syncthreads();
  }
}

// X <- orth(rows of Y): row normalization, then Cholesky QR twice; one workgroup, Y (b x n)
// staged in LDS.  Same arithmetic as the multi-kernel path up to summation order.
template <int B>
__global__ __launch_bounds__(kFT) void k_orth_fused(int n, const double* __restrict__ Y,
                                                    double* __restrict__ X, int* flag) {
  extern __shared__ __align__(16) double xl[];  // B x n
  __shared__ double red[kFT / 64 * 16], ch[16], G[16 * 16], Li[16 * 16];
  const int t = threadIdx.x;
  for (int e = t; e < B * n; e += kFT) xl[e] = Y[e];
  __syncthreads();
  {  // unit rows
    double v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = 0.0;
    for (int q = t; q < n; q += kFT)
#pragma unroll
      for (int i = 0; i < B; ++i) v[i] = fma(xl[i * n + q], xl[i * n + q], v[i]);
    wg_sum16(v, red, ch);
    for (int q = t; q < n; q += kFT)
#pragma unroll
      for (int i = 0; i < B; ++i) xl[i * n + q] *= ch[i] > 0.0 ? 1.0 / sqrt(ch[i]) : 0.0;
    __syncthreads();
  }
  for (int pass = 0; pass < 2; ++pass) {
    wg_gram<B, true>(n, xl, xl, red, ch, G);
    if (t < 64) chol_inv_wave<B>(G, 16, Li, 16, flag);
    __syncthreads();
    for (int q = t; q < n; q += kFT) {
      double col[B];
#pragma unroll
      for (int j = 0; j < B; ++j) col[j] = xl[j * n + q];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        double sm = 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) sm = fma(Li[i * 16 + j], col[j], sm);
        xl[i * n + q] = sm;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < B * n; e += kFT) X[e] = xl[e];
}

// Rayleigh-Ritz on the block X with T = X W: B = X T^T, B = Q diag(theta) Q^T (Jacobi),
// X <- Q^T X, T <- Q^T T (in place), res_i = ||T_i - theta_i X_i||.  One workgroup.
template <int B>
__global__ __launch_bounds__(kFT) void k_rr_fused(int n, double* __restrict__ X,
                                                  double* __restrict__ T,
                                                  double* __restrict__ theta,
                                                  double* __restrict__ res) {
  extern __shared__ __align__(16) double sm[];  // X then T, B x n each
  __shared__ double red[kFT / 64 * 16], ch[16], G[16 * 16], Qm[BMAX * BMAX];
  __shared__ double JA[BMAX][BMAX + 1], JV[BMAX][BMAX + 1], cs[2], th[BMAX];
  double* xl = sm;
  double* tl = sm + (size_t)B * n;
  const int t = threadIdx.x;
  for (int e = t; e < B * n; e += kFT) {
    xl[e] = X[e];
    tl[e] = T[e];
  }
  __syncthreads();
  wg_gram<B, false>(n, xl, tl, red, ch, G);
  if (t < 64) jacobi_wave(B, G, 16, Qm, th, JA, JV, cs);
  __syncthreads();
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = 0.0;
  for (int q = t; q < n; q += kFT) {
    double xc[B], tc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      xc[j] = xl[j * n + q];
      tc[j] = tl[j * n + q];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      double xs = 0.0, ts = 0.0;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        xs = fma(Qm[j * B + i], xc[j], xs);
        ts = fma(Qm[j * B + i], tc[j], ts);
      }
      X[(size_t)i * n + q] = xs;
      T[(size_t)i * n + q] = ts;
      const double r = ts - th[i] * xs;
      v[i] = fma(r, r, v[i]);
    }
  }
  wg_sum16(v, red, ch);
  if (t < B) {
    theta[t] = th[t];
    res[t] = sqrt(ch[t]);
  }
}

// Trace of W in double-double (one block).
__global__ __launch_bounds__(256) void k_trace_dd(int n, const double* W, double* out) {
  __shared__ double hs[256], ls[256];
  dd s = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += 256) s = dd_add_d(s, W[(size_t)i * n + i]);
  hs[threadIdx.x] = s.hi;
  ls[threadIdx.x] = s.lo;
  __syncthreads();
  if (threadIdx.x == 0) {
    dd acc = {0.0, 0.0};
    for (int i = 0; i < 256; ++i) acc = dd_add(acc, {hs[i], ls[i]});
    out[0] = acc.hi;
    out[1] = acc.lo;
  }
}

// lam = {tau, the k largest Ritz values ascending}, tau = (tr W - sum of them) / (n - k).
__global__ void k_ritz_pack(int b, int k, int n, const double* theta, const double* tr,
                            double* lam) {
  if (threadIdx.x != 0) return;
  double top = 0.0;
  for (int i = b - k; i < b; ++i) top += theta[i];
  lam[0] = ((tr[0] - top) + tr[1]) / (double)(n - k);
  for (int i = 0; i < k; ++i) lam[1 + i] = theta[b - k + i];
}

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// Deterministic pseudo-random start block (rows).
__global__ void k_start_block(int b, int n, double* X) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)b * n) return;
  uint32_t st = 0x243F6A88u ^ (uint32_t)(idx * 0x9E3779B9u + 0x7F4A7C15u);
  st ^= st << 13;
  st ^= st >> 17;
  st ^= st << 5;
  X[idx] = (double)(st & 0xFFFFFF) / (double)0x1000000 - 0.5;
}

}  // namespace

size_t spectral_workspace_bytes(int n, int k) {
  const int b = std::min(k, n);
  return (size_t)(3 * b * (size_t)n + 4 * 64 * 64 + 4 * b * b + 4 * b + 16) * sizeof(double) +
         64;
}

int trace_dd(const double* W, int n, double* out, hipStream_t s) {
  k_trace_dd<<<1, 256, 0, s>>>(n, W, out);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int spectral_top(const double* W, int n, int k, void* ws, double* lam_out, double* Vl_out,
                 double* tr_out, int max_sweeps, double* host_res, int* sweeps_out,
                 hipStream_t s) {
  const int b = k;
  if (k < 1 || k > BMAX || k >= n) return LRSDP_ERR_INVALID_ARG;
  double* X = static_cast<double*>(ws);
  double* T = X + (size_t)b * n;
  double* Y = T + (size_t)b * n;
  double* G = Y + (size_t)b * n;     // b x b (also B)
  double* Qm = G + 64 * 64;          // b x b
  double* Dinv = Qm + 64 * 64;       // 64 x 64
  double* theta = Dinv + 64 * 64;    // b
  double* res = theta + 64;          // b
  double* tr = res + 64;             // 2
  int* flag = reinterpret_cast<int*>(tr + 4);
  const size_t bn = (size_t)b * n;
  const int eg = grid_for((int64_t)bn, 256);

  k_trace_dd<<<1, 256, 0, s>>>(n, W, tr);
  k_clear_flag<<<1, 64, 0, s>>>(flag);
  k_start_block<<<eg, 256, 0, s>>>(b, n, T);
  // (the fused kernels keep b-sized register blocks: up to b = 8 they stay in registers)
  const bool fused = b <= 8 && 2 * bn * sizeof(double) <= kFusedLds;
  // X <- orth(rows of T): row normalization, then Cholesky QR twice (T -> Y -> X)
  auto orthonormalize = [&]() -> int {
    if (fused) {
      switch (b) {
#define LRSDP_ORTH(B)                                                            \
  case B:                                                                        \
    k_orth_fused<B><<<1, kFT, bn * sizeof(double), s>>>(n, T, X, flag); \
    break;
        LRSDP_ORTH(1) LRSDP_ORTH(2) LRSDP_ORTH(3) LRSDP_ORTH(4) LRSDP_ORTH(5) LRSDP_ORTH(6)
        LRSDP_ORTH(7) LRSDP_ORTH(8)
#undef LRSDP_ORTH
      }
      LRSDP_HIP(hipGetLastError());
      return LRSDP_OK;
    }
    k_row_normalize<<<b, 64, 0, s>>>(n, T);
    for (int pass = 0; pass < 2; ++pass) {
      const double* src = pass == 0 ? T : Y;
      k_gram<<<b * b, 64, 0, s>>>(b, n, src, src, G);
      small_chol_inv(b, G, Dinv, flag, s);
      k_lower_apply<<<eg, 256, 0, s>>>(b, n, Dinv, src, pass == 0 ? Y : X);
    }
    return LRSDP_OK;
  };
  LRSDP_TRY(orthonormalize());
  double best = 1e300;
  int sweeps = 0;
  int status = LRSDP_ERR_EIG;
  std::vector<double> h(133);
  for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
    LRSDP_TRY(rows_k(n, b, W, 0, X, T, s));                  // T = X W
    if (fused) {  // X <- Ritz vectors, T <- W X, theta, res: one launch
      switch (b) {
#define LRSDP_RR(B)                                                                     \
  case B:                                                                               \
    k_rr_fused<B><<<1, kFT, 2 * bn * sizeof(double), s>>>(n, X, T, theta, res); \
    break;
        LRSDP_RR(1) LRSDP_RR(2) LRSDP_RR(3) LRSDP_RR(4) LRSDP_RR(5) LRSDP_RR(6) LRSDP_RR(7)
        LRSDP_RR(8)
#undef LRSDP_RR
      }
    } else {
      k_gram<<<b * b, 64, 0, s>>>(b, n, X, T, G);              // B = X T^T
      k_jacobi<<<1, 64, 0, s>>>(b, G, Qm, theta);
      k_rotate<<<eg, 256, 0, s>>>(b, n, Qm, X, Y);             // Ritz vectors
      k_rotate<<<eg, 256, 0, s>>>(b, n, Qm, T, X);             // their images under W
      std::swap(X, Y);                                         // X: Ritz vectors, Y: W X
      std::swap(Y, T);                                         // T: W X, Y: free
      k_ritz_residual<<<b, 64, 0, s>>>(n, T, X, theta, res);
    }
    LRSDP_HIP(hipGetLastError());
    // the first sweep from the start block is not expected to converge: its check is skipped
    // (a Cholesky QR that lost rank there shows up at the next check)
    if (sweeps == 1 && max_sweeps > 1) {
      LRSDP_TRY(rows_k(n, b, W, 0, T, Y, s));
      std::swap(T, Y);
      LRSDP_TRY(orthonormalize());
      continue;
    }
    // theta, res, tr and the factorization flag are contiguous: one copy per sweep
    LRSDP_HIP(hipMemcpyAsync(h.data(), theta, 133 * sizeof(double), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipStreamSynchronize(s));
    const double* th = h.data();
    const double* rs = h.data() + 64;
    const double* trw = h.data() + 128;
    int hflag = 0;
    std::memcpy(&hflag, h.data() + 132, sizeof(int));
    double sum_top = 0.0, rmax = 0.0;
    bool finite = hflag == 0;
    for (int i = b - k; i < b; ++i) {
      sum_top += th[i];
      finite = finite && std::isfinite(th[i]) && std::isfinite(rs[i]);
      rmax = std::max(rmax, rs[i]);
    }
    if (!finite) break;  // lost rank in the Cholesky QR: no usable gap
    const double tau = ((trw[0] - sum_top) + trw[1]) / (double)(n - k);
    const double floor = 64.0 * 2.220446049250313e-16 * th[b - 1] * std::sqrt((double)n);
    if (host_res) *host_res = rmax;
    if (tau > 0.0 && rmax <= floor) {
      status = LRSDP_OK;
      break;
    }
    if (rmax < 0.5 * best) best = rmax;
    else if (sweeps > 6 && rmax > 0.9 * best) break;  // stalled: no usable gap
    // the next basis spans W^2 times the Ritz vectors: one more W-times-block product
    // squares the convergence factor of the sweep
    LRSDP_TRY(rows_k(n, b, W, 0, T, Y, s));
    std::swap(T, Y);
    LRSDP_TRY(orthonormalize());
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (status != LRSDP_OK) return status;
  // lam_out = {tau, top-k ascending}; Vl_out = the k top Ritz vectors (rows)
  k_ritz_pack<<<1, 64, 0, s>>>(b, k, n, theta, tr, lam_out);
  LRSDP_HIP(hipMemcpyAsync(Vl_out, X + (size_t)(b - k) * n, (size_t)k * n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  if (tr_out) LRSDP_HIP(hipMemcpyAsync(tr_out, tr, 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
  return LRSDP_OK;
}

}  // namespace lrsdp
