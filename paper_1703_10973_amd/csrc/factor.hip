// Algorithm 1 steps 1-2 on the device (steps A1-A4):
//   1a  tau = lambda_min(W), (V_l, Lambda_l) = the k largest eigenpairs      (eig.hip)
//   1b  U = V_l (Lambda_l - tau I)^{1/2};  W0 = W - U U^T;  Z = chol(2 W0 + U U^T)
//   2   bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U, block (J, L) of which is
//       tau^2 delta_JL I + Z^T B_JL Z,  B_JL = 1/2 [diag(Obar (u_J o u_L)) + D_{u_L} Obar D_{u_J}],
//       because A (A^T A)^{-1} A^T is the projector that samples the symmetric part of a
//       matrix on the pattern Obar (disjoint supports).  Each block is one sparse-times-
//       dense pass (R = B_JL Z) and one FP64 MFMA GEMM (Z^T R, Z triangular).
//       Deflation: the k(k-1)/2 vectors vec(Z^{-1} U K), K skew, span directions that
//       bold U annihilates, where bold S has eigenvalue tau^2; adding shift Q_N Q_N^T
//       (Q_N orthonormal, shift = max diag bold S) leaves bold U bold S^{-1} bold U^T unchanged.
//       L L^T = bold S, then bold S^{-1} = L^{-T} L^{-1} is formed once (TRTRI + LAUUM) so
//       that each PCG iteration applies it as one bandwidth-bound GEMV.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "dense.h"
#include "eig.h"

namespace lrsdp {
namespace {

constexpr int kT = 256;

// lam[0] <- (tr W - sum of the k largest) / (n - k), tr W a double-double pair.
__global__ void k_tau_mean(int n, int k, const double* tr, double* lam) {
  if (threadIdx.x != 0) return;
  double top = 0.0;
  for (int i = 0; i < k; ++i) top += lam[1 + i];
  lam[0] = ((tr[0] - top) + tr[1]) / (double)(n - k);
}

__global__ void k_make_U(int n, int k, const double* lam, const double* Vl, double* U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int j = idx / n;
  const double tau = lam[0];
  const double sc = sqrt(fmax(lam[1 + j] - tau, 0.0));
  U[idx] = Vl[idx] * sc;
}

// W0 = W - U U^T with U U^T accumulated error-free, rounded once; Zin = 2 W0 + U U^T.
__global__ void k_make_W0(int n, int k, const double* W, const double* U, double* W0,
                          double* Zin) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int p = (int)(idx / n), q = (int)(idx - (size_t)p * n);
  dd acc = {W[idx], 0.0};
  double uu = 0.0;
  for (int j = 0; j < k; ++j) {
    const double a = U[(size_t)j * n + p], b = U[(size_t)j * n + q];
    dd pr = two_prod(a, b);
    acc = dd_add(acc, {-pr.hi, -pr.lo});
    uu = fma(a, b, uu);
  }
  const double w0 = acc.hi + acc.lo;
  W0[idx] = w0;
  if (Zin) Zin[idx] = fma(2.0, w0, uu);
}

// P_J[a][c] = sum_{b in Obar(a)} u_J[b] Z[b][c] for every J at once (Z rows read once).
// Grid: (row a, column chunk); each thread owns one column c and k accumulators.
__global__ __launch_bounds__(kT) void k_PJ(int n, int k, const int32_t* rowptr,
                                           const int32_t* colidx, const double* U,
                                           const double* Z, double* PJ) {
  constexpr int KM = 16;
  const int a = blockIdx.x;
  const int c = blockIdx.y * kT + threadIdx.x;
  if (c >= n) return;
  double acc[KM];
#pragma unroll
  for (int J = 0; J < KM; ++J) acc[J] = 0.0;
  for (int e = rowptr[a]; e < rowptr[a + 1]; ++e) {
    const int b = colidx[e];
    const double z = Z[(size_t)b * n + c];
#pragma unroll
    for (int J = 0; J < KM; ++J)
      if (J < k) acc[J] = fma(U[(size_t)J * n + b], z, acc[J]);
  }
  const size_t nn = (size_t)n * n;
#pragma unroll
  for (int J = 0; J < KM; ++J)
    if (J < k) PJ[J * nn + (size_t)a * n + c] = acc[J];
}

// d_JL[a] = sum_{b in Obar(a)} u_J[b] u_L[b] for every pair J >= L (pair index J(J+1)/2 + L).
// One wavefront per row a; its lanes share the row's entries, then a wave reduction per pair.
__global__ __launch_bounds__(256) void k_dJL(int n, int k, const int32_t* rowptr,
                                             const int32_t* colidx, const double* U, double* d) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (a >= n) return;  // whole wavefront
  const int lo = rowptr[a], hi = rowptr[a + 1];
  for (int J = 0; J < k; ++J)
    for (int L = 0; L <= J; ++L) {
      double s = 0.0;
      for (int e = lo + lane; e < hi; e += 64) {
        const int b = colidx[e];
        s = fma(U[(size_t)J * n + b], U[(size_t)L * n + b], s);
      }
      s = wave_sum(s);
      if (lane == 0) d[(size_t)(J * (J + 1) / 2 + L) * n + a] = s;
    }
}

// Block pair p = J (J + 1) / 2 + L (L <= J) of the lower block triangle of bold S.
__device__ __forceinline__ void pair_of(int p, int* J, int* L) {
  int j = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  while (j * (j + 1) / 2 > p) --j;
  *J = j;
  *L = p - j * (j + 1) / 2;
}

// R_JL = B_JL Z = 1/2 (diag(d_JL) Z + D_{u_L} P_J) for the pairs q0 + y, y < gridDim.y, into
// R + y n^2; and (thread 0 of column 0) the batched-GEMM offsets of those pairs:
// A at 0, B at y n^2, C at block (J, L) of bold S (row pitch nk).
__global__ void k_R_pairs(int n, int nk, int q0, const double* Z, const double* U,
                          const double* PJ, const double* dd, double* R, int64_t* offs) {
  const int y = blockIdx.y, p = q0 + y;
  int J, L;
  pair_of(p, &J, &L);
  const size_t nn = (size_t)n * n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    offs[3 * y] = 0;
    offs[3 * y + 1] = (int64_t)y * (int64_t)nn;
    offs[3 * y + 2] = (int64_t)n * J * nk + (int64_t)n * L;
  }
  const double* dJL = dd + (size_t)p * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < nn;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(idx / n);
    R[y * nn + idx] = 0.5 * fma(dJL[a], Z[idx], U[(size_t)L * n + a] * PJ[J * nn + idx]);
  }
}

// S_JJ += v I for the k diagonal blocks (block J = blockIdx.y).
// the diagonal of the k diagonal blocks += tau^2 (tau = lam[0], on the device)
__global__ void k_add_diag(double* S, int n, int ld, const double* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t o = (size_t)n * blockIdx.y * ld + (size_t)n * blockIdx.y;
  const double tau = lam[0];
  if (i < n) S[o + (size_t)i * ld + i] += tau * tau;
}

// N (nk x r): column c <-> pair (i < j): block j holds y_i, block i holds -y_j, y = rows of Yt.
__global__ void k_null_basis(int n, int k, int r, const double* Yt, double* N) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t nk = (size_t)n * k;
  if (idx >= nk * r) return;
  const size_t row = idx / r;
  const int c = (int)(idx - row * r);
  const int blk = (int)(row / n), p = (int)(row - (size_t)blk * n);
  int i = 0, cc = c;
  while (cc >= k - 1 - i) {
    cc -= k - 1 - i;
    ++i;
  }
  const int j = i + 1 + cc;
  double v = 0.0;
  if (blk == j) v = Yt[(size_t)i * n + p];
  else if (blk == i) v = -Yt[(size_t)j * n + p];
  N[idx] = v;
}

// G = Q^T Q (r x r), Q N x r row-major: one workgroup per entry, fixed summation order.
__global__ __launch_bounds__(kT) void k_gram_cols(int N, int r, const double* __restrict__ Q,
                                                  double* __restrict__ G) {
  __shared__ double red[kT / kWave];
  const int a = blockIdx.x / r, b = blockIdx.x % r;
  double s = 0.0;
  for (int p = threadIdx.x; p < N; p += kT)
    s = fma(Q[(size_t)p * r + a], Q[(size_t)p * r + b], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) G[a * r + b] = s;
}

// When the Gram matrix of the null basis was not positive definite (U Z^{-T} rank-deficient,
// e.g. U = 0 for a W with equal top eigenvalues, where bold U = 0 leaves nothing to deflate),
// the deflation is dropped: basis and shift become 0, which the products that add the
// deflation term (here and in the matrix-free bold S) then skip consistently.
__global__ void k_deflate_guard(const int* flag, size_t count, double* QN, double* shift) {
  if (*flag == 0) return;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < count) QN[i] = 0.0;
  if (i == 0) *shift = 0.0;
}

__global__ __launch_bounds__(kT) void k_max_diag(const double* S, int N, int ld, double* out) {
  __shared__ double red[kT];
  double m = 0.0;
  for (int i = threadIdx.x; i < N; i += kT) m = fmax(m, S[(size_t)i * ld + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---- the augmented preconditioner of Section 4.2 (eqs sparse_prec, aug_prec)
// Eliminating x from eq aug_prec (1 x 1 pivots tau^2 (A^T A)_ii, no fill outside the pattern)
// leaves -tau (tau/2 I + B^T (A^T A)^{-1} B), B = A^T (U kron I).  Its block (X, Y) is
// (tau/2) delta_XY I + 1/2 [diag(d_XY) + D_{u_Y} Obar D_{u_X}] with d_XY = Obar (u_X o u_Y),
// supported on the pattern Obar plus the diagonal.  One wavefront per row a writes the row's
// entries of every block pair X >= Y into the zero-filled matrix (row a + n X, column b + n Y).
__global__ __launch_bounds__(256) void k_aug_schur(int n, int k, int nk, const int32_t* rowptr,
                                                   const int32_t* colidx, const double* U,
                                                   const double* d, const double* lam,
                                                   double* S) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (a >= n) return;  // whole wavefront
  const double half_tau = 0.5 * lam[0];
  const int lo = rowptr[a], hi = rowptr[a + 1];
  for (int X = 0; X < k; ++X)
    for (int Y = 0; Y <= X; ++Y) {
      const double dterm = 0.5 * d[(size_t)(X * (X + 1) / 2 + Y) * n + a] +
                           (X == Y ? half_tau : 0.0);
      double* row = S + (size_t)(a + (size_t)n * X) * nk + (size_t)n * Y;
      const double uya = 0.5 * U[(size_t)Y * n + a];
      bool diag_seen = false;
      for (int e = lo + lane; e < hi; e += 64) {
        const int b = colidx[e];
        double v = uya * U[(size_t)X * n + b];
        if (b == a) {
          v += dterm;
          diag_seen = true;
        }
        row[b] = v;
      }
      if (!__any(diag_seen) && lane == 0) row[a] = dterm;
    }
}

__global__ void k_fill(size_t cnt, double* a, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_f64_to_f32(size_t cnt, const double* a, float* b) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = static_cast<float>(a[i]);
}
__global__ void k_f64_to_bf16(size_t cnt, const double* a, uint16_t* b) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = f32_to_bf16_rne(static_cast<float>(a[i]));
}

}  // namespace

size_t work_doubles(int n, int m, int k) {
  const size_t nk = (size_t)n * k;
  return 12 * (size_t)m + 13 * nk + 2 * (size_t)k * k + 8192;
}

Work work_view(const lrsdp_factor* f) {
  Work w;
  const size_t m = f->P->m, nk = f->nk;
  double* b = f->work;
  double** mv[] = {&w.x, &w.r, &w.z, &w.p, &w.q, &w.t0, &w.t1, &w.t2, &w.t3, &w.ylo, &w.dd0, &w.dd1};
  for (auto pp : mv) {
    *pp = b;
    b += m;
  }
  double** kv[] = {&w.w, &w.wl, &w.t, &w.tl, &w.s, &w.sl, &w.y, &w.yl, &w.g0, &w.g1, &w.h, &w.h2, &w.h3};
  for (auto pp : kv) {
    *pp = b;
    b += nk;
  }
  w.kk = b;
  b += 2 * (size_t)f->k * f->k;
  w.part = b;
  return w;
}

int ensure_lowprec(lrsdp_factor* f, int precision, hipStream_t s) {
  lrsdp_ctx* ctx = f->P->ctx;
  const size_t nn = (size_t)f->n * f->n;
  if (precision == LRSDP_PREC_FP32 && !f->W0f) {
    LRSDP_TRY(dev_alloc_n(ctx, &f->W0f, nn));
    f->bytes += nn * sizeof(float);
    k_f64_to_f32<<<grid_for((int64_t)nn, 256), 256, 0, s>>>(nn, f->W0, f->W0f);
    LRSDP_HIP(hipGetLastError());
  }
  if (precision == LRSDP_PREC_BF16 && !f->W0b) {
    LRSDP_TRY(dev_alloc_n(ctx, &f->W0b, nn));
    f->bytes += nn * sizeof(uint16_t);
    k_f64_to_bf16<<<grid_for((int64_t)nn, 256), 256, 0, s>>>(nn, f->W0, f->W0b);
    LRSDP_HIP(hipGetLastError());
  }
  return LRSDP_OK;
}

void factor_release(lrsdp_factor* f) {
  lrsdp_ctx* ctx = f->P->ctx;
  const size_t nn = (size_t)f->n * f->n, nk = f->nk;
  dev_free(ctx, f->lam_dev, (f->k + 1) * sizeof(double));
  dev_free(ctx, f->W, nn * sizeof(double));
  dev_free(ctx, f->W0, nn * sizeof(double));
  dev_free(ctx, f->W0f, nn * sizeof(float));
  dev_free(ctx, f->W0b, nn * sizeof(uint16_t));
  dev_free(ctx, f->U, nk * sizeof(double));
  dev_free(ctx, f->Z, nn * sizeof(double));
  dev_free(ctx, f->Zt, nn * sizeof(double));
  dev_free(ctx, f->Sinv, nk * nk * sizeof(double));
  dev_free(ctx, f->QN, nk * (size_t)f->r * sizeof(double));
  dev_free(ctx, f->work, f->work_doubles * sizeof(double));
  dev_free(ctx, f->sc, 64 * sizeof(double));
  f->lam_dev = f->W = f->W0 = f->U = f->Z = f->Zt = f->Sinv = f->QN = f->work = f->sc = nullptr;
  f->W0f = nullptr;
  f->W0b = nullptr;
}

int export_sinv(const lrsdp_factor* f, double* out, hipStream_t s) {
  lrsdp_ctx* ctx = f->P->ctx;
  const int nk = f->nk;
  double* Lt = nullptr;  // L^{-1} with an explicit zero upper triangle
  LRSDP_TRY(dev_alloc_n(ctx, &Lt, (size_t)nk * nk));
  int rc = LRSDP_OK;
  if (hipMemcpyAsync(Lt, f->Sinv, (size_t)nk * nk * sizeof(double), hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    rc = LRSDP_ERR_DEVICE;
  if (rc == LRSDP_OK) rc = zero_upper(Lt, nk, nk, s);
  // a block-explicit factor: its (2, 1) block holds L21; form (L^{-1})_21 for the export
  double* X = nullptr;
  const size_t xs = f->sinv_split > 0 ? (size_t)(nk - f->sinv_split) * f->sinv_split : 0;
  if (rc == LRSDP_OK && xs) rc = dev_alloc_n(ctx, &X, xs);
  if (rc == LRSDP_OK && xs) rc = binv_full_inverse(Lt, nk, f->sinv_split, nk, X, s);
  if (rc == LRSDP_OK) rc = lauum(Lt, nk, nk, out, nk, s);
  if (rc == LRSDP_OK) rc = mirror_lower(out, nk, nk, s);
  if (hipStreamSynchronize(s) != hipSuccess && rc == LRSDP_OK) rc = LRSDP_ERR_DEVICE;
  dev_free(ctx, X, xs * sizeof(double));
  dev_free(ctx, Lt, (size_t)nk * nk * sizeof(double));
  return rc;
}

// Algorithm 1 step 2 with the augmented preconditioner of Section 4.2: the trailing block of
// eq aug_prec after x is eliminated, divided by -tau, formed from the pattern and factored
// (Cholesky and inverse, as bold S is).  tau, U and W0 are in place.
static int factor_setup_aug(lrsdp_factor* f, std::chrono::steady_clock::time_point t_start) {
  lrsdp_problem* P = f->P;
  lrsdp_ctx* ctx = P->ctx;
  hipStream_t s = ctx->stream;
  const int n = f->n, k = f->k, nk = f->nk;
  hipEvent_t* ev = ctx->phase_ev;
  const int npairs = k * (k + 1) / 2;
  double *Sb = nullptr, *ptmp = nullptr, *dd_ = nullptr;
  const size_t cS = (size_t)nk * nk, cT = std::max<size_t>(1, potrf_inv_tmp_doubles(nk)),
               cD = (size_t)npairs * n;
  int rc = dev_alloc_n(ctx, &Sb, cS);
  if (rc == LRSDP_OK) rc = dev_alloc_n(ctx, &ptmp, cT);
  if (rc == LRSDP_OK) rc = dev_alloc_n(ctx, &dd_, cD);
  auto free_tmp = [&]() {
    (void)hipStreamSynchronize(s);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    dev_free(ctx, Sb, cS * sizeof(double));
    dev_free(ctx, ptmp, cT * sizeof(double));
    dev_free(ctx, dd_, cD * sizeof(double));
  };
  if (rc != LRSDP_OK) {
    free_tmp();
    return rc;
  }
  int* flag_S = ctx->d_flag;
  do {
    if (hipEventRecord(ev[2], s) != hipSuccess) {  // no Z: the phase ends with W0
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    k_fill<<<grid_for((int64_t)cS, 256, 8192), 256, 0, s>>>(cS, Sb, 0.0);
    if (hipMemsetAsync(ctx->d_flag, 0, 3 * sizeof(int), s) != hipSuccess) {  // the flags
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    k_dJL<<<(n + 3) / 4, 256, 0, s>>>(n, k, P->rowptr, P->colidx, f->U, dd_);
    k_aug_schur<<<(n + 3) / 4, 256, 0, s>>>(n, k, nk, P->rowptr, P->colidx, f->U, dd_,
                                           f->lam_dev, Sb);
    if (hipGetLastError() != hipSuccess || hipEventRecord(ev[3], s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    SideStream side;
    if ((rc = ctx_side(ctx, &side))) break;
    if ((rc = potrf_binv(Sb, nk, nk, f->Sinv, nk, flag_S, ptmp, s, &side, &f->sinv_split)))
      break;
    if ((rc = mirror_lower(f->Sinv, nk, nk, s))) break;
    if (hipEventRecord(ev[4], s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    int fl = 0;
    if (hipMemcpyAsync(f->lam.data(), f->lam_dev, (k + 1) * sizeof(double),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&fl, flag_S, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    f->shift = 0.0;
    f->tau = f->lam[0];
    bool finite = true;
    for (double v : f->lam) finite = finite && std::isfinite(v);
    if (!finite) rc = LRSDP_ERR_EIG;
    else if (!(f->tau > 0.0)) rc = LRSDP_ERR_NOT_PD_W;
    else if (fl) rc = LRSDP_ERR_CHOL_S;
    f->tau2 = f->tau * f->tau;
  } while (0);
  free_tmp();
  LRSDP_TRY(rc);
  for (int i = 0; i < 4; ++i) {
    float ms = 0.0f;
    f->phase_ms[i] = hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess ? ms : 0.0;
  }
  auto t_end = std::chrono::steady_clock::now();
  f->setup_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
  return LRSDP_OK;
}

int factor_setup(lrsdp_factor* f, const double* W, const lrsdp_opts& o) {
  auto t_start = std::chrono::steady_clock::now();
  lrsdp_problem* P = f->P;
  lrsdp_ctx* ctx = P->ctx;
  hipStream_t s = ctx->stream;
  const int n = f->n, k = f->k, nk = f->nk;
  const size_t nn = (size_t)n * n;
  const bool aug = o.precond == LRSDP_PRECOND_AUG;
  f->precond = o.precond;
  f->r = (!aug && o.deflate && k >= 2) ? k * (k - 1) / 2 : 0;
  const int r = f->r;

  // persistent buffers
  LRSDP_TRY(dev_alloc_n(ctx, &f->lam_dev, (size_t)k + 1));
  LRSDP_TRY(dev_alloc_n(ctx, &f->W, nn));
  LRSDP_TRY(dev_alloc_n(ctx, &f->W0, nn));
  LRSDP_TRY(dev_alloc_n(ctx, &f->U, (size_t)nk));
  if (!aug) {  // the augmented preconditioner needs no Z
    LRSDP_TRY(dev_alloc_n(ctx, &f->Z, nn));
    LRSDP_TRY(dev_alloc_n(ctx, &f->Zt, nn));
  }
  LRSDP_TRY(dev_alloc_n(ctx, &f->Sinv, (size_t)nk * nk));
  if (r) LRSDP_TRY(dev_alloc_n(ctx, &f->QN, (size_t)nk * r));
  f->work_doubles = work_doubles(n, P->m, k);
  LRSDP_TRY(dev_alloc_n(ctx, &f->work, f->work_doubles));
  LRSDP_TRY(dev_alloc_n(ctx, &f->sc, (size_t)64));
  LRSDP_HIP(hipMemsetAsync(f->sc, 0, 64 * sizeof(double), ctx->stream));  // scalars, counters
  f->bytes = (k + 1 + (aug ? 3 : 5) * nn + (size_t)nk + (size_t)nk * nk + (size_t)nk * r +
              f->work_doubles + 64) * sizeof(double);

  LRSDP_HIP(hipMemcpyAsync(f->W, W, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipEvent_t* ev = ctx->phase_ev;  // phase boundaries, read after the final synchronization
  LRSDP_HIP(hipEventRecord(ev[0], s));

  // ---- 1a: the k largest eigenpairs and tau (temporary workspace).  lam_dev[0] = tau.
  double* Vl = f->U;  // eigenvectors land in U's buffer, scaled in place below
  int rc = LRSDP_ERR_EIG;
  f->eig_sweeps = 0;
  if (o.tau_rule == LRSDP_TAU_MEAN) {
    void* sws = nullptr;
    const size_t swb = spectral_workspace_bytes(n, k);
    LRSDP_TRY(dev_alloc(ctx, &sws, swb));
    int sweeps = 0;
    rc = spectral_top(f->W, n, k, sws, f->lam_dev, Vl, nullptr, 40, nullptr, &sweeps, s);
    dev_free(ctx, sws, swb);  // the pool hands it out again only in stream order
    if (rc == LRSDP_OK) f->eig_sweeps = sweeps;
    else if (rc != LRSDP_ERR_EIG) return rc;
  }
  if (rc != LRSDP_OK) {  // Householder path: exact lambda_min and the k largest pairs
    void* ews = nullptr;
    const size_t ewb = eig_workspace_bytes(n, k);
    LRSDP_TRY(dev_alloc(ctx, &ews, ewb));
    rc = eig_top_and_min(f->W, n, k, ews, f->lam_dev, Vl, s);
    if (rc == LRSDP_OK && o.tau_rule == LRSDP_TAU_MEAN) {
      double* tr = static_cast<double*>(ews);  // eigensolver scratch no longer needed
      rc = trace_dd(f->W, n, tr, s);
      if (rc == LRSDP_OK) k_tau_mean<<<1, 64, 0, s>>>(n, k, tr, f->lam_dev);
    }
    (void)hipStreamSynchronize(s);
    dev_free(ctx, ews, ewb);
  }
  LRSDP_TRY(rc);
  // tau and the eigenvalues are read at the end, with the factorization flags: the steps
  // below take tau from lam_dev (a W that is not positive definite only makes them compute
  // garbage, which is discarded)
  f->lam.assign(k + 1, 0.0);

  // ---- 1b: U, W0, Z
  LRSDP_HIP(hipEventRecord(ev[1], s));
  k_make_U<<<grid_for((int64_t)nk, 256), 256, 0, s>>>(n, k, f->lam_dev, Vl, f->U);
  k_make_W0<<<grid_for((int64_t)nn, 256), 256, 0, s>>>(n, k, f->W, f->U, f->W0, f->Z);
  LRSDP_HIP(hipGetLastError());
  if (aug) return factor_setup_aug(f, t_start);
  // temporaries: inverse diagonal blocks of Z, bold S and the Gram matrix; bold S itself;
  // P_J and the R_JL blocks of its formation
  const int npairs = k * (k + 1) / 2;
  const size_t pair_cap = std::max<size_t>(1, std::min<size_t>(npairs, (size_t)(1u << 28) / nn));
  struct Tmp {
    double* p = nullptr;
    size_t cnt = 0;
  } Zi{nullptr, nn}, ptmp{nullptr, std::max<size_t>(1, potrf_inv_tmp_doubles(nk))},
      Sb{nullptr, (size_t)nk * nk}, PJ{nullptr, (size_t)k * nn},
      Rb{nullptr, std::max(pair_cap * nn, (size_t)nk + 2 * (size_t)r * r)},
      dd_{nullptr, (size_t)npairs * n}, offs{nullptr, 3 * pair_cap},
      Q2{nullptr, std::max<size_t>(1, (size_t)nk * r)};
  Tmp* tmps[] = {&Zi, &ptmp, &Sb, &PJ, &Rb, &dd_, &offs, &Q2};
  for (Tmp* t : tmps) {
    if ((rc = dev_alloc_n(ctx, &t->p, t->cnt)) < 0) break;
  }
  auto free_tmp = [&]() {
    (void)hipStreamSynchronize(s);
    for (Tmp* t : tmps) dev_free(ctx, t->p, t->cnt * sizeof(double));
  };
  if (rc < 0) {
    free_tmp();
    return rc;
  }
  // the flags of the two factorizations are read once, at the end: a failed Z only makes
  // the steps after it compute garbage, which is discarded
  int* flag_S = ctx->d_flag;
  int* flag_Z = ctx->d_flag + 1;
  int* flag_scratch = ctx->d_flag + 2;
  do {
    if (hipMemsetAsync(ctx->d_flag, 0, 3 * sizeof(int), s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    if ((rc = potrf_inv(f->Z, n, n, Zi.p, n, flag_Z, ptmp.p, true, s))) break;
    if ((rc = zero_upper(f->Z, n, n, s))) break;
    if ((rc = transpose(f->Z, n, n, f->Zt, n, s))) break;
    if (hipEventRecord(ev[2], s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }

    // ---- 2: bold S (lower block triangle).  P_J = Obar D_{u_J} Z for every J in one sparse
    //      pass, R_JL = 1/2 (diag(d_JL) Z + D_{u_L} P_J), then batched GEMMs Z^T R_JL.
    double* S = Sb.p;
    {
      ProfMark pm = prof_begin(LRSDP_K_BZ, s);
      k_PJ<<<dim3(n, (n + kT - 1) / kT), kT, 0, s>>>(n, k, P->rowptr, P->colidx, f->U, f->Z, PJ.p);
      k_dJL<<<(n + 3) / 4, 256, 0, s>>>(n, k, P->rowptr, P->colidx, f->U, dd_.p);
      prof_end(pm, s, 8.0 * ((double)k + 1) * nn + 12.0 * P->nnz,
               2.0 * (double)P->nnz * n * k);
    }
    // chunks of pair_cap pairs (R_JL buffers); stream order keeps a chunk's R and offsets
    // from being overwritten before its GEMM has read them
    for (int q0 = 0; q0 < npairs && rc == LRSDP_OK; q0 += (int)pair_cap) {
      const int cnt = std::min<int>((int)pair_cap, npairs - q0);
      k_R_pairs<<<dim3(std::min<int64_t>(grid_for((int64_t)nn, 256), 1024), cnt), 256, 0, s>>>(
          n, nk, q0, f->Z, f->U, PJ.p, dd_.p, Rb.p, reinterpret_cast<int64_t*>(offs.p));
      GemmArgs g;
      g.M = n; g.N = n; g.K = n;
      g.A = f->Z; g.lda = n; g.transA = true;  // op(A) = Z^T, zero below its diagonal
      g.B = Rb.p; g.ldb = n;
      g.C = S; g.ldc = nk;
      g.flags = kKFromRow;
      g.batch = cnt;
      g.offs = reinterpret_cast<const int64_t*>(offs.p);
      rc = gemm(g, s);
    }
    if (rc != LRSDP_OK) break;
    k_add_diag<<<dim3(grid_for(n, 256), k), 256, 0, s>>>(S, n, nk, f->lam_dev);
    // ---- deflation of null(bold U) directions
    if (r) {
      double* Yt = Rb.p;  // k x n: (Z^{-1} U)^T = U Z^{-T}
      // Yt[j][p] = sum_{q <= p} Z^{-1}[p][q] U[j][q]
      if ((rc = rows_k(n, k, Zi.p, 1, f->U, Yt, s))) break;
      double* G = Rb.p + nk;        // r x r Gram matrix
      double* Gi = G + (size_t)r * r;  // the inverse of its Cholesky factor
      k_null_basis<<<grid_for((int64_t)nk * r, 256), 256, 0, s>>>(n, k, r, Yt, f->QN);
      for (int pass = 0; pass < 2 && rc == LRSDP_OK; ++pass) {  // Cholesky QR, twice
        double* Qin = pass == 0 ? f->QN : Q2.p;
        double* Qout = pass == 0 ? Q2.p : f->QN;
        k_gram_cols<<<r * r, kT, 0, s>>>(nk, r, Qin, G);
        if ((rc = potrf_inv(G, r, r, Gi, r, flag_scratch, ptmp.p, true, s))) break;
        GemmArgs h;  // Q <- Q R^{-1} = Q (L^{-1})^T
        h.M = nk; h.N = r; h.K = r;
        h.A = Qin; h.lda = r;
        h.B = Gi; h.ldb = r; h.transB = true;
        h.C = Qout; h.ldc = r;
        h.flags = kKToCol;
        if ((rc = gemm(h, s))) break;
      }
      if (rc) break;
      k_max_diag<<<1, kT, 0, s>>>(S, nk, nk, f->sc);  // the shift, kept on the device
      k_deflate_guard<<<grid_for((int64_t)nk * r, 256), 256, 0, s>>>(flag_scratch,
                                                                    (size_t)nk * r, f->QN, f->sc);
      GemmArgs g;
      g.M = nk; g.N = nk; g.K = r;
      g.A = f->QN; g.lda = r;
      g.B = f->QN; g.ldb = r; g.transB = true;
      g.C = S; g.ldc = nk;
      g.alpha_dev = f->sc; g.beta = 1.0; g.flags = kLowerOut;
      if ((rc = gemm(g, s))) break;
    }
    // ---- L L^T = bold S, then bold S^{-1} = L^{-T} L^{-1}
    // the factor keeps L^{-1} in the lower triangle and L^{-T} in the upper one, so that
    // bold S^{-1} w = L^{-T} (L^{-1} w) is two row-wise triangular GEMVs
    if (hipEventRecord(ev[3], s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    SideStream side;
    if ((rc = ctx_side(ctx, &side))) break;
    if ((rc = potrf_binv(S, nk, nk, f->Sinv, nk, flag_S, ptmp.p, s, &side, &f->sinv_split)))
      break;
    if ((rc = mirror_lower(f->Sinv, nk, nk, s))) break;
    if (hipEventRecord(ev[4], s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    // one host read for tau and the eigenvalues, both flags and the shift
    int fl[2] = {0, 0};
    double shift = 0.0;
    if (hipMemcpyAsync(f->lam.data(), f->lam_dev, (k + 1) * sizeof(double),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(fl, ctx->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        (r && hipMemcpyAsync(&shift, f->sc, sizeof(double), hipMemcpyDeviceToHost, s) !=
                  hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = LRSDP_ERR_DEVICE;
      break;
    }
    f->shift = shift;
    f->tau = f->lam[0];
    bool finite = true;
    for (double v : f->lam) finite = finite && std::isfinite(v);
    if (!finite) rc = LRSDP_ERR_EIG;
    else if (!(f->tau > 0.0)) rc = LRSDP_ERR_NOT_PD_W;
    else if (fl[1]) rc = LRSDP_ERR_CHOL_Z;
    else if (fl[0]) rc = LRSDP_ERR_CHOL_S;
    f->tau2 = f->tau * f->tau;
  } while (0);
  free_tmp();
  LRSDP_TRY(rc);
  for (int i = 0; i < 4; ++i) {
    float ms = 0.0f;
    f->phase_ms[i] = hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess ? ms : 0.0;
  }
  auto t_end = std::chrono::steady_clock::now();
  f->setup_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
  return LRSDP_OK;
}

}  // namespace lrsdp
