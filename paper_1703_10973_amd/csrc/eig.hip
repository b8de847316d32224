// Step A1: W = V Lambda V^T restricted to what Algorithm 1 step 1a consumes:
// tau = lambda_min(W) and the k largest eigenpairs (V_l, Lambda_l) (eqs Wsplit1, Wsplit2).
//
//  1. Householder tridiagonalization Q^T W Q = T, one fused kernel per column j: every
//     block rebuilds column j from the previous reflector (so no separate update pass is
//     needed), forms v_j, and one wavefront per trailing row applies the previous rank-2
//     update and accumulates that row of p_j = tau_j A22 v_j in the same sweep.
//  2. Sturm-count multisection on T (one wavefront per wanted eigenvalue, 64 shifts per
//     round): lambda_min and lambda_{n-k+1..n} to full FP64 accuracy.
//  3. Inverse iteration on T - lambda I (LU with partial pivoting) for the k vectors,
//     then modified Gram-Schmidt among them.
//  4. Back-transformation V_l = H_0 H_1 ... H_{n-3} X, one wavefront per vector.
#include "eig.h"

namespace lrsdp {
namespace {

constexpr int kT = 256;
constexpr int kPart = 256;  // stride of the per-block partial sums (max grid)

// ---------------------------------------------------------------- 1. tridiagonalization
struct TriState {
  int n;
  double* A;      // n x n working copy (full symmetric storage)
  double* V;      // n x n, row j holds v_j on [j+1, n)
  double* P;      // 2 x n, p_j by parity of j
  double* part;   // 2 x G partial sums of p_j . v_j
  double* tau;    // n
  double* d;      // n
  double* e;      // n
};

__global__ __launch_bounds__(kT) void k_tri_step(TriState S, int j, int G, int Gprev) {
  extern __shared__ double sh[];
  const int n = S.n;
  double* vj = sh;          // [n]  v_j (indices >= j+1 used)
  double* wp = sh + n;      // [n]  w_{j-1}
  double* vp = sh + 2 * n;  // [n]  v_{j-1}
  __shared__ double red[kT / kWave];
  __shared__ double bc[4];
  const int t = threadIdx.x;
  const bool has_prev = j > 0;
  const int par = j & 1, ppar = par ^ 1;

  // K_{j-1} = tau_{j-1}/2 * p_{j-1} . v_{j-1}  (fixed-order sum of the previous partials)
  double Kp = 0.0;
  if (has_prev) {
    if (t < kWave) {  // one wavefront sums the partials in a fixed tree order
      double s = 0.0;
      for (int g = t; g < Gprev; g += kWave) s += S.part[ppar * kPart + g];
      s = wave_sum(s);
      if (t == 0) bc[0] = 0.5 * S.tau[j - 1] * s;
    }
    __syncthreads();
    Kp = bc[0];
  }
  // stage v_{j-1}, w_{j-1} on [j, n) and the updated row j
  double nrm2 = 0.0;
  for (int g = j + t; g < n; g += kT) {
    double v = 0.0, w = 0.0;
    if (has_prev) {
      v = S.V[(size_t)(j - 1) * n + g];
      w = S.P[ppar * n + g] - Kp * v;
    }
    vp[g] = v;
    wp[g] = w;
  }
  __syncthreads();
  const double vpj = has_prev ? vp[j] : 0.0, wpj = has_prev ? wp[j] : 0.0;
  for (int g = j + t; g < n; g += kT) {
    double c = S.A[(size_t)j * n + g];
    if (has_prev) c = c - vpj * wp[g] - wpj * vp[g];
    vj[g] = c;  // temporarily the updated row j
    if (g > j) nrm2 = fma(c, c, nrm2);
  }
  nrm2 = block_sum(nrm2, red);
  // Householder reflector for x = c[j+1..n): H x = alpha e1 (LAPACK dlarfg convention)
  if (t == 0) {
    const double x0 = vj[j + 1];
    const double xnorm2 = nrm2 - x0 * x0;  // squared norm of x[1:]
    double alpha, tau, scal;
    if (xnorm2 <= 0.0) {
      alpha = x0;
      tau = 0.0;
      scal = 0.0;
    } else {
      const double nrm = sqrt(nrm2);
      alpha = (x0 >= 0.0) ? -nrm : nrm;
      tau = (alpha - x0) / alpha;
      scal = 1.0 / (x0 - alpha);
    }
    bc[1] = tau;
    bc[2] = scal;
    if (blockIdx.x == 0) {
      S.d[j] = vj[j];
      S.e[j] = alpha;
      S.tau[j] = tau;
    }
  }
  __syncthreads();
  const double tauj = bc[1], scal = bc[2];
  __syncthreads();
  for (int g = j + 1 + t; g < n; g += kT) {
    const double v = (g == j + 1) ? 1.0 : vj[g] * scal;
    vj[g] = v;
    if (blockIdx.x == 0) S.V[(size_t)j * n + g] = v;
  }
  __syncthreads();

  // trailing rows r in [j+1, n): apply update_{j-1}, store, and accumulate p_j[r]
  const int lane = t & (kWave - 1);
  const int gw = blockIdx.x * (kT / kWave) + t / kWave;
  const int nw = G * (kT / kWave);
  double mypart = 0.0;
  for (int r = j + 1 + gw; r < n; r += nw) {
    double* Ar = S.A + (size_t)r * n;
    const double vr = vp[r], wr = wp[r];
    double acc = 0.0;
    for (int c = j + 1 + lane; c < n; c += kWave) {
      double a = Ar[c];
      if (has_prev) a = a - vr * wp[c] - wr * vp[c];
      Ar[c] = a;
      acc = fma(a, vj[c], acc);
    }
    acc = wave_sum(acc);
    const double pr = tauj * acc;
    if (lane == 0) S.P[par * n + r] = pr;
    mypart = fma(pr, vj[r], mypart);
  }
  // mypart is identical across the lanes of a wave; sum one value per wave
  if (lane != 0) mypart = 0.0;
  mypart = block_sum(mypart, red);
  if (t == 0) S.part[par * kPart + blockIdx.x] = mypart;
}

// The last 2 x 2 block after reflector n-3 (or the whole matrix when n == 2).
__global__ void k_tri_final(TriState S, int Gprev) {
  if (threadIdx.x != 0) return;
  const int n = S.n;
  const int j = n - 2;  // pending update index j-1 = n-3 (if n > 2)
  double a00 = S.A[(size_t)j * n + j], a10 = S.A[(size_t)(j + 1) * n + j];
  double a11 = S.A[(size_t)(j + 1) * n + j + 1];
  if (n > 2) {
    const int ppar = (j - 1) & 1;
    double s = 0.0;
    for (int g = 0; g < Gprev; ++g) s += S.part[ppar * kPart + g];
    const double K = 0.5 * S.tau[j - 1] * s;
    const double* v = S.V + (size_t)(j - 1) * n;
    const double w0 = S.P[ppar * n + j] - K * v[j];
    const double w1 = S.P[ppar * n + j + 1] - K * v[j + 1];
    a00 = a00 - 2.0 * v[j] * w0;
    a10 = a10 - v[j + 1] * w0 - w1 * v[j];
    a11 = a11 - 2.0 * v[j + 1] * w1;
  }
  S.d[j] = a00;
  S.d[j + 1] = a11;
  S.e[j] = a10;
  S.tau[j] = 0.0;
  S.tau[j + 1] = 0.0;
}

// ---------------------------------------------------------------- 2. multisection
__device__ int sturm_count(int n, const double* d, const double* e2, double sigma,
                           double pivmin) {
  int cnt = 0;
  double q = d[0] - sigma;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - sigma) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__global__ __launch_bounds__(64) void k_e2(int n, const double* e, double* e2) {
  for (int i = threadIdx.x; i < n - 1; i += 64) e2[i] = e[i] * e[i];
}

// which[w] = index (0-based, ascending) of the eigenvalue wave w computes.
__global__ __launch_bounds__(64) void k_bisect(int n, const double* d, const double* e,
                                               const double* e2, const int* which,
                                               double* lam) {
  const int lane = threadIdx.x;
  const int target = which[blockIdx.x];
  // Gershgorin interval and pivmin (as in LAPACK dstebz)
  double lo = 1e300, hi = -1e300, emax2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i < n - 1) emax2 = fmax(emax2, e2[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    emax2 = fmax(emax2, __shfl_xor(emax2, o));
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double ulp = 2.220446049250313e-16;
  lo -= 2.0 * ulp * tnorm + 2.0 * pivmin;
  hi += 2.0 * ulp * tnorm + 2.0 * pivmin;
  for (int round = 0; round < 40; ++round) {
    const double width = hi - lo;
    if (width <= 2.0 * ulp * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
    const double sigma = lo + width * (double)(lane + 1) / 65.0;
    const int c = sturm_count(n, d, e2, sigma, pivmin);
    // new lo: largest sigma with c <= target; new hi: smallest sigma with c > target
    double cand_lo = (c <= target) ? sigma : -1e300;
    double cand_hi = (c > target) ? sigma : 1e300;
    for (int o = 32; o > 0; o >>= 1) {
      cand_lo = fmax(cand_lo, __shfl_xor(cand_lo, o));
      cand_hi = fmin(cand_hi, __shfl_xor(cand_hi, o));
    }
    if (cand_lo > lo) lo = cand_lo;
    if (cand_hi < hi) hi = cand_hi;
  }
  if (lane == 0) lam[blockIdx.x] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- 3. inverse iteration
// One block per eigenvector.  The LU of T - lambda I with partial pivoting and the solves
// are sequential recurrences, run by lane 0 on arrays kept in LDS (dynamic shared memory,
// 5 n doubles + n ints) when they fit, else in the global scratch `work`.
__global__ __launch_bounds__(64) void k_inverse_iteration(int n, const double* d,
                                                          const double* e, const double* lam,
                                                          int nvec, double* work, int* ipiv_all,
                                                          double* X, int use_lds) {
  extern __shared__ double shm[];
  const int q = blockIdx.x;
  if (q >= nvec) return;
  double* dl = use_lds ? shm : work + (size_t)q * 5 * n;
  double* dd = dl + n;
  double* du = dd + n;
  double* du2 = du + n;
  double* x = du2 + n;
  int* ipiv = use_lds ? reinterpret_cast<int*>(x + n) : ipiv_all + (size_t)q * n;
  const double lm = lam[q];
  const int t = threadIdx.x;
  double tn = 0.0;
  for (int i = t; i < n; i += 64) {
    tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0));
    dd[i] = d[i] - lm;
    dl[i] = (i < n - 1) ? e[i] : 0.0;
    du[i] = dl[i];
    du2[i] = 0.0;
    uint32_t st = 0x9E3779B9u * (uint32_t)(q + 1) + 0x85EBCA6Bu * (uint32_t)(i + 1);
    st ^= st << 13;
    st ^= st >> 17;
    st ^= st << 5;
    x[i] = 0.5 + (double)(st & 0xFFFFF) / (double)0x100000;
  }
  for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o));
  __syncthreads();
  if (t == 0) {
    const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
    for (int i = 0; i < n - 1; ++i) {  // LU with partial pivoting (tridiagonal)
      if (fabs(dd[i]) >= fabs(dl[i])) {
        ipiv[i] = i;
        if (dd[i] == 0.0) dd[i] = tiny;
        const double f = dl[i] / dd[i];
        dl[i] = f;
        dd[i + 1] = dd[i + 1] - f * du[i];
        du2[i] = 0.0;
      } else {
        const double f = dd[i] / dl[i];
        dd[i] = dl[i];
        dl[i] = f;
        const double tmp = du[i];
        du[i] = dd[i + 1];
        dd[i + 1] = tmp - f * dd[i + 1];
        if (i < n - 2) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du[i + 1];
        }
        ipiv[i] = i + 1;
      }
    }
    if (dd[n - 1] == 0.0) dd[n - 1] = tiny;
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i < n - 1; ++i) {
        if (ipiv[i] == i) {
          x[i + 1] = x[i + 1] - dl[i] * x[i];
        } else {
          const double tmp = x[i];
          x[i] = x[i + 1];
          x[i + 1] = tmp - dl[i] * x[i];
        }
      }
      x[n - 1] = x[n - 1] / dd[n - 1];
      if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
      double mx = fmax(fabs(x[n - 1]), n > 1 ? fabs(x[n - 2]) : 0.0);
      for (int i = n - 3; i >= 0; --i) {
        x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
        mx = fmax(mx, fabs(x[i]));
      }
      const double sc = 1.0 / mx;  // rescale against overflow in the next sweep
      for (int i = 0; i < n; ++i) x[i] *= sc;
    }
  }
  __syncthreads();
  double s2 = 0.0;
  for (int i = t; i < n; i += 64) s2 = fma(x[i], x[i], s2);
  s2 = wave_sum(s2);
  const double inv = 1.0 / sqrt(s2);
  for (int i = t; i < n; i += 64) X[(size_t)q * n + i] = x[i] * inv;
}

// Modified Gram-Schmidt among the nvec vectors (rows of X), one block.
__global__ __launch_bounds__(kT) void k_mgs(int n, int nvec, double* X) {
  __shared__ double red[kT / kWave];
  for (int a = 0; a < nvec; ++a) {
    double* xa = X + (size_t)a * n;
    for (int b = 0; b < a; ++b) {
      const double* xb = X + (size_t)b * n;
      double s = 0.0;
      for (int i = threadIdx.x; i < n; i += kT) s = fma(xa[i], xb[i], s);
      s = block_sum(s, red);
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += kT) xa[i] = fma(-s, xb[i], xa[i]);
      __syncthreads();
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) s = fma(xa[i], xa[i], s);
    s = block_sum(s, red);
    const double inv = 1.0 / sqrt(s);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kT) xa[i] *= inv;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- 4. back-transformation
// One wavefront per eigenvector, the vector in LDS; the next reflector's entries are loaded
// into registers while the current one is applied (a reflector touches n - j - 1 entries).
__global__ __launch_bounds__(64) void k_backtransform(int n, const double* V, const double* tau,
                                                      double* X) {
  extern __shared__ double x[];
  constexpr int R = 64;  // register slots per lane: rows up to 64 * 64 = 4096 entries
  const int lane = threadIdx.x;
  double* xg = X + (size_t)blockIdx.x * n;
  for (int i = lane; i < n; i += 64) x[i] = xg[i];
  __syncthreads();
  double vc[R], vn[R];
  auto fetch = [&](int j, double* dst) {
    const double* v = V + (size_t)j * n;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int g = j + 1 + lane + 64 * u;
      dst[u] = (g < n) ? v[g] : 0.0;
    }
  };
  if (n - 3 >= 0) fetch(n - 3, vc);
  for (int j = n - 3; j >= 0; --j) {
    if (j > 0) fetch(j - 1, vn);
    const double tj = tau[j];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int g = j + 1 + lane + 64 * u;
      if (g < n) s = fma(vc[u], x[g], s);
    }
    s = wave_sum(s) * tj;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int g = j + 1 + lane + 64 * u;
      if (g < n) x[g] = fma(-s, vc[u], x[g]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R; ++u) vc[u] = vn[u];
  }
  for (int i = lane; i < n; i += 64) xg[i] = x[i];
}

}  // namespace

size_t eig_workspace_bytes(int n, int k) {
  const int G = 256;
  size_t dbl = (size_t)n * n * 2 + 2 * (size_t)n + 2 * G + 4 * (size_t)n + (size_t)n +
               (size_t)(k + 1) * 6 * n + 64;
  return dbl * sizeof(double) + (size_t)(k + 1) * n * sizeof(int) + 256;
}

int eig_top_and_min(const double* W, int n, int k, void* workspace, double* lam_out,
                    double* Vl_out, hipStream_t s) {
  if (n < 2 || k < 1 || k >= n || n > 4096) return LRSDP_ERR_INVALID_ARG;
  const int G = 256;
  double* base = static_cast<double*>(workspace);
  TriState S;
  S.n = n;
  S.A = base;
  S.V = S.A + (size_t)n * n;
  S.P = S.V + (size_t)n * n;
  S.part = S.P + 2 * (size_t)n;
  S.tau = S.part + 2 * kPart;
  S.d = S.tau + n;
  S.e = S.d + n;
  double* e2 = S.e + n;
  double* work = e2 + n;                      // (k + 1) * 5 n
  double* X = work + (size_t)(k + 1) * 5 * n; // k x n
  int* ipiv = reinterpret_cast<int*>(X + (size_t)(k + 1) * n);
  LRSDP_HIP(hipMemcpyAsync(S.A, W, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  LRSDP_HIP(hipMemsetAsync(S.V, 0, (size_t)n * n * sizeof(double), s));
  const size_t sh = 3 * (size_t)n * sizeof(double);
  int gprev = 0;
  for (int j = 0; j + 2 < n; ++j) {
    const int rows = n - j - 1;
    int g = (rows + (kT / kWave) - 1) / (kT / kWave);
    if (g > G) g = G;
    ProfMark pm = prof_begin(LRSDP_K_TRI, s);
    hipLaunchKernelGGL(k_tri_step, dim3(g), dim3(kT), sh, s, S, j, g, gprev);
    prof_end(pm, s, 16.0 * rows * rows + 24.0 * n, 6.0 * rows * rows);
    gprev = g;
  }
  LRSDP_HIP(hipGetLastError());
  // the final kernel reads the previous step's partials with that step's grid size
  {
    const int jl = n - 3;
    int gl = 1;
    if (jl >= 0) {
      const int rows = n - jl - 1;
      gl = (rows + (kT / kWave) - 1) / (kT / kWave);
      if (gl > G) gl = G;
    }
    k_tri_final<<<1, 64, 0, s>>>(S, gl);
  }
  k_e2<<<1, 64, 0, s>>>(n, S.e, e2);
  // eigenvalue indices: 0 (lambda_min) then n-k .. n-1
  int* which = ipiv;  // reuse: first k+1 ints (ipiv is used after bisection)
  {
    std::vector<int> h(k + 1);
    h[0] = 0;
    for (int q = 0; q < k; ++q) h[q + 1] = n - k + q;
    LRSDP_HIP(hipMemcpyAsync(which, h.data(), (k + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    LRSDP_HIP(hipStreamSynchronize(s));
  }
  k_bisect<<<k + 1, 64, 0, s>>>(n, S.d, S.e, e2, which, lam_out);
  LRSDP_HIP(hipGetLastError());
  {
    const size_t inv_lds = 5 * (size_t)n * sizeof(double) + (size_t)n * sizeof(int);
    const int use_lds = inv_lds <= 150 * 1024 ? 1 : 0;
    k_inverse_iteration<<<k, 64, use_lds ? inv_lds : 0, s>>>(n, S.d, S.e, lam_out + 1, k, work,
                                                            ipiv, X, use_lds);
  }
  k_mgs<<<1, kT, 0, s>>>(n, k, X);
  k_backtransform<<<k, 64, (size_t)n * sizeof(double), s>>>(n, S.V, S.tau, X);
  LRSDP_HIP(hipGetLastError());
  LRSDP_HIP(hipMemcpyAsync(Vl_out, X, (size_t)k * n * sizeof(double), hipMemcpyDeviceToDevice,
                           s));
  return LRSDP_OK;
}

}  // namespace lrsdp
