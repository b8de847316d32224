// Steps A6 and A7: products with bold U = A^T (U kron Z) and the preconditioner.
//
// eq Umv:  bold U vec X = [A_i . (Z X U^T)]_i,  bold U^T y = vec(Z^T mat(A y) U)
// eq SMW2: H~^{-1} v = (tau^2 A^T A)^{-1} (v - bold U bold S^{-1} bold U^T (A^T A)^{-1} v)
// eq hessExp1 (split product): H v = A^T vec(W0 M W0) + A^T vec(U P^T W0 + W0 P U^T + U K U^T),
//   P = M U, K = U^T M U, M = mat(A v).
//
// n x k operands are stored column-major (k rows of n), which is also the nk layout of
// bold S (index p + n j).  Double-double variants carry w = bold U^T G^{-1} v (its sparse
// product M U) and t = bold S^{-1} w (FP64 inverse plus residual refinement against the
// matrix-free bold S) in extended precision, which keeps H~^{-1} positive definite when
// tau ~ 1e-8 makes the FP64 Sherman-Morrison-Woodbury form unstable.
#include "dense.h"

namespace lrsdp {
namespace {

constexpr int KMAX = 16;
constexpr int kT = 256;

// ---------------------------------------------------------------- M U (sparse x n x k)
// out[j][p] = sum_{e in row p} M_e U[j][col e], M_e = val_i * (scale_i * v_i) formed on the
// fly (i = src[e], scale = 1/g when ginv != nullptr).  Sixteen lanes share a row (fixed
// lane-to-entry map, then an xor-shuffle tree), so the summation order is fixed.
constexpr int kRL = 16;

// Reduce-scatter of K2 per-lane sums over groups of kRL lanes (K2 <= kRL, both powers of two):
// at the exchange across lane bit o the lower lanes keep the first half of the sums they carry
// and the upper lanes the second half, each adding its partner's copy, until every sub-group
// of kRL / K2 lanes carries one sum (sum index = (lane % kRL) / (kRL / K2)); butterflies finish
// the sub-groups.  Each sum pairs the same lanes in the same order as a butterfly of its own,
// with K2 - 1 + log2(kRL / K2) additions instead of K2 log2(kRL).
// one exchange level: H sums kept out of 2H, across lane bit O (compile-time, so every index
// into the accumulators is a constant and they stay in registers)
template <int H, int O, int K2>
__device__ __forceinline__ void rs_level(double (&acc)[K2], int sub) {
  if constexpr (H >= 1) {
    const bool upper = (sub & O) != 0;
#pragma unroll
    for (int s = 0; s < H; ++s) {
      const double send = upper ? acc[s] : acc[H + s];
      const double keep = upper ? acc[H + s] : acc[s];
      acc[s] = keep + __shfl_xor(send, O, kRL);
    }
    rs_level<H / 2, O / 2, K2>(acc, sub);
  }
}

template <int H, int O, int K2>
__device__ __forceinline__ void rs_level(dd (&acc)[K2], int sub) {
  if constexpr (H >= 1) {
    const bool upper = (sub & O) != 0;
#pragma unroll
    for (int s = 0; s < H; ++s) {
      const double sh = upper ? acc[s].hi : acc[H + s].hi;
      const double sl = upper ? acc[s].lo : acc[H + s].lo;
      const dd keep = {upper ? acc[H + s].hi : acc[s].hi, upper ? acc[H + s].lo : acc[s].lo};
      acc[s] = dd_add(keep, {__shfl_xor(sh, O, kRL), __shfl_xor(sl, O, kRL)});
    }
    rs_level<H / 2, O / 2, K2>(acc, sub);
  }
}

template <int K2>
__device__ __forceinline__ double group_reduce_scatter(double (&acc)[K2], int sub) {
  static_assert((K2 & (K2 - 1)) == 0 && K2 <= kRL, "K2 a power of two, at most kRL");
  rs_level<K2 / 2, kRL / 2, K2>(acc, sub);
  double v = acc[0];
#pragma unroll
  for (int o = kRL / K2 / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kRL);
  return v;
}

template <int K2>
__device__ __forceinline__ dd group_reduce_scatter(dd (&acc)[K2], int sub) {
  static_assert((K2 & (K2 - 1)) == 0 && K2 <= kRL, "K2 a power of two, at most kRL");
  rs_level<K2 / 2, kRL / 2, K2>(acc, sub);
  dd v = acc[0];
#pragma unroll
  for (int o = kRL / K2 / 2; o > 0; o >>= 1)
    v = dd_add(v, {__shfl_xor(v.hi, o, kRL), __shfl_xor(v.lo, o, kRL)});
  return v;
}

template <int K2>
__device__ __forceinline__ void spmm_U_body(int bx, int n, int k,
                                            const int32_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ colidx,
                                            const int32_t* __restrict__ src,
                                            const double* __restrict__ val,
                                            const double* __restrict__ ginv,
                                            const double* __restrict__ v,
                                            const double* __restrict__ U,
                                            double* __restrict__ out) {
  const int p = bx * (kT / kRL) + threadIdx.x / kRL;
  const int sub = threadIdx.x & (kRL - 1);
  const bool live = p < n;
  double acc[K2];
#pragma unroll
  for (int j = 0; j < K2; ++j) acc[j] = 0.0;
  if (live) {
    const int hi = rowptr[p + 1];
    for (int e = rowptr[p] + sub; e < hi; e += kRL) {
      const int q = colidx[e];
      const int i = src[e];
      const double mv = val[i] * (ginv ? v[i] * ginv[i] : v[i]);
#pragma unroll
      for (int j = 0; j < K2; ++j)
        if (j < k) acc[j] = fma(mv, U[(size_t)j * n + q], acc[j]);
    }
  }
  const double r = group_reduce_scatter<K2>(acc, sub);
  const int j = sub / (kRL / K2);
  if (live && sub % (kRL / K2) == 0 && j < k) out[(size_t)j * n + p] = r;
}
template <int K2>
__global__ __launch_bounds__(kT) void k_spmm_U(int n, int k, const int32_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ colidx,
                                               const int32_t* __restrict__ src,
                                               const double* __restrict__ val,
                                               const double* __restrict__ ginv,
                                               const double* __restrict__ v,
                                               const double* __restrict__ U,
                                               double* __restrict__ out) {
  spmm_U_body<K2>(blockIdx.x, n, k, rowptr, colidx, src, val, ginv, v, U, out);
}

// double-double version: M_e = (vh_i + vl_i) * scale_i * val_i, each product in double-double
template <int K2>
__device__ __forceinline__ void spmm_U_dd_body(int bx, int n, int k,
                                               const int32_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ colidx,
                                               const int32_t* __restrict__ src,
                                               const double* __restrict__ val,
                                               const double* __restrict__ ginv,
                                               const double* __restrict__ vh,
                                               const double* __restrict__ vl,
                                               const double* __restrict__ U,
                                               double* __restrict__ oh,
                                               double* __restrict__ ol) {
  const int p = bx * (kT / kRL) + threadIdx.x / kRL;
  const int sub = threadIdx.x & (kRL - 1);
  const bool live = p < n;
  dd acc[K2];
#pragma unroll
  for (int j = 0; j < K2; ++j) acc[j] = {0.0, 0.0};
  if (live) {
    const int hi = rowptr[p + 1];
    for (int e = rowptr[p] + sub; e < hi; e += kRL) {
      const int q = colidx[e];
      const int i = src[e];
      dd u = {vh[i], vl ? vl[i] : 0.0};
      if (ginv) u = dd_mul_d(u, ginv[i]);
      u = dd_mul_d(u, val[i]);
#pragma unroll
      for (int j = 0; j < K2; ++j)
        if (j < k) acc[j] = dd_fma2(acc[j], U[(size_t)j * n + q], u.hi, u.lo);
    }
  }
  const dd r = group_reduce_scatter<K2>(acc, sub);
  const int j = sub / (kRL / K2);
  if (live && sub % (kRL / K2) == 0 && j < k) {
    oh[(size_t)j * n + p] = r.hi;
    ol[(size_t)j * n + p] = r.lo;
  }
}
template <int K2>
__global__ __launch_bounds__(kT) void k_spmm_U_dd(int n, int k,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colidx,
                                                  const int32_t* __restrict__ src,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ ginv,
                                                  const double* __restrict__ vh,
                                                  const double* __restrict__ vl,
                                                  const double* __restrict__ U,
                                                  double* __restrict__ oh,
                                                  double* __restrict__ ol) {
  spmm_U_dd_body<K2>(blockIdx.x, n, k, rowptr, colidx, src, val, ginv, vh, vl, U, oh, ol);
}

// out = M U with M = mat(A (ginv o v)) (ginv may be nullptr)
int spmm_U(const lrsdp_problem* P, int k, const double* ginv, const double* v, const double* U,
           double* out, hipStream_t s) {
  const int grid = (P->n + kT / kRL - 1) / (kT / kRL);
#define LRSDP_SPMM(K2_)                                                                    \
  k_spmm_U<K2_><<<grid, kT, 0, s>>>(P->n, k, P->rowptr, P->colidx, P->src, P->val, ginv, v, U, \
                                    out)
  if (k <= 2) LRSDP_SPMM(2);
  else if (k <= 4) LRSDP_SPMM(4);
  else if (k <= 8) LRSDP_SPMM(8);
  else LRSDP_SPMM(16);
#undef LRSDP_SPMM
  return LRSDP_OK;
}
// (oh, ol) = M U in double-double, M = mat(A G^{-1} (vh + vl)) (ginv, vl may be nullptr)
int spmm_U_dd(const lrsdp_problem* P, int k, const double* ginv, const double* vh,
              const double* vl, const double* U, double* oh, double* ol, hipStream_t s) {
  const int grid = (P->n + kT / kRL - 1) / (kT / kRL);
#define LRSDP_SPMM_DD(K2_)                                                                   \
  k_spmm_U_dd<K2_><<<grid, kT, 0, s>>>(P->n, k, P->rowptr, P->colidx, P->src, P->val, ginv, vh, \
                                       vl, U, oh, ol)
  if (k <= 2) LRSDP_SPMM_DD(2);
  else if (k <= 4) LRSDP_SPMM_DD(4);
  else if (k <= 8) LRSDP_SPMM_DD(8);
  else LRSDP_SPMM_DD(16);
#undef LRSDP_SPMM_DD
  return LRSDP_OK;
}

// ---------------------------------------------------------------- dense n x n times n x k
// out[j][p] = sum_{q in range(p)} A[p][q] X[j][q]; range: 0 full, 1 q <= p, 2 q >= p.
// (FP64: k_rows_kr below.)  The double-double form takes one workgroup per row p: its four
// wavefronts split the row and every load of a thread is in flight at once.  Each wavefront
// then reduces its K2 column sums (k padded to K2) by a reduce-scatter butterfly: at the
// exchange across lane bit o, the lower lanes keep the first half of the columns they carry
// and the upper lanes the second half, each adding its partner's copy, until every group of
// 64 / K2 lanes carries one column (column = lane / (64 / K2)); plain butterflies finish the
// groups.  That is K2 - 1 + log2(64 / K2) double-double additions per wavefront instead of
// 6 k.  The four wavefronts' sums meet in a fixed order.
template <int K2>
__global__ __launch_bounds__(kT) void k_rows_k_dd(int n, int k, const double* __restrict__ A,
                                                  int range, const double* __restrict__ Xh,
                                                  const double* __restrict__ Xl,
                                                  double* __restrict__ oh,
                                                  double* __restrict__ ol, double c,
                                                  const double* __restrict__ th,
                                                  const double* __restrict__ tl) {
  static_assert(K2 >= 2 && K2 <= 16 && (K2 & (K2 - 1)) == 0, "K2 a power of two");
  constexpr int G = kWave / K2;  // lanes per column after the scatter
  __shared__ double red[kT / kWave][K2][2];
  const int p = blockIdx.x, t = threadIdx.x;
  const int lane = t & (kWave - 1), wid = t / kWave;
  const int qlo = (range == 2) ? p : 0;
  const int qhi = (range == 1) ? p + 1 : n;
  const double* a = A + (size_t)p * n;
  dd acc[K2];
#pragma unroll
  for (int j = 0; j < K2; ++j) acc[j] = {0.0, 0.0};
#pragma unroll 2
  for (int q = qlo + t; q < qhi; q += kT) {
    const double av = a[q];
#pragma unroll
    for (int j = 0; j < K2; ++j)
      if (j < k)
        acc[j] = dd_fma2(acc[j], av, Xh[(size_t)j * n + q], Xl ? Xl[(size_t)j * n + q] : 0.0);
  }
  // reduce-scatter: slot s of a lane holds the s-th column of the range it carries
#pragma unroll
  for (int o = kWave / 2, h = K2 / 2; h >= 1; o >>= 1, h >>= 1) {
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int s = 0; s < h; ++s) {
      const dd send = upper ? acc[s] : acc[h + s];
      const dd keep = upper ? acc[h + s] : acc[s];
      acc[s] = dd_add(keep, shfl_xor_dd(send, o));
    }
  }
  dd v = acc[0];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = dd_add(v, shfl_xor_dd(v, o));
  const int col = lane / G;
  if (lane % G == 0) {
    red[wid][col][0] = v.hi;
    red[wid][col][1] = v.lo;
  }
  __syncthreads();
  if (t < k) {
    dd u = dd_add({red[0][t][0], red[0][t][1]}, {red[1][t][0], red[1][t][1]});
    const dd w = dd_add({red[2][t][0], red[2][t][1]}, {red[3][t][0], red[3][t][1]});
    u = dd_add(u, w);
    if (th) u = dd_add(u, dd_mul_d({th[(size_t)t * n + p], tl[(size_t)t * n + p]}, c));
    oh[(size_t)t * n + p] = u.hi;
    ol[(size_t)t * n + p] = u.lo;
  }
}

// ---------------------------------------------------------------- sampled products
// z_i = (v_i - x_i) ginv_i / tau^2,  x_i = (coef_i / 2)(Y_a . U_b + Y_b . U_a)  [= (bold U t)_i]
__device__ __forceinline__ void smw_out_body(int bx, int m, int n, int k, const int32_t* a,
                                             const int32_t* b, const double* coef,
                                             const double* ginv, double inv_tau2,
                                             const double* Y, const double* U, const double* v,
                                             double* z) {
  const int i = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (i >= m) return;
  const int ai = a[i], bi = b[i];
  double s = 0.0;
  for (int j = 0; j < k; ++j) {
    const double* y = Y + (size_t)j * n;
    const double* u = U + (size_t)j * n;
    s = fma(y[ai], u[bi], s);
    s = fma(y[bi], u[ai], s);
  }
  const double x = 0.5 * coef[i] * s;
  z[i] = (v[i] - x) * ginv[i] * inv_tau2;
}
__global__ __launch_bounds__(256) void k_smw_out(int m, int n, int k, const int32_t* a,
                                                 const int32_t* b, const double* coef,
                                                 const double* ginv, double inv_tau2,
                                                 const double* Y, const double* U,
                                                 const double* v, double* z) {
  smw_out_body(blockIdx.x, m, n, k, a, b, coef, ginv, inv_tau2, Y, U, v, z);
}

// x_i = (coef_i / 2)(Y_a . U_b + Y_b . U_a) in double-double; optional z = (v - x) g^{-1}/tau^2
__global__ void k_sampled_dd(int m, int n, int k, const int32_t* a, const int32_t* b,
                             const double* coef, const double* Yh, const double* Yl,
                             const double* U, double* xh, double* xl, const double* v,
                             const double* ginv, double inv_tau2, double* z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int ai = a[i], bi = b[i];
  dd s = {0.0, 0.0};
  for (int j = 0; j < k; ++j) {
    const size_t o = (size_t)j * n;
    s = dd_fma2(s, U[o + bi], Yh[o + ai], Yl[o + ai]);
    s = dd_fma2(s, U[o + ai], Yh[o + bi], Yl[o + bi]);
  }
  s = dd_mul_d(s, 0.5 * coef[i]);
  if (z) {
    dd d = dd_add_d({-s.hi, -s.lo}, v[i]);
    z[i] = (d.hi + d.lo) * ginv[i] * inv_tau2;
  } else {
    xh[i] = s.hi;
    xl[i] = s.lo;
  }
}

// y <- y * ginv in double-double (in place)
__global__ void k_scale_dd(int m, const double* ginv, double* yh, double* yl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  dd u = dd_mul_d({yh[i], yl[i]}, ginv[i]);
  yh[i] = u.hi;
  yl[i] = u.lo;
}

// K = U^T P (k x k) in double-double, then symmetrized and rounded: one workgroup per (j, l).
__device__ __forceinline__ void UtP_body(int bx, int n, int k, const double* U, const double* Ph,
                                         const double* Pl, double* Kdd) {
  __shared__ double scr[2 * kT / kWave];
  const int j = bx / k, l = bx % k;
  dd s = {0.0, 0.0};
  for (int p = threadIdx.x; p < n; p += kT)
    s = dd_fma2(s, U[(size_t)j * n + p], Ph[(size_t)l * n + p], Pl[(size_t)l * n + p]);
  s = block_sum_dd(s, scr);
  if (threadIdx.x == 0) {
    Kdd[2 * (j * k + l)] = s.hi;
    Kdd[2 * (j * k + l) + 1] = s.lo;
  }
}
__global__ __launch_bounds__(kT) void k_UtP(int n, int k, const double* U, const double* Ph,
                                            const double* Pl, double* Kdd) {
  UtP_body(blockIdx.x, n, k, U, Ph, Pl, Kdd);
}

// Hv_i += coef_i [ sum_j (U_ja Q_jb + Q_ja U_jb) + U_a^T Ks U_b ],  Ks = (K + K^T) / 2
__device__ __forceinline__ void lowrank_add_body(int bx, int m, int n, int k, const int32_t* a,
                                                 const int32_t* b, const double* coef,
                                                 const double* U, const double* Q,
                                                 const double* Kdd, double* Hv) {
  const int i = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (i >= m) return;
  const int ai = a[i], bi = b[i];
  double s = 0.0;
  for (int j = 0; j < k; ++j) {
    const size_t o = (size_t)j * n;
    s = fma(U[o + ai], Q[o + bi], s);
    s = fma(Q[o + ai], U[o + bi], s);
  }
  double t = 0.0;
  for (int j = 0; j < k; ++j) {
    double kr = 0.0;
    for (int l = 0; l < k; ++l) {
      const double kjl = Kdd[2 * (j * k + l)] + Kdd[2 * (j * k + l) + 1];
      const double klj = Kdd[2 * (l * k + j)] + Kdd[2 * (l * k + j) + 1];
      kr = fma(0.5 * (kjl + klj), U[(size_t)l * n + bi], kr);
    }
    t = fma(U[(size_t)j * n + ai], kr, t);
  }
  Hv[i] += coef[i] * (s + t);
}
__global__ __launch_bounds__(256) void k_lowrank_add(int m, int n, int k, const int32_t* a,
                                                     const int32_t* b, const double* coef,
                                                     const double* U, const double* Q,
                                                     const double* Kdd, double* Hv) {
  lowrank_add_body(blockIdx.x, m, n, k, a, b, coef, U, Q, Kdd, Hv);
}

// ---------------------------------------------------------------- nk-vector helpers
// out = h + l rounded to FP64; zero[i] = 0 when zero is given
__global__ void k_dd_combine(int N, const double* h, const double* l, double* out,
                             double* zero) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    out[i] = h[i] + l[i];
    if (zero) zero[i] = 0.0;
  }
}
// (ah, al) - (bh, bl) rounded to FP64
__global__ void k_dd_sub_round(int N, const double* ah, const double* al, const double* bh,
                               const double* bl, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  dd d = dd_add({ah[i], al[i]}, {-bh[i], -bl[i]});
  out[i] = d.hi + d.lo;
}
// (th, tl) += d
__global__ void k_dd_accum(int N, double* th, double* tl, const double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  dd u = dd_add_d({th[i], tl[i]}, d[i]);
  th[i] = u.hi;
  tl[i] = u.lo;
}
// c = Q^T t  (r values, double-double), one workgroup per column of Q (nk x r row-major)
__global__ __launch_bounds__(kT) void k_Qt_dd(int N, int r, const double* Q, const double* th,
                                              const double* tl, double* c) {
  __shared__ double scr[2 * kT / kWave];
  const int col = blockIdx.x;
  dd s = {0.0, 0.0};
  for (int i = threadIdx.x; i < N; i += kT) s = dd_fma2(s, Q[(size_t)i * r + col], th[i], tl[i]);
  s = block_sum_dd(s, scr);
  if (threadIdx.x == 0) {
    c[2 * col] = s.hi;
    c[2 * col + 1] = s.lo;
  }
}
// s += shift * Q c  (double-double)
__global__ void k_Qc_dd(int N, int r, double shift, const double* Q, const double* c, double* sh,
                        double* sl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  dd acc = {0.0, 0.0};
  for (int q = 0; q < r; ++q) acc = dd_fma2(acc, Q[(size_t)i * r + q], c[2 * q], c[2 * q + 1]);
  acc = dd_mul_d(acc, shift);
  dd u = dd_add({sh[i], sl[i]}, acc);
  sh[i] = u.hi;
  sl[i] = u.lo;
}

// out[j][p] = sum_{q in range(p)} A[p][q] X[j][q] for R rows p per workgroup: every X value
// loaded serves R rows, so X (k x n, L2-resident) is read n / R times instead of n times.
// KC >= k bounds the accumulators; rows past n and q outside a row's range add nothing.
// With tadd != nullptr the result is fma(c, tadd, product) (an axpy folded in).
template <int R, int KC>
__device__ __forceinline__ void rows_kr_body(int bx, int n, int k, const double* __restrict__ A,
                                             int range, const double* __restrict__ X,
                                             double* __restrict__ out, double c,
                                             const double* __restrict__ tadd) {
  __shared__ double red[kT / kWave][R * KC];
  const int p0 = bx * R, t = threadIdx.x;
  const int lane = t & (kWave - 1), wid = t / kWave;
  int lo[R], hi[R];
  int qlo = n, qhi = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = p0 + r;
    lo[r] = (range == 2) ? p : 0;
    hi[r] = p >= n ? 0 : (range == 1) ? p + 1 : n;
    if (hi[r] > lo[r]) {
      qlo = min(qlo, lo[r]);
      qhi = max(qhi, hi[r]);
    }
  }
  double acc[R][KC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < KC; ++j) acc[r][j] = 0.0;
  constexpr int U = 4;  // columns per thread in flight at once
  for (int q0 = qlo + t; q0 < qhi; q0 += U * kT) {
    double xv[U][KC], av[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * kT;
#pragma unroll
      for (int j = 0; j < KC; ++j) xv[u][j] = (q < qhi && j < k) ? X[(size_t)j * n + q] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        av[u][r] = (q >= lo[r] && q < hi[r]) ? A[(size_t)(p0 + r) * n + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[r][j] = fma(av[u][r], xv[u][j], acc[r][j]);
  }
  // reduce-scatter over the S = R KC sums (slot r KC + j): at the exchange across lane bit o the
  // lower lanes keep the first half of the slots they carry and the upper lanes the second half,
  // each adding its partner's copy, until every group of 64 / S lanes carries one slot; plain
  // butterflies finish the groups.  Each slot's sum pairs the same lanes in the same order as a
  // butterfly of its own, with S - 1 + log2(64 / S) additions per wavefront instead of 6 R k.
  constexpr int S = R * KC, G = kWave / S;
  static_assert((S & (S - 1)) == 0 && S <= kWave, "R KC a power of two, at most 64");
  double* sl = &acc[0][0];
#pragma unroll
  for (int o = kWave / 2, h = S / 2; h >= 1; o >>= 1, h >>= 1) {
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int s = 0; s < h; ++s) {
      const double send = upper ? sl[s] : sl[h + s];
      const double keep = upper ? sl[h + s] : sl[s];
      sl[s] = keep + __shfl_xor(send, o, kWave);
    }
  }
  double v = sl[0];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  if (lane % G == 0) red[wid][lane / G] = v;
  __syncthreads();
  if (t < R * KC) {
    const int r = t / KC, j = t - r * KC, p = p0 + r;
    if (p < n && j < k) {
      const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
      out[(size_t)j * n + p] = tadd ? fma(c, tadd[(size_t)j * n + p], v) : v;
    }
  }
}
template <int R, int KC>
__global__ __launch_bounds__(kT) void k_rows_kr(int n, int k, const double* __restrict__ A,
                                                int range, const double* __restrict__ X,
                                                double* __restrict__ out, double c,
                                                const double* __restrict__ tadd) {
  rows_kr_body<R, KC>(blockIdx.x, n, k, A, range, X, out, c, tadd);
}

}  // namespace

int rows_k_axpy(int n, int k, const double* A, int range, const double* X, double* out,
                double c, const double* tadd, hipStream_t s) {
  if (n <= 0 || k <= 0) return LRSDP_OK;
  if (k > KMAX) return LRSDP_ERR_INVALID_ARG;
  constexpr int R = 4;
  const int grid = (n + R - 1) / R;
  if (k <= 4) k_rows_kr<R, 4><<<grid, kT, 0, s>>>(n, k, A, range, X, out, c, tadd);
  else if (k <= 8) k_rows_kr<R, 8><<<grid, kT, 0, s>>>(n, k, A, range, X, out, c, tadd);
  else k_rows_kr<R, 16><<<grid, kT, 0, s>>>(n, k, A, range, X, out, c, tadd);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int rows_k(int n, int k, const double* A, int range, const double* X, double* out,
           hipStream_t s) {
  return rows_k_axpy(n, k, A, range, X, out, 0.0, nullptr, s);
}

namespace {

// (oh, ol) = rows of A times X in double-double; with th != nullptr, + c (th, tl)
int rows_k_dd(int n, int k, const double* A, int range, const double* Xh, const double* Xl,
              double* oh, double* ol, hipStream_t s, double c = 0.0,
              const double* th = nullptr, const double* tl = nullptr) {
  if (k <= 2) k_rows_k_dd<2><<<n, kT, 0, s>>>(n, k, A, range, Xh, Xl, oh, ol, c, th, tl);
  else if (k <= 4) k_rows_k_dd<4><<<n, kT, 0, s>>>(n, k, A, range, Xh, Xl, oh, ol, c, th, tl);
  else if (k <= 8) k_rows_k_dd<8><<<n, kT, 0, s>>>(n, k, A, range, Xh, Xl, oh, ol, c, th, tl);
  else k_rows_k_dd<16><<<n, kT, 0, s>>>(n, k, A, range, Xh, Xl, oh, ol, c, th, tl);
  return LRSDP_OK;
}

// bold S t in double-double (deflated as factored), t = (th, tl) -> (sh, sl).
int schur_apply_dd(const lrsdp_factor* f, const double* th, const double* tl, double* sh,
                   double* sl, hipStream_t s) {
  const lrsdp_problem* P = f->P;
  const Work w = work_view(f);
  const int n = f->n, k = f->k, m = P->m, nk = f->nk;
  // a. Y = Z T (dd)        b. y = bold U t (dd)
  rows_k_dd(n, k, f->Z, 1, th, tl, w.y, w.yl, s);
  k_sampled_dd<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, w.y, w.yl, f->U,
                                                 w.t0, w.t1, nullptr, nullptr, 0.0, nullptr);
  // c. mat(A G^{-1} y) (dd)   d. P = M U (dd)   e. s = Z^T P (dd)
  spmm_U_dd(P, k, P->ginv, w.t0, w.t1, f->U, w.y, w.yl, s);
  // f. s = Z^T P + tau^2 t (one launch), + shift Q (Q^T t)
  rows_k_dd(n, k, f->Zt, 2, w.y, w.yl, sh, sl, s, f->tau2, th, tl);
  if (f->r) {
    k_Qt_dd<<<f->r, kT, 0, s>>>(nk, f->r, f->QN, th, tl, w.kk);
    k_Qc_dd<<<grid_for(nk, 256), 256, 0, s>>>(nk, f->r, f->shift, f->QN, w.kk, sh, sl);
  }
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

// ---------------------------------------------------------------- FP64 matrix-free bold S
// x_i = scale_i (coef_i / 2)(Y_a . U_b + Y_b . U_a)   [= scale_i (bold U t)_i]
__device__ __forceinline__ void sampled_f64_body(int bx, int m, int n, int k, const int32_t* a,
                                                 const int32_t* b, const double* coef,
                                                 const double* scale, const double* Y,
                                                 const double* U, double* x) {
  const int i = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (i >= m) return;
  const int ai = a[i], bi = b[i];
  double s = 0.0;
  for (int j = 0; j < k; ++j) {
    const size_t o = (size_t)j * n;
    s = fma(Y[o + ai], U[o + bi], s);
    s = fma(Y[o + bi], U[o + ai], s);
  }
  x[i] = 0.5 * coef[i] * s * (scale ? scale[i] : 1.0);
}
__global__ __launch_bounds__(256) void k_sampled_f64(int m, int n, int k, const int32_t* a,
                                                     const int32_t* b, const double* coef,
                                                     const double* scale, const double* Y,
                                                     const double* U, double* x) {
  sampled_f64_body(blockIdx.x, m, n, k, a, b, coef, scale, Y, U, x);
}
__device__ __forceinline__ void Qt_body(int bx, int N, int r, const double* Q, const double* t,
                                        double* c) {
  __shared__ double scr[kT / kWave];
  const int col = bx;
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += kT) s = fma(Q[(size_t)i * r + col], t[i], s);
  s = block_sum(s, scr);
  if (threadIdx.x == 0) c[col] = s;
}
__global__ __launch_bounds__(kT) void k_Qt(int N, int r, const double* Q, const double* t,
                                           double* c) {
  Qt_body(blockIdx.x, N, r, Q, t, c);
}
__device__ __forceinline__ void Qc_body(int bx, int N, int r, double shift, const double* Q,
                                        const double* c, double* s) {
  const int i = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (i >= N) return;
  double acc = 0.0;
  for (int q = 0; q < r; ++q) acc = fma(Q[(size_t)i * r + q], c[q], acc);
  s[i] = fma(shift, acc, s[i]);
}
__global__ __launch_bounds__(256) void k_Qc(int N, int r, double shift, const double* Q,
                                            const double* c, double* s) {
  Qc_body(blockIdx.x, N, r, shift, Q, c, s);
}

// s = bold S t in FP64 (deflated as factored), matrix-free through eq Umv.
int schur_apply_f64(const lrsdp_factor* f, const double* t, double* sout, hipStream_t s) {
  const lrsdp_problem* P = f->P;
  const Work w = work_view(f);
  const int n = f->n, k = f->k, m = P->m, nk = f->nk;
  rows_k(n, k, f->Z, 1, t, w.y, s);                                        // Z T
  k_sampled_f64<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, P->ginv, w.y,
                                                  f->U, w.t0);             // G^{-1} bold U t
  spmm_U(P, k, nullptr, w.t0, f->U, w.y, s);
  rows_k_axpy(n, k, f->Zt, 2, w.y, sout, f->tau2, t, s);  // Z^T M U + tau^2 t
  if (f->r) {
    k_Qt<<<f->r, kT, 0, s>>>(nk, f->r, f->QN, t, w.kk);
    k_Qc<<<grid_for(nk, 256), 256, 0, s>>>(nk, f->r, f->shift, f->QN, w.kk, sout);
  }
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

}  // namespace

// refine != 0: one step of FP64 residual refinement of t = bold S^{-1} w against the
// matrix-free bold S.  The explicit inverse alone acts like the inverse of a matrix off by
// ~u kappa(bold S) ||bold S||; after one step the error is that of a backward-stable solve,
// ~u ||bold S||, which keeps H~^{-1} positive definite while tau^2 >> u ||bold S||.
int precond_apply_f64(const lrsdp_factor* f, const double* v, double* z, hipStream_t s,
                      int refine) {
  const lrsdp_problem* P = f->P;
  const Work w = work_view(f);
  const int n = f->n, k = f->k, m = P->m, nk = f->nk;
  if (k > KMAX) return LRSDP_ERR_INVALID_ARG;
  spmm_U(P, k, P->ginv, v, f->U, w.y, s);                // M U, M = mat(A G^{-1} v)
  if (f->precond == LRSDP_PRECOND_AUG) {
    // H^{-1} v (eq aug_prec, x eliminated): w = B^T G^{-1} v = vec(M U), t = Sh^{-1} w with
    // Sh = tau/2 I + B^T G^{-1} B, z = (v - B t) G^{-1} / tau^2, B t = [A_i . (T U^T)]_i
    LRSDP_TRY(binv_apply(f->Sinv, nk, f->sinv_split, nk, w.y, nullptr, w.h, w.t, false, s));
    k_smw_out<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, P->ginv,
                                               1.0 / f->tau2, w.t, f->U, v, z);
    LRSDP_HIP(hipGetLastError());
    return LRSDP_OK;
  }
  rows_k(n, k, f->Zt, 2, w.y, w.w, s);                    // w = vec(Z^T M U)
  LRSDP_TRY(binv_apply(f->Sinv, nk, f->sinv_split, nk, w.w, nullptr, w.h, w.t, false, s));
  if (refine) {                                           // t += bold S^{-1} (w - bold S t)
    LRSDP_TRY(schur_apply_f64(f, w.t, w.s, s));
    LRSDP_TRY(binv_apply(f->Sinv, nk, f->sinv_split, nk, w.w, w.s, w.h, w.t, true, s));
  }
  rows_k(n, k, f->Z, 1, w.t, w.y, s);                      // Y = Z T
  k_smw_out<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, P->ginv,
                                             1.0 / f->tau2, w.y, f->U, v, z);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int precond_apply_dd(const lrsdp_factor* f, const double* v, double* z, hipStream_t s,
                     int nref) {
  const lrsdp_problem* P = f->P;
  const Work w = work_view(f);
  const int n = f->n, k = f->k, m = P->m, nk = f->nk;
  if (k > KMAX) return LRSDP_ERR_INVALID_ARG;
  // w = bold U^T G^{-1} v in double-double
  spmm_U_dd(P, k, P->ginv, v, nullptr, f->U, w.y, w.yl, s);
  rows_k_dd(n, k, f->Zt, 2, w.y, w.yl, w.w, w.wl, s);
  // t = bold S^{-1} w: FP64 inverse, refined against the matrix-free bold S in double-double
  k_dd_combine<<<grid_for(nk, 256), 256, 0, s>>>(nk, w.w, w.wl, w.g0, w.tl);  // tl = 0
  LRSDP_TRY(binv_apply(f->Sinv, nk, f->sinv_split, nk, w.g0, nullptr, w.h, w.t, false, s));
  for (int it = 0; it < nref; ++it) {
    LRSDP_TRY(schur_apply_dd(f, w.t, w.tl, w.s, w.sl, s));
    k_dd_sub_round<<<grid_for(nk, 256), 256, 0, s>>>(nk, w.w, w.wl, w.s, w.sl, w.g0);
    LRSDP_TRY(binv_apply(f->Sinv, nk, f->sinv_split, nk, w.g0, nullptr, w.h, w.g1, false, s));
    k_dd_accum<<<grid_for(nk, 256), 256, 0, s>>>(nk, w.t, w.tl, w.g1);
  }
  // x = bold U t (dd);  z = (v - x) G^{-1} / tau^2
  rows_k_dd(n, k, f->Z, 1, w.t, w.tl, w.y, w.yl, s);
  k_sampled_dd<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, w.y, w.yl, f->U,
                                                 nullptr, nullptr, v, P->ginv, 1.0 / f->tau2, z);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int split_apply(lrsdp_factor* f, const double* v, double* Hv, int precision, hipStream_t s) {
  lrsdp_problem* P = f->P;
  const Work w = work_view(f);
  const int n = f->n, k = f->k, m = P->m;
  if (k > KMAX) return LRSDP_ERR_INVALID_ARG;
  LRSDP_TRY(ensure_lowprec(f, precision, s));
  // A^T vec(W0 M W0) in the requested precision
  if (precision == LRSDP_PREC_FP32) LRSDP_TRY(hv_apply_f32(P, f->W0f, v, Hv, s));
  else if (precision == LRSDP_PREC_BF16) LRSDP_TRY(hv_apply_bf16(P, f->W0b, v, Hv, s));
  else LRSDP_TRY(hv_apply_f64(P, f->W0, v, Hv, s));
  // P = M U (dd), Q = W0 P, K = U^T P (dd), then the sampled rank-k terms
  spmm_U_dd(P, k, nullptr, v, nullptr, f->U, w.g0, w.g1, s);
  rows_k(n, k, f->W0, 0, w.g0, w.s, s);
  k_UtP<<<k * k, kT, 0, s>>>(n, k, f->U, w.g0, w.g1, w.kk);
  k_lowrank_add<<<grid_for(m, 256), 256, 0, s>>>(m, n, k, P->a, P->b, P->coef, f->U, w.s, w.kk,
                                                  Hv);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

// ---------------------------------------------------------------- lock-step batches
// The same bodies on a packed grid (bl_find): each instance runs the grid it runs alone.
namespace {

// The dense n x n operand of a rows-times-k product: 0 W0, 1 Z, 2 Z^T
__device__ __forceinline__ const double* pick_a(const BInst& d, int which) {
  return which == 0 ? d.W0 : which == 1 ? d.Z : d.Zt;
}
#define LRSDP_BL_HEAD(KIND)                       \
  int bx;                                         \
  const int z = bl_find(b, KIND, blockIdx.x, &bx); \
  if (!b.act[z]) return;                          \
  const BInst& d = b.I[z];

template <int K2>
__global__ __launch_bounds__(kT) void k_spmm_U_b(const BL b, int use_ginv, int vrole,
                                                 int orole) {
  LRSDP_BL_HEAD(kKrowsU)
  spmm_U_body<K2>(bx, d.n, d.k, d.rowptr, d.colidx, d.src, d.val, use_ginv ? d.ginv : nullptr,
                  d.v[vrole], d.U, d.v[orole]);
}
template <int K2>
__global__ __launch_bounds__(kT) void k_spmm_U_dd_b(const BL b, int vrole, int hrole,
                                                    int lrole) {
  LRSDP_BL_HEAD(kKrowsU)
  spmm_U_dd_body<K2>(bx, d.n, d.k, d.rowptr, d.colidx, d.src, d.val, nullptr, d.v[vrole],
                     nullptr, d.U, d.v[hrole], d.v[lrole]);
}
// out = rows of A times X (+ c tadd: c = tau^2 when add_tau2, tadd = v[trole])
__global__ __launch_bounds__(kT) void k_rows_kr_b(const BL b, int which, int range, int xrole,
                                                  int orole, int add_tau2, int trole) {
  LRSDP_BL_HEAD(kKrows)
  rows_kr_body<4, 4>(bx, d.n, d.k, pick_a(d, which), range, d.v[xrole], d.v[orole],
                     add_tau2 ? d.tau2 : 0.0, add_tau2 ? d.v[trole] : nullptr);
}
__global__ __launch_bounds__(kT) void k_UtP_b(const BL b) {
  LRSDP_BL_HEAD(kKkk)
  UtP_body(bx, d.n, d.k, d.U, d.v[kVwg0], d.v[kVwg1], d.kk);
}
__global__ __launch_bounds__(256) void k_lowrank_add_b(const BL b, int orole) {
  LRSDP_BL_HEAD(kKm256)
  lowrank_add_body(bx, d.m, d.n, d.k, d.a, d.b, d.coef, d.U, d.v[kVws], d.kk, d.v[orole]);
}
__global__ __launch_bounds__(256) void k_sampled_f64_b(const BL b) {
  LRSDP_BL_HEAD(kKm256)
  sampled_f64_body(bx, d.m, d.n, d.k, d.a, d.b, d.coef, d.ginv, d.v[kVwy], d.U, d.v[kVwt0]);
}
__global__ __launch_bounds__(kT) void k_Qt_b(const BL b) {
  LRSDP_BL_HEAD(kKr)
  Qt_body(bx, d.nk, d.r, d.QN, d.v[kVwt], d.kk);
}
__global__ __launch_bounds__(256) void k_Qc_b(const BL b) {
  LRSDP_BL_HEAD(kKnk256)
  if (d.r == 0) return;
  Qc_body(bx, d.nk, d.r, d.shift, d.QN, d.kk, d.v[kVws]);
}
__global__ __launch_bounds__(256) void k_smw_out_b(const BL b, int vrole, int zrole) {
  LRSDP_BL_HEAD(kKm256)
  smw_out_body(bx, d.m, d.n, d.k, d.a, d.b, d.coef, d.ginv, d.inv_tau2, d.v[kVwy], d.U,
               d.v[vrole], d.v[zrole]);
}
#undef LRSDP_BL_HEAD

// k <= 2 and k <= 4 use K2 = 2 and 4, as spmm_U does; the batch holds one K2 class
int k2_of(int k) { return k <= 2 ? 2 : 4; }

int bl_rows(const BLaunch& L, int which, int range, int xrole, int orole, bool add_tau2,
            int trole, hipStream_t s) {
  k_rows_kr_b<<<L.tot[kKrows], kT, 0, s>>>(L.b, which, range, xrole, orole, add_tau2 ? 1 : 0,
                                           trole);
  return LRSDP_OK;
}
int bl_spmm_U(const BLaunch& L, bool use_ginv, int vrole, int orole, hipStream_t s) {
  const int grid = L.tot[kKrowsU];
  if (k2_of(L.kmax) == 2) k_spmm_U_b<2><<<grid, kT, 0, s>>>(L.b, use_ginv ? 1 : 0, vrole, orole);
  else k_spmm_U_b<4><<<grid, kT, 0, s>>>(L.b, use_ginv ? 1 : 0, vrole, orole);
  return LRSDP_OK;
}

}  // namespace

// L.kmax: the largest k of the batch; the batch holds instances of one K2 class (k <= 2 or
// 3 <= k <= 4), and rows_k's kernel (R = 4, KC = 4) covers k <= 4.
int bl_split_apply(const BLaunch& L, int precision, int cb, int vrole, int orole,
                   hipStream_t s) {
  if (L.b.count <= 0) return LRSDP_OK;
  if (L.kmax > 4) return LRSDP_ERR_INVALID_ARG;
  LRSDP_TRY(bl_hv(L, precision, cb, false, vrole, orole, s));
  const int grid = L.tot[kKrowsU];
  if (k2_of(L.kmax) == 2) k_spmm_U_dd_b<2><<<grid, kT, 0, s>>>(L.b, vrole, kVwg0, kVwg1);
  else k_spmm_U_dd_b<4><<<grid, kT, 0, s>>>(L.b, vrole, kVwg0, kVwg1);
  LRSDP_TRY(bl_rows(L, 0, 0, kVwg0, kVws, false, 0, s));
  k_UtP_b<<<L.tot[kKkk], kT, 0, s>>>(L.b);
  k_lowrank_add_b<<<L.tot[kKm256], 256, 0, s>>>(L.b, orole);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int bl_precond_f64(const BLaunch& L, int refine, int vrole, int zrole, hipStream_t s) {
  if (L.b.count <= 0) return LRSDP_OK;
  if (L.kmax > 4) return LRSDP_ERR_INVALID_ARG;
  LRSDP_TRY(bl_spmm_U(L, true, vrole, kVwy, s));                     // M U
  LRSDP_TRY(bl_rows(L, 2, 2, kVwy, kVww, false, 0, s));              // w = vec(Z^T M U)
  LRSDP_TRY(bl_gemv_pair(L, kVww, -1, kVwh, kVwt, false, s));        // t = S^{-1} w
  if (refine) {  // t += S^{-1} (w - bold S t), bold S t as in schur_apply_f64
    LRSDP_TRY(bl_rows(L, 1, 1, kVwt, kVwy, false, 0, s));
    k_sampled_f64_b<<<L.tot[kKm256], 256, 0, s>>>(L.b);
    LRSDP_TRY(bl_spmm_U(L, false, kVwt0, kVwy, s));
    LRSDP_TRY(bl_rows(L, 2, 2, kVwy, kVws, true, kVwt, s));
    if (L.rmax > 0) {
      k_Qt_b<<<L.tot[kKr], kT, 0, s>>>(L.b);
      k_Qc_b<<<L.tot[kKnk256], 256, 0, s>>>(L.b);
    }
    LRSDP_TRY(bl_gemv_pair(L, kVww, kVws, kVwh, kVwt, true, s));
  }
  LRSDP_TRY(bl_rows(L, 1, 1, kVwt, kVwy, false, 0, s));              // Y = Z T
  k_smw_out_b<<<L.tot[kKm256], 256, 0, s>>>(L.b, vrole, zrole);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

}  // namespace lrsdp
