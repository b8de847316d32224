// Steps A5 / A7 / A8-residual: the matrix-free Hessian product of eq hesseqn2,
//   (H v)_i = A_i . (W M W),  M = mat(A v) = sum_i v_i A_i,
// as three stages that never form a dense n x n intermediate in HBM:
//   1. scatter   mval[e] = val_{src(e)} v_{src(e)} on the symmetric CSR pattern of M;
//   2. SpMM      Tt = W M (= (M W)^T, M and W symmetric) for a block of CB rows of W that
//                sits in LDS; M's pattern is streamed (it is small and L2-resident);
//   3. gather    (W M W)_{ab} = W[a, :] . Tt[b, :] for the constraints owned by the block's
//                rows, one wavefront per constraint with a wave reduction; the LDS copy of Tt
//                is read, W's row a streams from L2 / HBM with coalesced 64-wide loads.
// Work per product: 2 (nnz + m) n flops; HBM traffic: W once (the LDS blocks) plus the
// gather's row reads, which hit L2 / MALL for n up to a few thousand.
#include <mutex>

#include "internal.h"

namespace lrsdp {
namespace {

constexpr int kThreads = 1024;
constexpr size_t kLdsBudget = 80 * 1024;  // two workgroups of 16 wavefronts per CU
constexpr size_t kLdsMax = 160 * 1024;    // one workgroup per CU

__device__ __forceinline__ void scatter_body(int bx, int nnz, const int32_t* __restrict__ src,
                                             const double* __restrict__ val,
                                             const double* __restrict__ v,
                                             double* __restrict__ mval) {
  int e = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (e < nnz) {
    int i = src[e];
    mval[e] = val[i] * v[i];
  }
}
__global__ __launch_bounds__(256) void k_scatter(int nnz, const int32_t* __restrict__ src,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ mval) {
  scatter_body(blockIdx.x, nnz, src, val, v, mval);
}

template <typename TW, typename TA>
__device__ __forceinline__ TA load_w(const TW* W, size_t idx);
template <>
__device__ __forceinline__ double load_w<double, double>(const double* W, size_t idx) {
  return W[idx];
}
template <>
__device__ __forceinline__ float load_w<float, float>(const float* W, size_t idx) {
  return W[idx];
}
template <>
__device__ __forceinline__ float load_w<uint16_t, float>(const uint16_t* W, size_t idx) {
  return bf16_to_f32(W[idx]);
}

template <typename TA>
__device__ __forceinline__ TA to_ta(double x);
template <>
__device__ __forceinline__ double to_ta<double>(double x) { return x; }
template <>
__device__ __forceinline__ float to_ta<float>(double x) { return static_cast<float>(x); }

// Which of the block's CB rows owns list position t (own_ptr is the prefix over rows).
__device__ __forceinline__ int owner_row(const int32_t* own_ptr, int c0, int cb, int t) {
  int c = 0;
  while (c + 1 < cb && own_ptr[c0 + c + 1] <= t) ++c;
  return c;
}

// kTG: the workgroup's rows of Tt live in global scratch tg (n x ldn, L2-resident), not in
// LDS, which then holds only the CB rows of W (large n).
template <typename TW, typename TA, int CB, bool kBf16Values, bool kTG>
__device__ __forceinline__ void hv_body(
    int bx, int n, int ldn, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ colidx, const double* __restrict__ mval,
    const TW* __restrict__ W, const int32_t* __restrict__ own_ptr,
    const int32_t* __restrict__ own_con, const int32_t* __restrict__ own_oth,
    const double* __restrict__ coef, double* __restrict__ Hv, TA* __restrict__ tg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TA* Wb = reinterpret_cast<TA*>(smem_raw);  // [CB][ldn]
  const int c0 = bx * CB;
  TA* Tt = kTG ? tg + (size_t)c0 * ldn : Wb + CB * ldn;  // [CB][ldn]
  const int cb = min(CB, n - c0);

  // 1. stage rows c0..c0+cb-1 of W
  for (int idx = threadIdx.x; idx < CB * n; idx += kThreads) {
    int c = idx / n, q = idx - c * n;
    Wb[c * ldn + q] = (c < cb) ? load_w<TW, TA>(W, (size_t)(c0 + c) * n + q) : TA(0);
  }
  __syncthreads();

  // 2. Tt[c][p] = sum_q M_pq W[c0 + c, q] over the sorted pattern of row p.  Eight lanes
  //    share a row (coalesced loads of the pattern, several in flight per lane), then a
  //    three-step shuffle reduction; a fixed lane-to-entry map keeps the sum order fixed.
  {
    const int sub = threadIdx.x & 7;
    for (int p = threadIdx.x >> 3; p < n; p += kThreads / 8) {
      TA acc[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[c] = TA(0);
      const int lo = rowptr[p], hi = rowptr[p + 1];
#pragma unroll 2
      for (int e = lo + sub; e < hi; e += 8) {
        const int q = colidx[e];
        TA mv = to_ta<TA>(mval[e]);
        if constexpr (kBf16Values) mv = bf16_to_f32(f32_to_bf16_rne(mv));
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = fma(mv, Wb[c * ldn + q], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        TA v = acc[c];
        v += __shfl_xor(v, 1, 8);
        v += __shfl_xor(v, 2, 8);
        v += __shfl_xor(v, 4, 8);
        acc[c] = v;
      }
      if (sub == 0) {
#pragma unroll
        for (int c = 0; c < CB; ++c)
          if (!kTG || c < cb) Tt[c * ldn + p] = acc[c];  // (global rows stop at n)
      }
    }
  }
  __syncthreads();

  // 3. one wavefront per owned constraint: X_ab = W[a, :] . Tt[b - c0, :]
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nwv = kThreads / kWave;
  const int t0 = own_ptr[c0], t1 = own_ptr[c0 + cb];
  for (int t = t0 + wid; t < t1; t += nwv) {
    const int c = owner_row(own_ptr, c0, cb, t);
    const int a = own_oth[t];
    const TW* wa = W + (size_t)a * n;
    const TA* tt = Tt + c * ldn;
    TA s = TA(0);
#pragma unroll 8
    for (int p = lane; p < n; p += kWave) s = fma(load_w<TW, TA>(wa, p), tt[p], s);
    s = wave_sum(s);
    if (lane == 0) {
      const int i = own_con[t];
      Hv[i] = coef[i] * static_cast<double>(s);
    }
  }
}
template <typename TW, typename TA, int CB, bool kBf16Values, bool kTG>
__global__ __launch_bounds__(kThreads) void k_hv_fused(
    int n, int ldn, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ mval, const TW* __restrict__ W,
    const int32_t* __restrict__ own_ptr, const int32_t* __restrict__ own_con,
    const int32_t* __restrict__ own_oth, const double* __restrict__ coef,
    double* __restrict__ Hv, TA* __restrict__ tg) {
  hv_body<TW, TA, CB, kBf16Values, kTG>(blockIdx.x, n, ldn, rowptr, colidx, mval, W, own_ptr,
                                        own_con, own_oth, coef, Hv, tg);
}

// Rows of W per workgroup: as many as the LDS holds (up to 8; rows_lds = LDS bytes per row),
// while at least ~200 workgroups remain so that every CU gets one; fewer rows per
// workgroup cost only extra (L2-resident) passes over the pattern.
int rows_per_wg(int n, size_t budget, size_t row_bytes) {
  int cb = static_cast<int>(budget / row_bytes);
  if (cb < 1) return 0;
  cb = cb >= 8 ? 8 : cb >= 4 ? 4 : cb >= 2 ? 2 : 1;
  while (cb > 1 && (n + cb - 1) / cb < 200) cb >>= 1;
  return cb;
}

// Rows of W per H v workgroup for TA values of ta_bytes, and whether the rows of T go to the
// global scratch (*tg); 0 when none fit.
int hv_shape(int n, size_t ta_bytes, bool have_tscr, bool* tg) {
  int cb = rows_per_wg(n, kLdsBudget, 2 * (size_t)n * ta_bytes);
  if (cb < 1) cb = rows_per_wg(n, kLdsMax, 2 * (size_t)n * ta_bytes);
  *tg = have_tscr && cb < 4;
  if (*tg) cb = rows_per_wg(n, kLdsMax, (size_t)n * ta_bytes);
  return cb;
}
// the same for the double-double residual (three double rows per row of W)
int res_shape(int n, bool have_tscr, bool* tg) {
  const size_t row_bytes = 3 * (size_t)n * sizeof(double);
  int cb = rows_per_wg(n, kLdsBudget, row_bytes);
  if (cb < 1) cb = rows_per_wg(n, kLdsMax, row_bytes);
  *tg = have_tscr && cb < 4;
  if (*tg) cb = rows_per_wg(n, kLdsMax, (size_t)n * sizeof(double));
  return cb >= 4 ? 4 : cb;
}

// mval: nnz doubles of scratch for the values of mat(A v) (the problem's own, or the fixed
// array of the allocation-free entry point).
template <typename TW, typename TA, bool kBf16Values>
int launch_hv(const lrsdp_problem* P, const TW* W, const double* v, double* Hv, double* mval,
              hipStream_t s) {
  const int n = P->n;
  k_scatter<<<grid_for(P->nnz, 256), 256, 0, s>>>(P->nnz, P->src, P->val, v, mval);
  const int ldn = n;
  // W and T rows in LDS (two workgroups per CU, else one); with the global scratch, only W
  bool tg = false;
  const int cb = hv_shape(n, sizeof(TA), P->tscr != nullptr, &tg);
  if (cb < 1) return LRSDP_ERR_INVALID_ARG;
  const size_t smem = (size_t)cb * (tg ? 1 : 2) * ldn * sizeof(TA);
  TA* tgp = reinterpret_cast<TA*>(P->tscr);
  const int grid = (n + cb - 1) / cb;
  ProfMark pm = prof_begin(LRSDP_K_HV, s);
#define LRSDP_HV_CASE(CBV)                                                                     \
  case CBV:                                                                                    \
    if (tg)                                                                                    \
      hipLaunchKernelGGL((k_hv_fused<TW, TA, CBV, kBf16Values, true>), dim3(grid),             \
                         dim3(kThreads), smem, s, n, ldn, P->rowptr, P->colidx, mval, W,       \
                         P->own_ptr, P->own_con, P->own_oth, P->coef, Hv, tgp);                \
    else                                                                                       \
      hipLaunchKernelGGL((k_hv_fused<TW, TA, CBV, kBf16Values, false>), dim3(grid),            \
                         dim3(kThreads), smem, s, n, ldn, P->rowptr, P->colidx, mval, W,       \
                         P->own_ptr, P->own_con, P->own_oth, P->coef, Hv, nullptr);            \
    break;
  switch (cb) {
    LRSDP_HV_CASE(1)
    LRSDP_HV_CASE(2)
    LRSDP_HV_CASE(4)
    LRSDP_HV_CASE(8)
  }
#undef LRSDP_HV_CASE
  LRSDP_HIP(hipGetLastError());
  // algorithmic bytes of H v as a two-pass product: W read by both passes, T = M W written
  // once and read once (2 (s_W + s_T) n^2), 24 bytes per constraint and 20 per pattern entry;
  // the fused kernel keeps T on chip, so it moves less than this.  Flops 2 (nnz + m) n.
  prof_end(pm, s,
           2.0 * ((double)sizeof(TW) + sizeof(TA)) * n * n + 24.0 * P->m + 20.0 * P->nnz,
           2.0 * ((double)P->nnz + P->m) * n);
  return LRSDP_OK;
}

// ---------------------------------------------------------------- double-double residual
// res = r - H (y + ylo) with every product error-free: the rows of T = W mat(A (y + ylo)) and the
// gathers A_i . (T W) are compensated dot products (Dot2), whose partial results are combined
// in double-double.

__device__ __forceinline__ void scatter_dd_body(int bx, int nnz, const int32_t* __restrict__ src,
                                                const double* __restrict__ val,
                                                const double* __restrict__ y,
                                                const double* __restrict__ ylo,
                                                double* __restrict__ mhi,
                                                double* __restrict__ mlo) {
  int e = bx * 256 + threadIdx.x;  // 256 threads per workgroup
  if (e < nnz) {
    int i = src[e];
    dd p = two_prod(val[i], y[i]);
    if (ylo) p.lo = fma(val[i], ylo[i], p.lo);
    p = quick_two_sum(p.hi, p.lo);
    mhi[e] = p.hi;
    mlo[e] = p.lo;
  }
}
__global__ __launch_bounds__(256) void k_scatter_dd(int nnz, const int32_t* __restrict__ src,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ ylo,
                                                    double* __restrict__ mhi,
                                                    double* __restrict__ mlo) {
  scatter_dd_body(blockIdx.x, nnz, src, val, y, ylo, mhi, mlo);
}

// kTG: the rows of (Th, Tl) live in global scratch (tgh, tgl: n x ldn each), as in k_hv_fused.
template <int CB, bool kTG>
__device__ __forceinline__ void residual_dd_body(
    int bx, int n, int ldn, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ colidx, const double* __restrict__ mhi,
    const double* __restrict__ mlo, const double* __restrict__ W,
    const int32_t* __restrict__ own_ptr, const int32_t* __restrict__ own_con,
    const int32_t* __restrict__ own_oth, const double* __restrict__ coef,
    const double* __restrict__ r, double* __restrict__ res, double* __restrict__ res_lo,
    double* __restrict__ tgh, double* __restrict__ tgl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Wb = reinterpret_cast<double*>(smem_raw);  // [CB][ldn]
  const int c0 = bx * CB;
  double* Th = kTG ? tgh + (size_t)c0 * ldn : Wb + CB * ldn;
  double* Tl = kTG ? tgl + (size_t)c0 * ldn : Th + CB * ldn;
  const int cb = min(CB, n - c0);
  for (int idx = threadIdx.x; idx < CB * n; idx += kThreads) {
    int c = idx / n, q = idx - c * n;
    Wb[c * ldn + q] = (c < cb) ? W[(size_t)(c0 + c) * n + q] : 0.0;
  }
  __syncthreads();
  {
    const int sub = threadIdx.x & 7;
    for (int p = threadIdx.x >> 3; p < n; p += kThreads / 8) {
      dot2 part[CB];
      dd acc[CB];
      const int lo = rowptr[p], hi = rowptr[p + 1];
      for (int e = lo + sub; e < hi; e += 8) {
        const int q = colidx[e];
        const double h = mhi[e], l = mlo[e];
#pragma unroll
        for (int c = 0; c < CB; ++c) dot2_add(part[c], Wb[c * ldn + q], h, l);
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        dd v = dot2_result(part[c]);
        v = dd_add(v, {__shfl_xor(v.hi, 1, 8), __shfl_xor(v.lo, 1, 8)});
        v = dd_add(v, {__shfl_xor(v.hi, 2, 8), __shfl_xor(v.lo, 2, 8)});
        v = dd_add(v, {__shfl_xor(v.hi, 4, 8), __shfl_xor(v.lo, 4, 8)});
        acc[c] = v;
      }
      if (sub == 0) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          if (kTG && c >= cb) continue;  // (global rows stop at n)
          Th[c * ldn + p] = acc[c].hi;
          Tl[c * ldn + p] = acc[c].lo;
        }
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nwv = kThreads / kWave;
  const int t0 = own_ptr[c0], t1 = own_ptr[c0 + cb];
  for (int t = t0 + wid; t < t1; t += nwv) {
    const int c = owner_row(own_ptr, c0, cb, t);
    const int a = own_oth[t];
    const double* wa = W + (size_t)a * n;
    dot2 part;
    for (int p = lane; p < n; p += kWave) dot2_add(part, wa[p], Th[c * ldn + p], Tl[c * ldn + p]);
    const dd s = wave_sum_dd(dot2_result(part));
    if (lane == 0) {
      const int i = own_con[t];
      dd hv = dd_mul_d(s, coef[i]);
      dd d = dd_add_d({-hv.hi, -hv.lo}, r[i]);
      res[i] = d.hi;
      if (res_lo) res_lo[i] = d.lo;
    }
  }
}
template <int CB, bool kTG>
__global__ __launch_bounds__(kThreads) void k_residual_dd(
    int n, int ldn, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ mhi, const double* __restrict__ mlo,
    const double* __restrict__ W, const int32_t* __restrict__ own_ptr,
    const int32_t* __restrict__ own_con, const int32_t* __restrict__ own_oth,
    const double* __restrict__ coef, const double* __restrict__ r, double* __restrict__ res,
    double* __restrict__ res_lo, double* __restrict__ tgh, double* __restrict__ tgl) {
  residual_dd_body<CB, kTG>(blockIdx.x, n, ldn, rowptr, colidx, mhi, mlo, W, own_ptr, own_con,
                            own_oth, coef, r, res, res_lo, tgh, tgl);
}

// ---------------------------------------------------------------- lock-step batches
// The same bodies on a packed grid (bl_find): each instance runs its own grid, so it computes
// exactly what it computes alone.
template <typename TW>
__device__ __forceinline__ const TW* pick_w(const BInst& d, bool whole);
template <>
__device__ __forceinline__ const double* pick_w<double>(const BInst& d, bool whole) {
  return whole ? d.W : d.W0;
}
template <>
__device__ __forceinline__ const float* pick_w<float>(const BInst& d, bool) { return d.W0f; }
template <>
__device__ __forceinline__ const uint16_t* pick_w<uint16_t>(const BInst& d, bool) {
  return d.W0b;
}

__global__ __launch_bounds__(256) void k_scatter_b(const BL b, int vrole) {
  int bx;
  const int z = bl_find(b, kKnnz256, blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  scatter_body(bx, d.nnz, d.src, d.val, d.v[vrole], d.mval);
}
template <typename TW, typename TA, int CB, bool kBf16Values>
__global__ __launch_bounds__(kThreads) void k_hv_fused_b(const BL b, int whole, int orole) {
  int bx;
  const int z = bl_find(b, hv_kind(CB), blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  hv_body<TW, TA, CB, kBf16Values, false>(bx, d.n, d.n, d.rowptr, d.colidx, d.mval,
                                          pick_w<TW>(d, whole != 0), d.own_ptr, d.own_con,
                                          d.own_oth, d.coef, d.v[orole], nullptr);
}
__global__ __launch_bounds__(256) void k_scatter_dd_b(const BL b) {
  int bx;
  const int z = bl_find(b, kKnnz256, blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  scatter_dd_body(bx, d.nnz, d.src, d.val, d.v[kVy], d.v[kVyl], d.mval, d.mlo);
}
template <int CB>
__global__ __launch_bounds__(kThreads) void k_residual_dd_b(const BL b) {
  int bx;
  const int z = bl_find(b, res_kind(CB), blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  residual_dd_body<CB, false>(bx, d.n, d.n, d.rowptr, d.colidx, d.mval, d.mlo, d.W, d.own_ptr,
                              d.own_con, d.own_oth, d.coef, d.v[kVrhs], d.v[kVdd0], d.v[kVdd1],
                              nullptr, nullptr);
}

template <typename TW, typename TA, bool kBf16Values>
int launch_hv_b(const BLaunch& L, int cb, bool whole, int orole, hipStream_t s) {
  const size_t smem = (size_t)cb * 2 * L.nmax * sizeof(TA);
  const int grid = L.tot[hv_kind(cb)];
  const int w = whole ? 1 : 0;
  switch (cb) {
    case 1: k_hv_fused_b<TW, TA, 1, kBf16Values><<<grid, kThreads, smem, s>>>(L.b, w, orole); break;
    case 2: k_hv_fused_b<TW, TA, 2, kBf16Values><<<grid, kThreads, smem, s>>>(L.b, w, orole); break;
    case 4: k_hv_fused_b<TW, TA, 4, kBf16Values><<<grid, kThreads, smem, s>>>(L.b, w, orole); break;
    case 8: k_hv_fused_b<TW, TA, 8, kBf16Values><<<grid, kThreads, smem, s>>>(L.b, w, orole); break;
    default: return LRSDP_ERR_INVALID_ARG;
  }
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

}  // namespace

int bl_hv(const BLaunch& L, int precision, int cb, bool whole_w, int vrole, int orole,
          hipStream_t s) {
  if (L.b.count <= 0) return LRSDP_OK;
  k_scatter_b<<<L.tot[kKnnz256], 256, 0, s>>>(L.b, vrole);
  if (precision == LRSDP_PREC_FP32) return launch_hv_b<float, float, false>(L, cb, false, orole, s);
  if (precision == LRSDP_PREC_BF16) return launch_hv_b<uint16_t, float, true>(L, cb, false, orole, s);
  return launch_hv_b<double, double, false>(L, cb, whole_w, orole, s);
}

int bl_residual_dd(const BLaunch& L, int cb, hipStream_t s) {
  if (L.b.count <= 0) return LRSDP_OK;
  k_scatter_dd_b<<<L.tot[kKnnz256], 256, 0, s>>>(L.b);
  const size_t smem = (size_t)cb * 3 * L.nmax * sizeof(double);
  const int grid = L.tot[res_kind(cb)];
  switch (cb) {
    case 1: k_residual_dd_b<1><<<grid, kThreads, smem, s>>>(L.b); break;
    case 2: k_residual_dd_b<2><<<grid, kThreads, smem, s>>>(L.b); break;
    case 4: k_residual_dd_b<4><<<grid, kThreads, smem, s>>>(L.b); break;
    default: return LRSDP_ERR_INVALID_ARG;
  }
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int hv_apply_f64(const lrsdp_problem* P, const double* W, const double* v, double* Hv,
                 hipStream_t s) {
  return launch_hv<double, double, false>(P, W, v, Hv, P->mval, s);
}
int hv_apply_f32(const lrsdp_problem* P, const float* W, const double* v, double* Hv,
                 hipStream_t s) {
  return launch_hv<float, float, false>(P, W, v, Hv, P->mval, s);
}
int hv_apply_bf16(const lrsdp_problem* P, const uint16_t* W, const double* v, double* Hv,
                  hipStream_t s) {
  return launch_hv<uint16_t, float, true>(P, W, v, Hv, P->mval, s);
}

// ---------------------------------------------------------------- allocation-free H v
// The fixed scratch of lrsdp_hessian_apply_noalloc: the values of mat(A v), nnz doubles.  Every
// GPU the library runs on holds one copy until the process ends; its address on each device
// comes from hipGetSymbolAddress at context creation (the array's name is not a device
// address in host code).
namespace {
constexpr size_t kScratchDoubles = (size_t)2 << 20;  // 16 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return LRSDP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return LRSDP_OK;
  void* ptr = nullptr;  // the caller has made `device` current
  LRSDP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return LRSDP_OK;
}

size_t noalloc_scratch_doubles() { return kScratchDoubles; }

int hv_apply_f64_noalloc(const lrsdp_problem* P, const double* W, const double* v, double* Hv,
                         int device, hipStream_t s) {
  if ((size_t)P->nnz > kScratchDoubles || P->tscr != nullptr) return LRSDP_ERR_SCRATCH;
  double* buf = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    buf = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  }
  if (!buf) return LRSDP_ERR_DEVICE;
  return launch_hv<double, double, false>(P, W, v, Hv, buf, s);
}

int hv_residual_dd(const lrsdp_problem* P, const double* W, const double* r, const double* y,
                   const double* ylo, double* res, double* res_lo, hipStream_t s) {
  const int n = P->n;
  // mat(A y) in double-double: two nnz arrays carved from the problem's scratch space
  double* mhi = P->mval;
  double* mlo = P->vec_scratch;  // sized max(4 m, nnz) at problem creation
  k_scatter_dd<<<grid_for(P->nnz, 256), 256, 0, s>>>(P->nnz, P->src, P->val, y, ylo, mhi, mlo);
  const int ldn = n;
  bool tg = false;
  const int cb = res_shape(n, P->tscr != nullptr, &tg);
  if (cb < 1) return LRSDP_ERR_INVALID_ARG;
  const size_t smem = (size_t)cb * (tg ? 1 : 3) * ldn * sizeof(double);
  double* tgh = P->tscr;
  double* tgl = tg ? P->tscr + (size_t)n * n : nullptr;
  const int grid = (n + cb - 1) / cb;
  ProfMark pm = prof_begin(LRSDP_K_RESDD, s);
#define LRSDP_RES_CASE(CBV)                                                                 \
  case CBV:                                                                                 \
    if (tg)                                                                                 \
      hipLaunchKernelGGL((k_residual_dd<CBV, true>), dim3(grid), dim3(kThreads), smem, s,   \
                         n, ldn, P->rowptr, P->colidx, mhi, mlo, W, P->own_ptr,             \
                         P->own_con, P->own_oth, P->coef, r, res, res_lo, tgh, tgl);        \
    else                                                                                    \
      hipLaunchKernelGGL((k_residual_dd<CBV, false>), dim3(grid), dim3(kThreads), smem, s,  \
                         n, ldn, P->rowptr, P->colidx, mhi, mlo, W, P->own_ptr,             \
                         P->own_con, P->own_oth, P->coef, r, res, res_lo, nullptr, nullptr); \
    break;
  switch (cb) {
    LRSDP_RES_CASE(1)
    LRSDP_RES_CASE(2)
    LRSDP_RES_CASE(4)
  }
#undef LRSDP_RES_CASE
  LRSDP_HIP(hipGetLastError());
  prof_end(pm, s, 8.0 * n * n + 20.0 * P->nnz + 40.0 * P->m, 2.0 * ((double)P->nnz + P->m) * n);
  return LRSDP_OK;
}

}  // namespace lrsdp
