// Dense FP64 linear algebra on CDNA4 matrix cores for the setup of Algorithm 1.
//
// GEMM: 64 x 64 output tile per workgroup, four wavefronts each owning a 32 x 32 quarter
// as 2 x 2 v_mfma_f64_16x16x4_f64 accumulators; K advances 16 at a time through LDS.
// Operand fragments follow the MFMA register layout: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the 16 x 16 result lives as D[l / 16 + 4 r][l % 16], r = 0..3
// (rows interleaved across the four result registers).
// Triangular operands skip whole zero tiles through per-tile K ranges (GemmFlags).
//
// POTRF / TRSM / TRTRI / LAUUM are recursive (split at a multiple of 64) so that nearly all
// their flops land in that GEMM; the 64 x 64 leaves are single-workgroup LDS kernels.
#include <algorithm>

#include "dense.h"

namespace lrsdp {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int PITCH = TM + 4;  // LDS row pitch (doubles) of the K-major operand tiles
constexpr int NB = 64;         // leaf size of the recursive factorizations

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ double As[2][TK][PITCH];
  __shared__ double Bs[2][TK][PITCH];
  const double* __restrict__ Ap = g.A;
  const double* __restrict__ Bp = g.B;
  double* __restrict__ Cp = g.C;
  if (g.offs) {  // batched: per-z element offsets of A, B, C
    const int z = blockIdx.y;
    Ap += g.offs[3 * z];
    Bp += g.offs[3 * z + 1];
    Cp += g.offs[3 * z + 2];
  }
  const int tiles_n = (g.N + TN - 1) / TN;
  const int ti = blockIdx.x / tiles_n;
  const int tj = blockIdx.x - ti * tiles_n;
  const int i0 = ti * TM, j0 = tj * TN;
  const bool lower = (g.flags & kLowerOut) != 0;
  if (lower && j0 > i0 + TM - 1) return;
  int klo = 0, khi = g.K;
  if (g.flags & kKFromRow) klo = max(klo, i0);
  if (g.flags & kKToRow) khi = min(khi, i0 + TM);
  if (g.flags & kKFromCol) klo = max(klo, j0);
  if (g.flags & kKToCol) khi = min(khi, j0 + TN);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // each thread stages 4 values of op(A) and 4 of op(B) per K step
  double ra[4], rb[4];
  auto load = [&](int k0) {
    if (!TA) {
      const int r = t >> 2, kq = (t & 3) * 4, i = i0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + kq + u;
        ra[u] = (i < g.M && k < khi) ? Ap[(size_t)i * g.lda + k] : 0.0;
      }
    } else {
      const int kk = t >> 4, iq = (t & 15) * 4, k = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + iq + u;
        ra[u] = (i < g.M && k < khi) ? Ap[(size_t)k * g.lda + i] : 0.0;
      }
    }
    if (!TB) {
      const int kk = t >> 4, jq = (t & 15) * 4, k = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + jq + u;
        rb[u] = (j < g.N && k < khi) ? Bp[(size_t)k * g.ldb + j] : 0.0;
      }
    } else {
      const int r = t >> 2, kq = (t & 3) * 4, j = j0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + kq + u;
        rb[u] = (j < g.N && k < khi) ? Bp[(size_t)j * g.ldb + k] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
    if (!TA) {
      const int r = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) As[buf][kq + u][r] = ra[u];
    } else {
      const int kk = t >> 4, iq = (t & 15) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) As[buf][kk][iq + u] = ra[u];
    }
    if (!TB) {
      const int kk = t >> 4, jq = (t & 15) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) Bs[buf][kk][jq + u] = rb[u];
    } else {
      const int r = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) Bs[buf][kq + u][r] = rb[u];
    }
  };

  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

  if (klo < khi) {
    load(klo);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = klo; k0 < khi; k0 += TK) {
    const bool more = k0 + TK < khi;
    if (more) load(k0 + TK);  // next tile's global loads in flight during the MFMAs
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
      const double a0 = As[buf][k4 + lk][wm * 32 + lr];
      const double a1 = As[buf][k4 + lk][wm * 32 + 16 + lr];
      const double b0 = Bs[buf][k4 + lk][wn * 32 + lr];
      const double b1 = Bs[buf][k4 + lk][wn * 32 + 16 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + mi * 16 + lk + 4 * r;
        const int j = j0 + wn * 32 + ni * 16 + lr;
        if (i < g.M && j < g.N && (!lower || j <= i)) {
          double c = g.alpha * acc[mi][ni][r];
          if (g.beta != 0.0) c = fma(g.beta, Cp[(size_t)i * g.ldc + j], c);
          Cp[(size_t)i * g.ldc + j] = c;
        }
      }
}

// ---------------------------------------------------------------- leaves (N <= 64)

// Cholesky of a diagonal block (N <= 64) and the inverse of its factor, in LDS.
// Right-looking: at step j every row i > j subtracts a_ij a_cj / a_jj from its trailing
// entries c in (j, i], and the reduced identity rows Y (which become L^{-1}) subtract
// l_ij (Y[j, :] / l_jj), the recurrence of forward substitution on L X = I.  Thread
// (i = t % 64, g = t / 64) owns row i, columns c = g (mod 4): one barrier per step.
// Rows beyond N are padded with the identity.  A non-positive pivot sets *flag.
__global__ __launch_bounds__(256) void k_potrf_inv_leaf(double* A, int N, int lda, int* flag,
                                                        double* Dinv) {
  __shared__ double S[NB][NB + 1];
  __shared__ double Y[NB][NB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    double v = 0.0;
    if (r < N && c <= r) v = A[(size_t)r * lda + c];
    else if (r == c) v = 1.0;
    S[r][c] = v;
    Y[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int i = t & 63, g = t >> 6;
  for (int j = 0; j < NB; ++j) {
    double piv = S[j][j];
    if (!(piv > 0.0)) {
      if (t == 0 && j < N) atomicOr(flag, 1);
      piv = 1.0;
    }
    const double dj = sqrt(piv), inv_dj = 1.0 / dj;
    if (i > j) {
      const double lij = S[i][j] * inv_dj;
      for (int c = j + 1 + ((g - (j + 1)) & 3); c <= i; c += 4)
        S[i][c] = fma(-lij, S[c][j] * inv_dj, S[i][c]);
      for (int c = g; c <= j; c += 4) Y[i][c] = fma(-lij, Y[j][c] * inv_dj, Y[i][c]);
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    const double dr = sqrt(S[r][r] > 0.0 ? S[r][r] : 1.0);
    if (r < N && c < N) {
      double l = 0.0;
      if (c < r) l = S[r][c] / sqrt(S[c][c] > 0.0 ? S[c][c] : 1.0);
      else if (c == r) l = dr;
      A[(size_t)r * lda + c] = l;
    }
    Dinv[e] = (c <= r) ? Y[r][c] / dr : 0.0;
  }
}

// Copy the lower triangle of a 64 x 64 inverse block into an N x N diagonal block.
__global__ void k_put_block(const double* D, double* L, int N, int ldl) {
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int r = e / N, c = e - r * N;
    L[(size_t)r * ldl + c] = (c <= r) ? D[r * NB + c] : 0.0;
  }
}

// ---------------------------------------------------------------- elementwise helpers

__global__ void k_mirror(double* A, int N, int lda) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;  // source tile (bi, bj) with bi >= bj
  if (bj > bi) return;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    int i = bi * 32 + y, j = bj * 32 + tx;
    tile[y][tx] = (i < N && j < N) ? A[(size_t)i * lda + j] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    int i = bj * 32 + y, j = bi * 32 + tx;  // destination (j-tile row)
    if (i < N && j < N && j > i) A[(size_t)i * lda + j] = tile[tx][y];
  }
}

__global__ void k_zero_upper(double* A, int N, int lda) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (i < N && j < N && j > i) A[(size_t)i * lda + j] = 0.0;
}

__global__ void k_transpose(const double* A, int N, int lda, double* B, int ldb) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int y = ty; y < 32; y += 8) {
    int i = bi * 32 + y, j = bj * 32 + tx;
    tile[y][tx] = (i < N && j < N) ? A[(size_t)i * lda + j] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    int i = bj * 32 + y, j = bi * 32 + tx;
    if (i < N && j < N) B[(size_t)i * ldb + j] = tile[tx][y];
  }
}

__global__ __launch_bounds__(256) void k_gemv(const double* __restrict__ A, int N, int lda,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const double* a = A + (size_t)row * lda;
  double s = 0.0;
  for (int c = lane; c < N; c += 64) s = fma(a[c], x[c], s);
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

int split64(int N) {
  int h = (N + 1) / 2;
  int n1 = ((h + NB - 1) / NB) * NB;
  if (n1 >= N) n1 = N - NB;
  return n1;
}

}  // namespace

// Flops of one GEMM call with its tile skipping, and its compulsory bytes.
static void gemm_cost(const GemmArgs& g, double* flops, double* bytes) {
  const int tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
  double f = 0.0;
  const bool lower = (g.flags & kLowerOut) != 0;
  for (int ti = 0; ti < tm; ++ti) {
    const int i0 = ti * TM, ih = std::min(g.M, i0 + TM) - i0;
    for (int tj = 0; tj < tn; ++tj) {
      const int j0 = tj * TN, jh = std::min(g.N, j0 + TN) - j0;
      if (lower && j0 > i0 + TM - 1) continue;
      int klo = 0, khi = g.K;
      if (g.flags & kKFromRow) klo = std::max(klo, i0);
      if (g.flags & kKToRow) khi = std::min(khi, i0 + TM);
      if (g.flags & kKFromCol) klo = std::max(klo, j0);
      if (g.flags & kKToCol) khi = std::min(khi, j0 + TN);
      if (khi > klo) f += 2.0 * ih * jh * (khi - klo);
    }
  }
  *flops = f;
  *bytes = 8.0 * ((double)g.M * g.K + (double)g.K * g.N +
                  (double)g.M * g.N * (g.beta != 0.0 ? 2.0 : 1.0));
}

int gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return LRSDP_OK;
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  ProfMark pm = prof_begin(LRSDP_K_GEMM, s);
  const dim3 grid(tiles, g.offs ? g.batch : 1);
  if (!g.transA && !g.transB)
    k_gemm<false, false><<<grid, 256, 0, s>>>(g);
  else if (!g.transA && g.transB)
    k_gemm<false, true><<<grid, 256, 0, s>>>(g);
  else if (g.transA && !g.transB)
    k_gemm<true, false><<<grid, 256, 0, s>>>(g);
  else
    k_gemm<true, true><<<grid, 256, 0, s>>>(g);
  LRSDP_HIP(hipGetLastError());
  if (pm.kid >= 0) {
    double fl = 0.0, by = 0.0;
    gemm_cost(g, &fl, &by);
    const double nb = g.offs ? g.batch : 1;
    prof_end(pm, s, by * nb, fl * nb);
  }
  return LRSDP_OK;
}

size_t dinv_doubles(int N) { return (size_t)((N + NB - 1) / NB) * NB * NB; }

int potrf(double* A, int N, int lda, int* flag, double* dinv, hipStream_t s) {
  if (N <= 0) return LRSDP_OK;
  if (N <= NB) {
    k_potrf_inv_leaf<<<1, 256, 0, s>>>(A, N, lda, flag, dinv);
    LRSDP_HIP(hipGetLastError());
    return LRSDP_OK;
  }
  const int N1 = split64(N), N2 = N - N1;
  LRSDP_TRY(potrf(A, N1, lda, flag, dinv, s));
  double* A21 = A + (size_t)N1 * lda;
  LRSDP_TRY(trsm_rlt(A21, N2, N1, lda, A, lda, dinv, s));
  GemmArgs g;
  g.M = N2; g.N = N2; g.K = N1;
  g.A = A21; g.lda = lda; g.transA = false;
  g.B = A21; g.ldb = lda; g.transB = true;
  g.C = A21 + N1; g.ldc = lda;
  g.alpha = -1.0; g.beta = 1.0; g.flags = kLowerOut;
  LRSDP_TRY(gemm(g, s));
  return potrf(A21 + N1, N2, lda, flag, dinv + (size_t)(N1 / NB) * NB * NB, s);
}

// The leaf B L^{-T} with N <= 64 is a GEMM against the stored inverse block; it may run in
// place because a single column tile of C covers all N columns and every workgroup reads
// only its own rows of B before it writes them.
int trsm_rlt(double* B, int M, int N, int ldb, const double* L, int ldl, const double* dinv,
             hipStream_t s) {
  if (M <= 0 || N <= 0) return LRSDP_OK;
  if (N <= NB) {
    GemmArgs g;
    g.M = M; g.N = N; g.K = N;
    g.A = B; g.lda = ldb;
    g.B = dinv; g.ldb = NB; g.transB = true;
    g.C = B; g.ldc = ldb;
    return gemm(g, s);
  }
  const int N1 = split64(N), N2 = N - N1;
  LRSDP_TRY(trsm_rlt(B, M, N1, ldb, L, ldl, dinv, s));
  GemmArgs g;
  g.M = M; g.N = N2; g.K = N1;
  g.A = B; g.lda = ldb; g.transA = false;
  g.B = L + (size_t)N1 * ldl; g.ldb = ldl; g.transB = true;
  g.C = B + N1; g.ldc = ldb;
  g.alpha = -1.0; g.beta = 1.0;
  LRSDP_TRY(gemm(g, s));
  return trsm_rlt(B + N1, M, N2, ldb, L + (size_t)N1 * ldl + N1, ldl,
                  dinv + (size_t)(N1 / NB) * NB * NB, s);
}

int trtri(double* L, int N, int ldl, double* tmp, const double* dinv, hipStream_t s) {
  if (N <= 0) return LRSDP_OK;
  if (N <= NB) {
    k_put_block<<<1, 256, 0, s>>>(dinv, L, N, ldl);
    LRSDP_HIP(hipGetLastError());
    return LRSDP_OK;
  }
  const int N1 = split64(N), N2 = N - N1;
  double* L11 = L;
  double* L21 = L + (size_t)N1 * ldl;
  double* L22 = L21 + N1;
  LRSDP_TRY(trtri(L11, N1, ldl, tmp, dinv, s));
  LRSDP_TRY(trtri(L22, N2, ldl, tmp, dinv + (size_t)(N1 / NB) * NB * NB, s));
  GemmArgs g;  // tmp = L21 L11^{-1}
  g.M = N2; g.N = N1; g.K = N1;
  g.A = L21; g.lda = ldl;
  g.B = L11; g.ldb = ldl;
  g.C = tmp; g.ldc = N1;
  g.flags = kKFromCol;
  LRSDP_TRY(gemm(g, s));
  GemmArgs h;  // L21 = -L22^{-1} tmp
  h.M = N2; h.N = N1; h.K = N2;
  h.A = L22; h.lda = ldl;
  h.B = tmp; h.ldb = N1;
  h.C = L21; h.ldc = ldl;
  h.alpha = -1.0; h.beta = 0.0;
  h.flags = kKToRow;
  return gemm(h, s);
}

int lauum(const double* M, int N, int ldm, double* X, int ldx, hipStream_t s) {
  GemmArgs g;
  g.M = N; g.N = N; g.K = N;
  g.A = M; g.lda = ldm; g.transA = true;
  g.B = M; g.ldb = ldm; g.transB = false;
  g.C = X; g.ldc = ldx;
  g.flags = kKFromRow | kKFromCol | kLowerOut;
  return gemm(g, s);
}

int mirror_lower(double* A, int N, int lda, hipStream_t s) {
  const int nt = (N + 31) / 32;
  k_mirror<<<dim3(nt, nt), dim3(32, 8), 0, s>>>(A, N, lda);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int zero_upper(double* A, int N, int lda, hipStream_t s) {
  k_zero_upper<<<dim3((N + 255) / 256, N), 256, 0, s>>>(A, N, lda);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int transpose(const double* A, int N, int lda, double* B, int ldb, hipStream_t s) {
  const int nt = (N + 31) / 32;
  k_transpose<<<dim3(nt, nt), dim3(32, 8), 0, s>>>(A, N, lda, B, ldb);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int gemv(const double* A, int N, int lda, const double* x, double* y, hipStream_t s) {
  ProfMark pm = prof_begin(LRSDP_K_GEMV, s);
  k_gemv<<<(N + 3) / 4, 256, 0, s>>>(A, N, lda, x, y);
  LRSDP_HIP(hipGetLastError());
  prof_end(pm, s, 8.0 * (double)N * N + 16.0 * N, 2.0 * (double)N * N);
  return LRSDP_OK;
}

}  // namespace lrsdp
