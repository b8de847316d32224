// Dense FP64 linear algebra on CDNA4 matrix cores for the setup of Algorithm 1.
//
// GEMM: 64 x 64 (or, for small products, 32 x 32) output tile per workgroup, each wavefront
// owning a 32 x 32 block as 2 x 2 v_mfma_f64_16x16x4_f64 accumulators; K advances 16 at a
// time through double-buffered LDS.
// Operand fragments follow the MFMA register layout: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the 16 x 16 result lives as D[l / 16 + 4 r][l % 16], r = 0..3
// (rows interleaved across the four result registers).
// Triangular operands skip whole zero tiles through per-tile K ranges (GemmFlags), and the
// entries the flags declare zero inside the remaining tiles are staged as zeros unread.
//
// The Cholesky factor and its inverse come out of one recursion (split at a multiple of 64):
// [L11 0; L21 L22] with L21 = A21 L11^{-T}, L22 from A22 - L21 L21^T, and
// (L^{-1})_21 = -L22^{-1} L21 L11^{-1}, so nearly all flops land in the GEMM and no
// triangular solve is sequential beyond the 64 x 64 leaves (register-resident kernels).
#include <algorithm>

#include "dense.h"

namespace lrsdp {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TK = 16;
constexpr int NB = 64;  // leaf size of the recursive factorizations

// Output tile (16 FM WM) x (16 FN WN) per workgroup; each of WM x WN wavefront positions
// owns a (16 FM) x (16 FN) block as FM x FN MFMA accumulators, and KS wavefronts share each
// position by splitting every K chunk of 16 KS columns (intra-workgroup split-K), so one load
// latency covers KS times more K; the KS partial blocks are summed through LDS in a fixed
// order.  Larger blocks per wavefront reuse each LDS operand read for more MFMAs and larger
// tiles re-read less of A and B.
template <bool TA, bool TB, int WM, int WN, int KS, int FM, int FN>
__global__ __launch_bounds__(64 * WM * WN * KS) void k_gemm(GemmArgs g) {
  constexpr int TMv = 16 * FM * WM, TNv = 16 * FN * WN, NT = 64 * WM * WN * KS, TKc = TK * KS;
  constexpr int EA = TMv * TKc / NT, EB = TNv * TKc / NT;  // staged values per thread
  __shared__ double As[2][TKc][TMv + 1];  // odd row pitch: the transposed stores and the
  __shared__ double Bs[2][TKc][TNv + 1];  // MFMA operand reads spread over the banks
  const double* __restrict__ Ap = g.A;
  const double* __restrict__ Bp = g.B;
  double* __restrict__ Cp = g.C;
  if (g.offs) {  // batched: per-z element offsets of A, B, C
    const int z = blockIdx.y;
    Ap += g.offs[3 * z];
    Bp += g.offs[3 * z + 1];
    Cp += g.offs[3 * z + 2];
  }
  const int tiles_m = (g.M + TMv - 1) / TMv, tiles_n = (g.N + TNv - 1) / TNv;
  const bool lower = (g.flags & kLowerOut) != 0;
  // (workgroups are dealt to the eight XCDs in turn, which spreads tiles of unequal K
  // ranges evenly over them; a contiguous tile range per XCD measured slower here)
  const int tile = blockIdx.x;
  const bool tri_grid = lower && tiles_m == tiles_n;
  int ti, tj;
  if (tri_grid) {  // the grid covers only the lower triangle of tiles
    ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    while (ti * (ti + 1) / 2 > tile) --ti;
    tj = tile - ti * (ti + 1) / 2;
  } else if ((g.flags & (kKToCol | kKFromCol)) && !(g.flags & (kKToRow | kKFromRow))) {
    tj = tile / tiles_m;  // the K range follows the tile column: walk the grid column by column
    ti = tile - tj * tiles_m;
  } else {
    ti = tile / tiles_n;
    tj = tile - ti * tiles_n;
  }
  // triangular operands: start with the tiles whose K range is longest (a permutation of the
  // full grid only: on the lower-triangle grid it would send tiles across the diagonal)
  if (!tri_grid && (g.flags & kKToCol)) tj = tiles_n - 1 - tj;
  if (!tri_grid && (g.flags & kKToRow)) ti = tiles_m - 1 - ti;
  const int i0 = ti * TMv, j0 = tj * TNv;
  if (lower && j0 > i0 + TMv - 1) return;
  int klo = 0, khi = g.K;
  if (g.flags & kKFromRow) klo = max(klo, i0);
  if (g.flags & kKToRow) khi = min(khi, i0 + TMv);
  if (g.flags & kKFromCol) klo = max(klo, j0);
  if (g.flags & kKToCol) khi = min(khi, j0 + TNv);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int ks = w / (WM * WN), wmn = w % (WM * WN);
  const int wm = wmn / WN, wn = wmn % WN;
  const int lr = lane & 15, lk = lane >> 4;

  // staging map: consecutive threads walk the contiguous dimension of each operand.  Entries
  // a flag declares zero are staged as zeros without being read, so a triangular operand's
  // other triangle may hold anything (a tile's K range follows its own edges, and a 128-wide
  // diagonal tile would otherwise read the block beside a 64-aligned diagonal block).
  const bool a_from = (g.flags & kKFromRow) != 0, a_to = (g.flags & kKToRow) != 0;
  const bool b_from = (g.flags & kKFromCol) != 0, b_to = (g.flags & kKToCol) != 0;
  double ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = t + u * NT;
      int i, k;
      if (!TA) {
        i = i0 + e / TKc;
        k = k0 + e % TKc;
      } else {
        i = i0 + e % TMv;
        k = k0 + e / TMv;
      }
      const bool nz = i < g.M && k < khi && !(a_from && k < i) && !(a_to && k > i);
      ra[u] = nz ? (TA ? Ap[(size_t)k * g.lda + i] : Ap[(size_t)i * g.lda + k]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = t + u * NT;
      int j, k;
      if (!TB) {
        j = j0 + e % TNv;
        k = k0 + e / TNv;
      } else {
        j = j0 + e / TKc;
        k = k0 + e % TKc;
      }
      const bool nz = j < g.N && k < khi && !(b_from && k < j) && !(b_to && k > j);
      rb[u] = nz ? (TB ? Bp[(size_t)j * g.ldb + k] : Bp[(size_t)k * g.ldb + j]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = t + u * NT;
      if (!TA) As[buf][e % TKc][e / TKc] = ra[u];
      else As[buf][e / TMv][e % TMv] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = t + u * NT;
      if (!TB) Bs[buf][e / TNv][e % TNv] = rb[u];
      else Bs[buf][e % TKc][e / TKc] = rb[u];
    }
  };

  v4d acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

  if (klo < khi) {
    load(klo);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = klo; k0 < khi; k0 += TKc) {
    const bool more = k0 + TKc < khi;
    if (more) load(k0 + TKc);  // next chunk's global loads in flight during the MFMAs
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
      const int kr = ks * TK + k4 + lk;
      double av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) av[a] = As[buf][kr][wm * 16 * FM + 16 * a + lr];
#pragma unroll
      for (int b = 0; b < FN; ++b) bv[b] = Bs[buf][kr][wn * 16 * FN + 16 * b + lr];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  if constexpr (KS > 1) {  // fold the K slices: wavefronts ks > 0 park their blocks in LDS
    constexpr int PB = 64 * 4 * FM * FN;  // doubles parked per wavefront
    static_assert((KS - 1) * WM * WN * PB <= 2 * TKc * (TMv + 1), "LDS too small");
    double* park = &As[0][0][0];
    if (ks > 0) {
      double* mine = park + ((size_t)(ks - 1) * WM * WN + wmn) * PB;
#pragma unroll
      for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
#pragma unroll
          for (int r = 0; r < 4; ++r) mine[((mi * FN + ni) * 4 + r) * 64 + lane] = acc[mi][ni][r];
    }
    __syncthreads();
    if (ks > 0) return;
#pragma unroll
    for (int o = 1; o < KS; ++o) {
      const double* theirs = park + ((size_t)(o - 1) * WM * WN + wmn) * PB;
#pragma unroll
      for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mi][ni][r] += theirs[((mi * FN + ni) * 4 + r) * 64 + lane];
    }
  }

#pragma unroll
  for (int mi = 0; mi < FM; ++mi)
#pragma unroll
    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 16 * FM + mi * 16 + lk + 4 * r;
        const int j = j0 + wn * 16 * FN + ni * 16 + lr;
        if (i < g.M && j < g.N && (!lower || j <= i)) {
          double c = (g.alpha_dev ? *g.alpha_dev : g.alpha) * acc[mi][ni][r];
          if (g.beta != 0.0) c = fma(g.beta, Cp[(size_t)i * g.ldc + j], c);
          Cp[(size_t)i * g.ldc + j] = c;
        }
      }
}

// ---------------------------------------------------------------- leaf (N <= 64)


__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 1/sqrt(x) for x > 0: hardware estimate plus two Newton steps (a few ulp; the
// factorization does not need correct rounding).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Cholesky factor L of a diagonal block (N <= 64) and L^{-1}, by 8-column panels.
// Wavefront g owns the matrix columns [8g, 8g + 8) and the rows [8g, 8g + 8) of L^{-1}, both
// as MFMA accumulators of a 64 x 16 block (four 16 x 16 tiles; columns 8..15 stay zero): the
// matrix block as it is, the L^{-1} rows transposed.  Between barrier P - 1 and barrier P:
//   wavefront P factors panel P alone: it moves its block to rows-in-lanes form through LDS
//   (lane i holds row i), takes the pivots and l_cj by cross-lane reads, and publishes the
//   panel's columns;
//   wavefront P - 1 finishes rows [8(P-1), 8P) of L^{-1} the same way (an 8 x 8 forward
//   substitution whose coefficients are its panel's l values) and publishes them.
// After barrier P every wavefront g > P applies panel P's rank-8 update to its matrix
// columns, and the wavefronts g >= P apply panel P - 1's update to their rows of L^{-1}; the
// wavefront that factors panel P + 1 defers that one until after the next barrier.  Each
// update is a 64 x 8 x 8 product on the matrix cores, whose operands every lane reads from
// LDS once (lane-distinct values) instead of every lane reading the same 8 x 8 block; the
// products add their terms in the unblocked algorithm's order (the factors came out bit for
// bit equal to those of one FMA per term).  Only
// the lower triangle of the matrix block is L: rows above a wavefront's columns are not
// updated, and panels are published with zeros there.  Rows and columns beyond N are the
// identity.  A non-positive pivot sets *flag (the result is then garbage).  Writes L (lower,
// zero above the diagonal) into A and L^{-1} (zero above the diagonal) into Li
// (li_rows x li_rows).
constexpr int LW = NB / 8;   // wavefronts of the leaf kernel
constexpr int LP = NB / LW;  // panel width = columns (rows of L^{-1}) per wavefront
static_assert(LP == 8 && NB == 64, "8-column panels of a 64-row block in 16 x 16 x 4 MFMAs");

// LDS of the leaf: Ls[4][NB][LP + 1] (panel P's columns of L, row-indexed, buffer P % 4)
// and Xs[2][LP][NB] (panel P's rows of L^{-1}, buffer P % 2); separately Cv[2][NB][LP + 1]
// (the form change of the factoring wavefront's block, 0, and of the finishing one's, 1).
constexpr int kLeafLds = 4 * NB * (LP + 1) + 2 * LP * NB;  // doubles
constexpr int kLeafConv = 2 * NB * (LP + 1);               // doubles

// The leaf's work by its NB * LW threads.  The block comes from A (global, row pitch lda) or,
// when Ain is given, from LDS (row pitch NB + 1); L goes to A in either case.
__device__ __forceinline__ void leaf_factor(double* __restrict__ A, int N, int lda,
                                            const double* Ain, int* flag,
                                            double* __restrict__ Li, int ldi, int li_rows,
                                            double* lds, double* conv) {
  double(*Ls)[NB][LP + 1] = reinterpret_cast<double(*)[NB][LP + 1]>(lds);
  double(*Xs)[LP][NB] = reinterpret_cast<double(*)[LP][NB]>(lds + 4 * NB * (LP + 1));
  double(*Cv)[NB][LP + 1] = reinterpret_cast<double(*)[NB][LP + 1]>(conv);
  const int t = threadIdx.x, i = t & (NB - 1), g = t / NB;
  const int lr = i & 15, lk = i >> 4;  // MFMA roles: tile row / column lr, K or row group lk
  // ca: this wavefront's matrix columns; cy: its rows of L^{-1}, transposed (row = column
  // of L^{-1}).  Tile u, register r: row 16u + lk + 4r, column LP g + lr (lr < LP).
  v4d ca[4], cy[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * u + lk + 4 * r, col = g * LP + lr;
      double v = 0.0;
      if (lr < LP) {
        if (row < N && col <= row) v = Ain ? Ain[row * (NB + 1) + col] : A[(size_t)row * lda + col];
        else if (row == col) v = 1.0;
      }
      ca[u][r] = v;
      cy[u][r] = (lr < LP && row == col) ? 1.0 : 0.0;
    }
  double a[LP], y[LP], inv[LP];  // rows-in-lanes forms; 1 / l_jj of this wavefront's panel
#pragma unroll
  for (int q = 0; q < LP; ++q) a[q] = y[q] = inv[q] = 0.0;
  bool bad = false;
  // acc(tiles u0..3) -= (64 x 8 block of rows 16u + m, entry opnd(16u + m, k)) x
  // (panel p's rows [LP g, LP g + LP))^T
  auto update = [&](v4d(&acc)[4], int u0, int u1, int lb, auto opnd) {
    double bq[2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) bq[kk] = lr < LP ? Ls[lb][g * LP + lr][4 * kk + lk] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < u0 || u > u1) continue;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-opnd(16 * u + lr, 4 * kk + lk), bq[kk],
                                                      acc[u], 0, 0, 0);
    }
  };
  // the block of acc into rows-in-lanes form out[q] = block(row i, column q), via Cv[cb]
  auto to_rows = [&](const v4d(&acc)[4], int cb, double(&out)[LP]) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (lr < LP) Cv[cb][16 * u + lk + 4 * r][lr] = acc[u][r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < LP; ++q) out[q] = Cv[cb][i][q];
  };
  // this wavefront's rows of L^{-1} -= (panel p's l_cj) x (panel p's rows of L^{-1}); the
  // rows of L^{-1} of panel p are zero beyond column LP p + LP - 1
  auto y_update = [&](int p) {
    const int xb = p & 1;
    update(cy, 0, (LP * p + LP - 1) >> 4, p & 3,
           [&](int row, int k) { return Xs[xb][k][row]; });
  };
  for (int P = 0; P <= LW; ++P) {
    const int j0 = P * LP;
    if (P < LW && g == P) {  // factor panel P: every update from panels < P is in
      to_rows(ca, 0, a);
      const int jl0 = __builtin_amdgcn_readfirstlane(j0);
#pragma unroll
      for (int jj = 0; jj < LP; ++jj) {
        const double piv = readlane_d(a[jj], jl0 + jj);
        bad |= !(piv > 0.0) && (j0 + jj < N);
        inv[jj] = rsqrt_nr(piv);
        const double l = a[jj] * inv[jj];
        a[jj] = l;
#pragma unroll
        for (int qq = jj + 1; qq < LP; ++qq) a[qq] = fma(-l, readlane_d(l, jl0 + qq), a[qq]);
      }
#pragma unroll
      for (int q = 0; q < LP; ++q) Ls[P & 3][i][q] = (i >= j0 + q) ? a[q] : 0.0;
      __builtin_amdgcn_s_setprio(0);
    }
    if (P >= 1 && g == P - 1) {  // rows of L^{-1} of panel P - 1: all updates are in
      to_rows(cy, 1, y);
      const int jl0 = __builtin_amdgcn_readfirstlane(j0 - LP);
#pragma unroll
      for (int jj = 0; jj < LP; ++jj) {
        y[jj] *= inv[jj];
#pragma unroll
        for (int kk = jj + 1; kk < LP; ++kk)
          y[kk] = fma(-readlane_d(a[jj], jl0 + kk), y[jj], y[kk]);
      }
#pragma unroll
      for (int q = 0; q < LP; ++q) Xs[(P - 1) & 1][q][i] = y[q];
    }
    if (P == LW) break;
    __syncthreads();
    // the next panel's wavefront issues first on its SIMD (its update is on the critical path);
    // it drops back to normal priority once it has published its panel
    if (g == P + 1) __builtin_amdgcn_s_setprio(2);
    if (g > P) {  // rank-8 update of this wavefront's matrix columns (rows >= LP g) by panel P
      const int lb = P & 3;
      update(ca, (g * LP) >> 4, 3, lb, [&](int row, int k) { return Ls[lb][row][k]; });
    }
    if (g == P && P >= 2) y_update(P - 2);  // deferred while this wavefront factored
    if (P >= 1 && g >= P && g != P + 1) y_update(P - 1);
  }
  if (bad && i == 0) atomicOr(flag, 1);
#pragma unroll
  for (int q = 0; q < LP; ++q) {
    const int c = g * LP + q;
    if (i < N && c < N) A[(size_t)i * lda + c] = (c <= i) ? a[q] : 0.0;
    // lane i holds column i of row c of L^{-1}
    if (c < li_rows && i < li_rows) Li[(size_t)c * ldi + i] = (i <= c) ? y[q] : 0.0;
  }
}

__global__ __launch_bounds__(NB * LW) void k_chol_leaf(double* __restrict__ A, int N, int lda,
                                                       int* flag, double* __restrict__ Li,
                                                       int ldi, int li_rows) {
  __shared__ double lds[kLeafLds];
  __shared__ double conv[kLeafConv];
  leaf_factor(A, N, lda, nullptr, flag, Li, ldi, li_rows, lds, conv);
}

// ---------------------------------------------------------------- right-looking node
// Below a few thousand rows the recursion's cost is its chain of small launches, not its
// flops.  There a node is factored right-looking by 64-blocks, one launch per block column
// j.  L^{-1} = X is built alongside from its block recurrence
// X_ik = -L_ii^{-1} sum_{k <= m < i} L_im X_mk: the sums Y_ik accumulate in Li as the block
// columns m finish, and X_ik = L_ii^{-1} Y_ik once L_ii^{-1} is known.  Every block product is
// one 64 x 64 x 64 MFMA tile.
//
// The panel of column j (L_ij = A_ij L_jj^{-T} and X_jk = L_jj^{-1} Y_jk) is not a launch of
// its own: each tile of step j that needs a panel block forms it in LDS from A_ij or Y_jk, and
// the panel blocks are stored in place by step j + 1, when nothing reads their old values
// any more (two small launches store the last two panels).  Recomputed blocks are the same
// tile products on the same operands, so every stored value is the one a separate panel
// launch would store.

__device__ __forceinline__ int rl_rows(int b, int N) { return min(64, N - 64 * b); }

// Ps/Qs <- the 64 x 64 operand blocks of P op(Q) (entries past Mv rows / Nv columns / Kv of
// K read as zero): Ps[k][m] = P[m][k], Qs[k][n] = op(Q)[k][n].  Ends with a barrier.
__device__ __forceinline__ void tile_load(const double* P, int ldp, const double* Q, int ldq,
                                          bool qT, int Mv, int Nv, int Kv, double (*Ps)[65],
                                          double (*Qs)[65]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double pv[8], qv[8];  // all loads in flight before the first LDS store
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int rr = w + 8 * u, cc = lane;
    pv[u] = (rr < Mv && cc < Kv) ? P[(size_t)rr * ldp + cc] : 0.0;
    qv[u] = (qT ? (rr < Nv && cc < Kv) : (rr < Kv && cc < Nv)) ? Q[(size_t)rr * ldq + cc] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int rr = w + 8 * u, cc = lane;
    Ps[cc][rr] = pv[u];
    if (qT) Qs[cc][rr] = qv[u];
    else Qs[rr][cc] = qv[u];
  }
  __syncthreads();
}

// acc = (the product of the blocks in Ps, Qs) by 512 threads: wavefront w computes the
// 32 x 32 quadrant ((w >> 1) & 1, w & 1) over the K half w >> 2, and the upper half parks its
// partial sums in `park` (64 x 64 doubles of LDS, which may alias Ps) for the lower half to
// add.  Every wavefront passes the same barriers; returns true on the lower four, which then
// hold the product.
__device__ __forceinline__ bool tile_mma(const double (*Ps)[65], const double (*Qs)[65],
                                         double* park, v4d (&acc)[2][2]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, kh = w >> 2, wm = (w >> 1) & 1, wn = w & 1;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k4 = 0; k4 < 32; k4 += 4) {
    const int kr = 32 * kh + k4 + lk;
    const double a0 = Ps[kr][wm * 32 + lr];
    const double a1 = Ps[kr][wm * 32 + 16 + lr];
    const double b0 = Qs[kr][wn * 32 + lr];
    const double b1 = Qs[kr][wn * 32 + 16 + lr];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  __syncthreads();  // every wavefront is done with the operands (park may alias Ps)
  double* mine = park + (size_t)(w & 3) * 64 * 16;
  if (kh == 1) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int q = 0; q < 4; ++q) mine[((mi * 2 + ni) * 4 + q) * 64 + lane] = acc[mi][ni][q];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[mi][ni][q] += mine[((mi * 2 + ni) * 4 + q) * 64 + lane];
  }
  __syncthreads();  // park is free again
  return kh == 0;
}

// H <- the product held by the lower wavefronts, transposed (H[c][i] = acc(i, c), the layout
// of an operand block loaded into Ps, or into Qs with qT) or not (H[i][c], Qs without qT).
// Ends with a barrier.
__device__ __forceinline__ void tile_stash(bool lower, const v4d (&acc)[2][2], bool transposed,
                                           double (*H)[65]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, wm = (w >> 1) & 1, wn = w & 1;
  const int lr = lane & 15, lk = lane >> 4;
  if (lower) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = wm * 32 + mi * 16 + lk + 4 * q, c = wn * 32 + ni * 16 + lr;
          if (transposed) H[c][i] = acc[mi][ni][q];
          else H[i][c] = acc[mi][ni][q];
        }
  }
  __syncthreads();
}

// C (Mv x Nv at ldc) = alpha acc + beta cv by the lower wavefronts
__device__ __forceinline__ void tile_store(bool lower, const v4d (&acc)[2][2],
                                           const double (&cv)[2][2][4], double* C, int ldc,
                                           int Mv, int Nv, double alpha, double beta) {
  if (!lower) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, wm = (w >> 1) & 1, wn = w & 1;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = wm * 32 + mi * 16 + lk + 4 * q;
        const int c = wn * 32 + ni * 16 + lr;
        if (i < Mv && c < Nv) {
          double v = alpha * acc[mi][ni][q];
          if (beta != 0.0) v = fma(beta, cv[mi][ni][q], v);
          C[(size_t)i * ldc + c] = v;
        }
      }
}

// cv <- the block of C that the lower wavefronts will store into (entries past Mv x Nv, and
// above the diagonal when lowerOnly, read as zero)
__device__ __forceinline__ void tile_old(const double* C, int ldc, int Mv, int Nv,
                                         bool lowerOnly, double (&cv)[2][2][4]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, kh = w >> 2, wm = (w >> 1) & 1, wn = w & 1;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = wm * 32 + mi * 16 + lk + 4 * q, c = wn * 32 + ni * 16 + lr;
        cv[mi][ni][q] = (kh == 0 && i < Mv && c < Nv && (!lowerOnly || c <= i))
                            ? C[(size_t)i * ldc + c] : 0.0;
      }
}

// acc = the product of the blocks in Ps, Qs when op(Q) is upper triangular (Qs[k][n] = 0 for
// k > n: the factor L_jj^{-T} of a panel block L_ij = A_ij L_jj^{-T}), by 512 threads with K
// unsplit: the 16 x 16 output tile (ti, tc) sums its nonzero K range [0, 16 tc + 16) in one
// MFMA chain.  Wavefront w computes the tiles (w & 3, 3) and (w & 3, 0) when w < 4, else
// (w & 3, 2) and (w & 3, 1): 20 MFMAs each (40 per SIMD) instead of 32, and no partial sums
// to fold.  Ends with a barrier (Ps and Qs are free again).
__device__ __forceinline__ void tile_mma_uq(const double (*Ps)[65], const double (*Qs)[65],
                                            v4d (&acc)[2]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, ti = w & 3;
  const int lr = lane & 15, lk = lane >> 4;
  const int tc0 = w < 4 ? 3 : 2, tc1 = 3 - tc0;
  acc[0] = acc[1] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k16 = 0; k16 < 16 * tc0 + 16; k16 += 16) {
    const bool both = k16 < 16 * tc1 + 16;
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      const int kr = k16 + k4 + lk;
      const double a = Ps[kr][16 * ti + lr];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Qs[kr][16 * tc0 + lr], acc[0], 0, 0, 0);
      if (both)
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Qs[kr][16 * tc1 + lr], acc[1], 0, 0, 0);
    }
  }
  __syncthreads();
}

// H[c][i] = acc(i, c) for the tiles of tile_mma_uq (the layout of an operand block loaded
// into Ps, or into Qs with qT).  Ends with a barrier.
__device__ __forceinline__ void tile_stash_uq(const v4d (&acc)[2], double (*H)[65]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, ti = w & 3;
  const int lr = lane & 15, lk = lane >> 4;
  const int tc0 = w < 4 ? 3 : 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = 16 * (h == 0 ? tc0 : 3 - tc0) + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) H[c][16 * ti + lk + 4 * q] = acc[h][q];
  }
  __syncthreads();
}

// C (Mv x Nv at ldc) = the product of tile_mma_uq
__device__ __forceinline__ void tile_store_uq(const v4d (&acc)[2], double* C, int ldc, int Mv,
                                              int Nv) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, ti = w & 3;
  const int lr = lane & 15, lk = lane >> 4;
  const int tc0 = w < 4 ? 3 : 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = 16 * (h == 0 ? tc0 : 3 - tc0) + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * ti + lk + 4 * q;
      if (i < Mv && c < Nv) C[(size_t)i * ldc + c] = acc[h][q];
    }
  }
}

// The lower 16 x 16 tiles of a symmetric product H^T H (H[k][m] = P[m][k], so the product is
// P P^T): ten tiles, each K = 64 in two halves, make 20 MFMA chains of 8; wavefront w takes
// jobs w, w + 8 and w + 16 (< 20), five per SIMD.  Job j is the half j / 10 of lower tile
// j % 10 (row-major: (0,0), (1,0), (1,1), (2,0), ...).  The second halves are parked in
// `park` (2560 doubles, may alias neither H nor Out) and added to the first in that order;
// Out[i][c] (row pitch 65) = Cv(i, c) - the product, with Cv read from C (rows past Mv and
// entries above the diagonal as zero).  Entries of Out above the diagonal tiles are not written,
// those above the diagonal inside a diagonal tile are garbage.  Ends with a barrier.
__device__ __forceinline__ void tile_syrk_lower(const double (*H)[65], const double* C, int ldc,
                                                int Mv, double* park, double* Out) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  auto tile_i = [](int t) { return t >= 6 ? 3 : t >= 3 ? 2 : t >= 1 ? 1 : 0; };
  auto tile_c = [&](int t) { const int i = tile_i(t); return t - i * (i + 1) / 2; };
  v4d acc[3];
  double cv[3][4];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int j = w + 8 * s, t = j % 10;
    const int ti = tile_i(t), tc = tile_c(t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * ti + lk + 4 * q, c = 16 * tc + lr;
      cv[s][q] = (j < 10 && i < Mv && c <= i) ? C[(size_t)i * ldc + c] : 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int j = w + 8 * s;
    acc[s] = (v4d){0.0, 0.0, 0.0, 0.0};
    if (j >= 20) continue;
    const int t = j % 10, k0 = 32 * (j / 10);
    const int ti = tile_i(t), tc = tile_c(t);
#pragma unroll
    for (int k4 = 0; k4 < 32; k4 += 4) {
      const int kr = k0 + k4 + lk;
      acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(H[kr][16 * ti + lr], H[kr][16 * tc + lr],
                                                    acc[s], 0, 0, 0);
    }
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int j = w + 8 * s;
    if (j >= 10 && j < 20) {
#pragma unroll
      for (int q = 0; q < 4; ++q) park[((j - 10) * 4 + q) * 64 + lane] = acc[s][q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int j = w + 8 * s;
    if (j < 10) {
      const int ti = tile_i(j), tc = tile_c(j);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v = acc[s][q] + park[(j * 4 + q) * 64 + lane];
        Out[(16 * ti + lk + 4 * q) * 65 + 16 * tc + lr] = cv[s][q] - v;
      }
    }
  }
  __syncthreads();
}

// Tile tp of the panel of column jp (r = nb - 1 - jp):
//   tp < r:         L_ij = A_ij L_jj^{-T}, i = jp + 1 + tp (in place in A);
//   r <= tp < r+jp: X_jk = L_jj^{-1} Y_jk, k = tp - r (in place in Li).
__device__ __forceinline__ void panel_tile(double* A, int lda, double* Li, int ldi, int N,
                                           int jp, int tp, double (*Ps)[65], double (*Qs)[65]) {
  const int nb = (N + 63) >> 6, r = nb - 1 - jp;
  const double* Ljinv = Li + (size_t)(64 * jp) * ldi + 64 * jp;
  v4d acc[2][2];
  double cv[2][2][4] = {};
  if (tp < r) {
    const int i = jp + 1 + tp;
    double* C = A + (size_t)(64 * i) * lda + 64 * jp;
    tile_load(C, lda, Ljinv, ldi, true, rl_rows(i, N), 64, 64, Ps, Qs);
    v4d au[2];
    tile_mma_uq(Ps, Qs, au);
    tile_store_uq(au, C, lda, rl_rows(i, N), 64);
  } else {
    const int k = tp - r, mj = rl_rows(jp, N);
    double* C = Li + (size_t)(64 * jp) * ldi + 64 * k;
    tile_load(Ljinv, ldi, C, ldi, false, mj, 64, mj, Ps, Qs);
    const bool lo = tile_mma(Ps, Qs, &Ps[0][0], acc);
    tile_store(lo, acc, cv, C, ldi, mj, 64, 1.0, 0.0);
  }
}

// The panel of column j alone (the last two columns of a node).
__global__ __launch_bounds__(512) void k_rl_panel(double* __restrict__ A, int lda,
                                                  double* __restrict__ Li, int ldi, int N,
                                                  int j) {
  __shared__ double Ps[64][65];  // odd row pitch against bank conflicts
  __shared__ double Qs[64][65];
  panel_tile(A, lda, Li, ldi, N, j, blockIdx.x, Ps, Qs);
}

// Step j of a node (r = nb - 1 - j >= 1), one block product chain per workgroup:
//   tile 0:                  L_dj (d = j + 1) formed, A_dd -= L_dj L_dj^T into LDS, then the
//                            leaf of block d (its Cholesky factor and inverse);
//   tiles t < r(r+1)/2:      A_ik -= L_ij L_kj^T, j < k <= i, (i, k) != (d, d), with L_ij and
//                            L_kj formed from A_ij, A_kj;
//   next r (j + 1) tiles:    Y_ik = [k < j] Y_ik - L_ij X_jk, i > j, k <= j, with L_ij and
//                            (k < j) X_jk formed from A_ij, Y_jk (X_jj = L_jj^{-1} is stored);
//   the rest:                the stores of the panel of column j - 1.
// The blocks a tile writes are read by no other tile of the launch.
__global__ __launch_bounds__(512) void k_rl_fused(double* __restrict__ A, int lda,
                                                  double* __restrict__ Li, int ldi, int N,
                                                  int j, int* flag) {
  static_assert(NB == 64 && NB * LW == 512 && kLeafLds <= 64 * 65 && kLeafConv <= 64 * 65,
                "leaf inside a tile step");
  __shared__ double Ps[64][65];
  __shared__ double Qs[64][65];
  __shared__ double H1[64][65];  // formed panel blocks
  __shared__ double H2[64][65];
  const int nb = (N + 63) >> 6, r = nb - 1 - j, t = blockIdx.x;
  const int ta = r * (r + 1) / 2, ty = ta + r * (j + 1);
  const double* Ljinv = Li + (size_t)(64 * j) * ldi + 64 * j;
  v4d acc[2][2];
  double cv[2][2][4];
  if (t >= ty) {  // deferred stores of the previous column's panel
    panel_tile(A, lda, Li, ldi, N, j - 1, t - ty, Ps, Qs);
    return;
  }
  if (t == 0) {  // A_dd -= L_dj L_dj^T, then the leaf of block d
    const int d = j + 1, nd = rl_rows(d, N);
    double* Add = A + (size_t)(64 * d) * lda + 64 * d;
    tile_load(A + (size_t)(64 * d) * lda + 64 * j, lda, Ljinv, ldi, true, nd, 64, 64, Ps, Qs);
    v4d au[2];
    tile_mma_uq(Ps, Qs, au);
    tile_stash_uq(au, H1);
    double* Al = &Qs[0][0];  // the updated block, row pitch NB + 1
    tile_syrk_lower(H1, Add, lda, nd, &Ps[0][0], Al);
    leaf_factor(Add, nd, lda, Al, flag, Li + (size_t)(64 * d) * ldi + 64 * d, ldi, nd,
                &Ps[0][0], &H1[0][0]);
    return;
  }
  if (t < ta) {  // A_ik -= L_ij L_kj^T
    int ii = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
    while (ii * (ii + 1) / 2 > t) --ii;
    const int i = j + 1 + ii, k = j + 1 + (t - ii * (ii + 1) / 2);
    const int mi = rl_rows(i, N), mk = rl_rows(k, N);
    double* C = A + (size_t)(64 * i) * lda + 64 * k;
    tile_old(C, lda, mi, mk, false, cv);
    tile_load(A + (size_t)(64 * i) * lda + 64 * j, lda, Ljinv, ldi, true, mi, 64, 64, Ps, Qs);
    v4d au[2];
    tile_mma_uq(Ps, Qs, au);
    tile_stash_uq(au, H1);
    if (k != i) {
      tile_load(A + (size_t)(64 * k) * lda + 64 * j, lda, Ljinv, ldi, true, mk, 64, 64, Ps, Qs);
      tile_mma_uq(Ps, Qs, au);
      tile_stash_uq(au, H2);
    }
    const bool lo = tile_mma(H1, k != i ? H2 : H1, &Ps[0][0], acc);
    tile_store(lo, acc, cv, C, lda, mi, mk, -1.0, 1.0);
    return;
  }
  {  // Y_ik = [k < j] Y_ik - L_ij X_jk
    const int i = j + 1 + (t - ta) / (j + 1), k = (t - ta) % (j + 1);
    const int mi = rl_rows(i, N);
    double* C = Li + (size_t)(64 * i) * ldi + 64 * k;
    const double beta = (k < j) ? 1.0 : 0.0;
    tile_old(C, ldi, beta != 0.0 ? mi : 0, 64, false, cv);
    tile_load(A + (size_t)(64 * i) * lda + 64 * j, lda, Ljinv, ldi, true, mi, 64, 64, Ps, Qs);
    v4d au[2];
    tile_mma_uq(Ps, Qs, au);
    tile_stash_uq(au, H1);
    bool lo;
    if (k < j) {  // X_jk = L_jj^{-1} Y_jk
      tile_load(Ljinv, ldi, Li + (size_t)(64 * j) * ldi + 64 * k, ldi, false, 64, 64, 64, Ps,
                Qs);
      lo = tile_mma(Ps, Qs, &Ps[0][0], acc);
      tile_stash(lo, acc, false, H2);
      lo = tile_mma(H1, H2, &Ps[0][0], acc);
    } else {      // X_jj = L_jj^{-1}, stored by the leaf
      tile_load(Ljinv, ldi, Ljinv, ldi, false, 0, 64, 64, Ps, Qs);
      lo = tile_mma(H1, Qs, &Ps[0][0], acc);
    }
    tile_store(lo, acc, cv, C, ldi, mi, 64, -1.0, beta);
  }
}

__global__ void k_copy_block(const double* __restrict__ S, int lds, double* __restrict__ D,
                             int ldd, int M, int N) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (idx >= (size_t)M * N) return;
  const int i = (int)(idx / N), j = (int)(idx - (size_t)i * N);
  D[(size_t)i * ldd + j] = S[(size_t)i * lds + j];
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

// y = tri(A) x for rows r < R of A, with tri the lower (upper = 0: columns [0, min(r + 1, C)))
// or upper (upper = 1: columns [r, C)) part including the diagonal.  One wavefront per row,
// eight independent accumulators so that eight loads per lane are in flight (the rows are long
// and the product is bound by HBM).  kAcc: y += the product.  When y2 is given, the row's result
// is also stored there (y2[r] += it when acc2).  (A vector x - xs is formed first, k_sub_vec.)
template <bool kAcc>
__device__ __forceinline__ void gemv_tri_body(int bx, const double* __restrict__ A, int R, int C,
                                              int lda, const double* __restrict__ x,
                                              double* __restrict__ y, int upper,
                                              double* __restrict__ y2, int acc2) {
  const int lane = threadIdx.x & 63;
  const int row = bx * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const double* a = A + (size_t)row * lda;
  const int lo = upper ? row : 0, hi = upper ? C : min(row + 1, C);
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = lo + lane;
  for (; c + 7 * 64 < hi; c += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = fma(a[c + u * 64], x[c + u * 64], s[u]);
  }
  for (int u = 0; c < hi; c += 64, ++u) s[u] = fma(a[c], x[c], s[u]);
  double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  t = wave_sum(t);
  if (lane == 0) {
    y[row] = kAcc ? y[row] + t : t;
    if (y2) y2[row] = acc2 ? y2[row] + t : t;
  }
}
template <bool kAcc>
__global__ __launch_bounds__(256) void k_gemv_tri(const double* __restrict__ A, int R, int C,
                                                  int lda, const double* __restrict__ x,
                                                  double* __restrict__ y, int upper,
                                                  double* __restrict__ y2, int acc2) {
  gemv_tri_body<kAcc>(blockIdx.x, A, R, C, lda, x, y, upper, y2, acc2);
}
// lock-step batch (packed grid): y = tri(L^{-1} or L^{-T}) x with the instance's Sinv
template <bool kAcc>
__global__ __launch_bounds__(256) void k_gemv_tri_b(const BL b, int xr, int yr, int upper) {
  int bx;
  const int z = bl_find(b, kKgemv, blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  gemv_tri_body<kAcc>(bx, d.Sinv, d.nk, d.nk, d.nk, d.v[xr], d.v[yr], upper, nullptr, 0);
}

// d = x - xs, each difference rounded once.  (The triangular GEMVs then read one vector: with
// x - xs formed inside them the compiler keeps fewer loads in flight, 40 VGPRs against 64, and
// the product took 18 us against 9 at 2528 rows.)
__global__ __launch_bounds__(256) void k_sub_vec(int N, const double* __restrict__ x,
                                                 const double* __restrict__ xs,
                                                 double* __restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N) d[i] = x[i] - xs[i];
}

// lock-step batch (packed grid): d = x - xs over the instance's nk entries
__global__ __launch_bounds__(256) void k_sub_vec_b(const BL b, int xr, int xsr, int dr) {
  int bx;
  const int z = bl_find(b, kKnk256, blockIdx.x, &bx);
  if (!b.act[z]) return;
  const BInst& d = b.I[z];
  const int i = bx * 256 + threadIdx.x;
  if (i < d.nk) d.v[dr][i] = d.v[xr][i] - d.v[xsr][i];
}

// y[r] = (b[r] - bs[r]) - sum_{c < K} A[r][c] x[c] for rows r < R (kSub; else b[r] - ...), one
// wavefront per row with eight loads in flight per lane, like k_gemv_tri.
template <bool kSub>
__global__ __launch_bounds__(256) void k_gemv_rect(const double* __restrict__ A, int R, int K,
                                                   int lda, const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ bs,
                                                   double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const double* a = A + (size_t)row * lda;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = lane;
  for (; c + 7 * 64 < K; c += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = fma(a[c + u * 64], x[c + u * 64], s[u]);
  }
  for (int u = 0; c < K; c += 64, ++u) s[u] = fma(a[c], x[c], s[u]);
  double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  t = wave_sum(t);
  if (lane == 0) y[row] = (kSub ? b[row] - bs[row] : b[row]) - t;
}

int split64(int N) {
  int h = (N + 1) / 2;
  int n1 = ((h + NB - 1) / NB) * NB;
  if (n1 >= N) n1 = N - NB;
  return n1;
}

}  // namespace

// Flops of one GEMM call with its tile skipping (tile edge te), and its compulsory bytes.
static void gemm_cost(const GemmArgs& g, int te, double* flops, double* bytes) {
  const int tm = (g.M + te - 1) / te, tn = (g.N + te - 1) / te;
  double f = 0.0;
  const bool lower = (g.flags & kLowerOut) != 0;
  for (int ti = 0; ti < tm; ++ti) {
    const int i0 = ti * te, ih = std::min(g.M, i0 + te) - i0;
    for (int tj = 0; tj < tn; ++tj) {
      const int j0 = tj * te, jh = std::min(g.N, j0 + te) - j0;
      if (lower && j0 > i0 + te - 1) continue;
      int klo = 0, khi = g.K;
      if (g.flags & kKFromRow) klo = std::max(klo, i0);
      if (g.flags & kKToRow) khi = std::min(khi, i0 + te);
      if (g.flags & kKFromCol) klo = std::max(klo, j0);
      if (g.flags & kKToCol) khi = std::min(khi, j0 + te);
      if (khi > klo) f += 2.0 * ih * jh * (khi - klo);
    }
  }
  *flops = f;
  *bytes = 8.0 * ((double)g.M * g.K + (double)g.K * g.N +
                  (double)g.M * g.N * (g.beta != 0.0 ? 2.0 : 1.0));
}

// Algorithmic flops of one GEMM call: 2 x the multiply-adds on the structurally nonzero
// operand entries (the triangular zeros the flags declare, entry by entry rather than by tile)
// of the output entries computed (the lower triangle with kLowerOut).  For output row i the
// K range is [a, b) with a = i (kKFromRow) and b = i + 1 (kKToRow); column j narrows it to
// [max(a, j), .) (kKFromCol) or (., min(b, j + 1)) (kKToCol).  Summed in closed form per row.
static double gemm_alg_flops(const GemmArgs& g) {
  const bool fc = (g.flags & kKFromCol) != 0, tc = (g.flags & kKToCol) != 0;
  double f = 0.0;
  for (int i = 0; i < g.M; ++i) {
    const double a = (g.flags & kKFromRow) ? i : 0;
    const double b = (g.flags & kKToRow) ? std::min(g.K, i + 1) : g.K;
    const double J = (g.flags & kLowerOut) ? std::min(g.N, i + 1) : g.N;
    if (b <= a) continue;
    double s = 0.0;
    if (!fc && !tc) {
      s = J * (b - a);
    } else if (fc && !tc) {  // sum_j (b - max(a, j))+
      s = std::min(J, a) * (b - a);
      const double j1 = std::min(J, b);
      if (j1 > a) s += (j1 - a) * b - (a + j1 - 1.0) * (j1 - a) / 2.0;
    } else if (!fc && tc) {  // sum_j (min(b, j + 1) - a)+
      const double j1 = std::min(J, b);
      if (j1 > a) s += (j1 - a) * (j1 - a + 1.0) / 2.0;
      if (J > b) s += (J - b) * (b - a);
    } else {  // both: one term for each j in [a, b)
      s = std::max(0.0, std::min(J, b) - a);
    }
    f += s;
  }
  return 2.0 * f;
}

template <int WM, int WN, int KS, int FM = 2, int FN = 2>
static void launch_gemm(const GemmArgs& g, hipStream_t s) {
  constexpr int te_m = 16 * FM * WM, te_n = 16 * FN * WN;
  const int tm = (g.M + te_m - 1) / te_m, tn = (g.N + te_n - 1) / te_n;
  // a lower-triangular output of a square tile grid launches only its lower tiles
  const int tiles = ((g.flags & kLowerOut) && tm == tn) ? tm * (tm + 1) / 2 : tm * tn;
  const dim3 grid(tiles, g.offs ? g.batch : 1), block(64 * WM * WN * KS);
  if (!g.transA && !g.transB)
    k_gemm<false, false, WM, WN, KS, FM, FN><<<grid, block, 0, s>>>(g);
  else if (!g.transA && g.transB)
    k_gemm<false, true, WM, WN, KS, FM, FN><<<grid, block, 0, s>>>(g);
  else if (g.transA && !g.transB)
    k_gemm<true, false, WM, WN, KS, FM, FN><<<grid, block, 0, s>>>(g);
  else
    k_gemm<true, true, WM, WN, KS, FM, FN><<<grid, block, 0, s>>>(g);
}

int gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return LRSDP_OK;
  // 32 x 32 tiles with four wavefronts splitting K for small products, 64 x 64 tiles with
  // two for medium ones, 128 x 128 tiles of eight wavefronts (each a 64 x 32 block) once there
  // are thousands of them: they re-read half as much of A and B (thresholds from sweeps of
  // the factorization's shapes and the large configuration's solve)
  // (a triangular operand's K ranges follow the tile edges, so large tiles skip less of it and
  // need more tiles before they pay)
  const int64_t t64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * (g.offs ? g.batch : 1);
  const bool tri = (g.flags & (kKFromRow | kKToRow | kKFromCol | kKToCol)) != 0;
  const bool big = t64 >= 8192 || (!tri && t64 >= 1024);
  const int te = big ? 128 : t64 >= 320 ? 64 : 32;
  ProfMark pm = prof_begin((g.flags & kInverseOnly) ? LRSDP_K_GEMMINV : LRSDP_K_GEMM, s);
  // (big triangular products and lower-triangle outputs with K >= 256: 16 wavefronts of 32 x 32 blocks,
  // 50-52 against 49-51 TFLOP/s for eight 64 x 32 blocks at n = 10 000, and 40.0 against 37.9
  // for the lower-triangle product at 2500 rows; full products keep the eight: 57 against 51.
  // The batched transposed-A products of the bold S formation at n = 1000 take their 64 x 64
  // tiles without the K split: 33.7 against 31.4 TFLOP/s.)
  const bool syrk = (g.flags & kLowerOut) && g.K >= 256;  // (not the thin deflation update)
  if (big && (tri || syrk)) launch_gemm<4, 4, 1, 2, 2>(g, s);
  else if (big) launch_gemm<2, 4, 1, 4, 2>(g, s);
  else if (t64 >= 320 && g.offs && g.transA) launch_gemm<2, 2, 1>(g, s);
  else if (t64 >= 320) launch_gemm<2, 2, 2>(g, s);
  else launch_gemm<1, 1, 4>(g, s);
  LRSDP_HIP(hipGetLastError());
  if (pm.kid >= 0) {  // compulsory bytes, algorithmic flops
    double fl = 0.0, by = 0.0;
    gemm_cost(g, te, &fl, &by);
    const double nb = g.offs ? g.batch : 1;
    prof_end(pm, s, by * nb, gemm_alg_flops(g) * nb);
  }
  return LRSDP_OK;
}

// Scratch: a node keeps its L21 in tmp[0, N1 N2) while its trailing factorization runs on
// tmp beyond it (the side-stream product may still be reading L21 then).
// nodes up to this size are factored right-looking (no scratch)
constexpr int kRLMax = 1280;

size_t potrf_inv_tmp_doubles(int N) {
  if (N <= kRLMax) return 0;
  const int N1 = split64(N), N2 = N - N1;
  return (size_t)N1 * N2 + std::max(potrf_inv_tmp_doubles(N1), potrf_inv_tmp_doubles(N2));
}

// nodes at least this large move P to the side stream (below it the events cost more than
// the overlap gains)
constexpr int kSideMin = 512;

// Right-looking factorization of a node of N <= kRLMax rows (L into A's lower triangle,
// L^{-1} into Li's), 64-block columns in order.  (Splitting off the trailing tiles that the
// next column waits for, onto a second stream, measured slower: the cross-stream waits
// cost more than the overlap gains at this size.)
// Profiled flops of the right-looking steps are the Cholesky's own (the method's): at block
// column j with r block rows below it, the panel solve L_ij = A_ij L_jj^{-T} (NB^3 per block)
// and the trailing update of the r (r + 1) / 2 lower blocks (2 NB^3 each, NB^3 on the
// diagonal), r^2 NB^3 + r NB^3 in all, plus the next diagonal block's Cholesky NB^3 / 3;
// summed over the node this is N^3 / 3.  The L^{-1} products and the recomputed panel blocks
// the steps also execute are not counted.
static int rl_factor(double* A, int N, int lda, double* Li, int ldi, int* flag, hipStream_t s) {
  const int nb = (N + NB - 1) / NB;
  const double nb3 = (double)NB * NB * NB;
  const double tile_bytes = 4.0 * NB * NB * 8;
  const double leaf_flops = nb3 / 3.0, leaf_bytes = 3.0 * 8 * NB * NB;
  {  // the first block column's leaf; every later one runs inside the previous step
    const int n0 = std::min(NB, N);
    ProfMark pm = prof_begin(LRSDP_K_LEAF, s);
    k_chol_leaf<<<1, NB * LW, 0, s>>>(A, n0, lda, flag, Li, ldi, n0);
    LRSDP_HIP(hipGetLastError());
    // Cholesky n0^3 / 3 flops; A read, L and L^{-1} written
    prof_end(pm, s, 3.0 * 8 * n0 * n0, (double)n0 * n0 * n0 / 3.0);
  }
  for (int j = 0; j + 1 < nb; ++j) {
    const int r = nb - 1 - j;
    const int ta = r * (r + 1) / 2, ty = r * (j + 1), tp = j >= 1 ? r + j : 0;
    // block products: A tiles 3 (2 on the diagonal), Y tiles 3 (2 for k = j), panel stores 1
    const double products = 3.0 * (ta - 1) - (r - 1) + 2.0 + 3.0 * ty - r + tp;
    ProfMark pm = prof_begin(LRSDP_K_TILE, s);
    k_rl_fused<<<ta + ty + tp, 512, 0, s>>>(A, lda, Li, ldi, N, j, flag);
    LRSDP_HIP(hipGetLastError());
    prof_end(pm, s, products * tile_bytes + leaf_bytes,
             ((double)r * r + r) * nb3 + leaf_flops);
  }
  for (int j = std::max(0, nb - 2); j < nb; ++j) {  // the last two panels
    const int tiles = (nb - 1 - j) + j;
    if (tiles == 0) continue;
    ProfMark pm = prof_begin(LRSDP_K_TILE, s);
    k_rl_panel<<<tiles, 512, 0, s>>>(A, lda, Li, ldi, N, j);
    LRSDP_HIP(hipGetLastError());
    // the panel stores of the last two block columns: no Cholesky flops left
    prof_end(pm, s, tiles * tile_bytes, 0.0);
  }
  return LRSDP_OK;
}

static int potrf_inv_rec(double* A, int N, int lda, double* Li, int ldi, int* flag,
                         double* tmp, bool want_L, hipStream_t s, const SideStream* side,
                         int depth) {
  if (N <= 0) return LRSDP_OK;
  if (N <= kRLMax) return rl_factor(A, N, lda, Li, ldi, flag, s);
  const int N1 = split64(N), N2 = N - N1;
  double* A21 = A + (size_t)N1 * lda;
  double* A22 = A21 + N1;
  double* Li21 = Li + (size_t)N1 * ldi;
  double* Li22 = Li21 + N1;
  double* sub = tmp + (size_t)N1 * N2;  // the children's scratch
  LRSDP_TRY(potrf_inv_rec(A, N1, lda, Li, ldi, flag, tmp, want_L, s, side, depth + 1));
  {  // tmp = L21 = A21 L11^{-T}
    GemmArgs g;
    g.M = N2; g.N = N1; g.K = N1;
    g.A = A21; g.lda = lda;
    g.B = Li; g.ldb = ldi; g.transB = true;  // op(B)[k][j] = L11^{-1}[j][k], zero for k > j
    g.C = tmp; g.ldc = N1;
    g.flags = kKToCol;
    LRSDP_TRY(gemm(g, s));
  }
  // L21 lives in A21 when the caller wants L (then P = L21 L11^{-1} waits in tmp, after the
  // trailing factorization); otherwise L21 stays in tmp and P overwrites A21 at once, on
  // the side stream when there is one.
  const double* L21 = tmp;
  int ld21 = N1;
  if (want_L) {
    const size_t cnt = (size_t)N2 * N1;
    k_copy_block<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(tmp, N1, A21, lda, N2, N1);
    LRSDP_HIP(hipGetLastError());
    L21 = A21;
    ld21 = lda;
  }
  GemmArgs pg;  // P = L21 L11^{-1}
  pg.M = N2; pg.N = N1; pg.K = N1;
  pg.A = L21; pg.lda = ld21;
  pg.B = Li; pg.ldb = ldi;  // L11^{-1}[k][j], zero for k < j
  pg.flags = kKFromCol | kInverseOnly;
  const bool use_side = !want_L && side && side->stream && N >= kSideMin && depth < side->depths;
  hipEvent_t ev_in = use_side ? side->ev[2 * depth] : nullptr;
  hipEvent_t ev_out = use_side ? side->ev[2 * depth + 1] : nullptr;
  if (!want_L) {
    pg.C = A21; pg.ldc = lda;
    if (use_side) {
      LRSDP_HIP(hipEventRecord(ev_in, s));
      LRSDP_HIP(hipStreamWaitEvent(side->stream, ev_in, 0));
      LRSDP_TRY(gemm(pg, side->stream));
      LRSDP_HIP(hipEventRecord(ev_out, side->stream));
    } else {
      LRSDP_TRY(gemm(pg, s));
    }
  }
  {  // A22 -= L21 L21^T (lower)
    GemmArgs g;
    g.M = N2; g.N = N2; g.K = N1;
    g.A = L21; g.lda = ld21;
    g.B = L21; g.ldb = ld21; g.transB = true;
    g.C = A22; g.ldc = lda;
    g.alpha = -1.0; g.beta = 1.0; g.flags = kLowerOut;
    LRSDP_TRY(gemm(g, s));
  }
  LRSDP_TRY(potrf_inv_rec(A22, N2, lda, Li22, ldi, flag, sub, want_L, s, side, depth + 1));
  if (want_L) {
    pg.C = tmp; pg.ldc = N1;
    LRSDP_TRY(gemm(pg, s));
  }
  if (use_side) LRSDP_HIP(hipStreamWaitEvent(s, ev_out, 0));
  {  // (L^{-1})_21 = -L22^{-1} P
    GemmArgs g;
    g.M = N2; g.N = N1; g.K = N2;
    g.A = Li22; g.lda = ldi;  // zero for k > i
    g.B = want_L ? tmp : A21; g.ldb = want_L ? N1 : lda;
    g.C = Li21; g.ldc = ldi;
    g.alpha = -1.0; g.flags = kKToRow | kInverseOnly;
    LRSDP_TRY(gemm(g, s));
  }
  return LRSDP_OK;
}

int potrf_inv(double* A, int N, int lda, double* Li, int ldi, int* flag, double* tmp,
              bool want_L, hipStream_t s, const SideStream* side) {
  return potrf_inv_rec(A, N, lda, Li, ldi, flag, tmp, want_L, s, side, 0);
}

// From this size on a node is kept block-explicit: its (2, 1) block keeps L21 and the two
// products that would turn it into (L^{-1})_21 = -L22^{-1} L21 L11^{-1} are skipped, the largest
// of the inverse work (n k = 5000: the factor of bold S 3.96 -> 3.33 ms).  Both of its blocks are
// again such nodes while they are this large: the node's own L21 = A21 L11^{-T} is then solved
// over the leading block's tree (trsm_tree), with the flops of one triangular solve.  The
// diagonal is the leaves of the tree, each holding its explicit inverse, and every entry below
// the leaves' blocks is L's (n k = 40 000: 16 leaves of 2496-2528 rows).  Applying L^{-1} then
// takes 2 b - 1 dependent GEMVs per triangle for b leaves over the same bytes (PCG +0.3 ms per
// solve at n k = 5000, where b = 2).
// (Keeping -L21 L11^{-1} instead, formed on the side stream while the trailing block factors,
// needs four: at n k = 5000 it cost 0.4 ms more setup than it saved in the PCG, and at
// n k = 40000 the product competed with the trailing factorization: 528 -> 661 ms.)
constexpr int kBlockInvMin = 4096;
constexpr int kBinvMaxDepth = 5;  // at most 2^5 = kBinvMaxBlocks leaves
static_assert((1 << kBinvMaxDepth) <= kBinvMaxBlocks, "leaf count");

static bool binv_leaf(int N, int depth) { return N < kBlockInvMin || depth >= kBinvMaxDepth; }

static void binv_leaves(int o, int N, int depth, int* offs, int* nb) {
  if (binv_leaf(N, depth)) {
    offs[(*nb)++] = o;
    return;
  }
  const int N1 = split64(N);
  binv_leaves(o, N1, depth + 1, offs, nb);
  binv_leaves(o + N1, N - N1, depth + 1, offs, nb);
}

int binv_blocks(int N, int* offs) {
  int nb = 0;
  binv_leaves(0, N, 0, offs, &nb);
  offs[nb] = N;
  return nb;
}

// Lo = Ai L^{-T} for the node of order n at Li's diagonal position D (block-explicit below it as
// potrf_binv leaves it): Ai (rows x n, in A's storage, pitch lda) is overwritten on the way;
// Lo (rows x n, pitch ldi) receives the result.  Left to right over the node's two blocks:
// Lo_1 = Ai_1 L11^{-T}; Ai_2 -= Lo_1 L21^T; Lo_2 = Ai_2 L22^{-T}.
static int trsm_tree(double* Ai, int lda, double* Lo, int ldi, const double* D, int rows, int n,
                     int depth, hipStream_t s) {
  if (binv_leaf(n, depth)) {
    GemmArgs g;
    g.M = rows; g.N = n; g.K = n;
    g.A = Ai; g.lda = lda;
    g.B = D; g.ldb = ldi; g.transB = true;  // op(B)[k][j] = L^{-1}[j][k], zero for k > j
    g.C = Lo; g.ldc = ldi;
    g.flags = kKToCol;
    return gemm(g, s);
  }
  const int n1 = split64(n), n2 = n - n1;
  LRSDP_TRY(trsm_tree(Ai, lda, Lo, ldi, D, rows, n1, depth + 1, s));
  {  // Ai_2 -= Lo_1 L21^T
    GemmArgs g;
    g.M = rows; g.N = n2; g.K = n1;
    g.A = Lo; g.lda = ldi;
    g.B = D + (size_t)n1 * ldi; g.ldb = ldi; g.transB = true;
    g.C = Ai + n1; g.ldc = lda;
    g.alpha = -1.0; g.beta = 1.0;
    LRSDP_TRY(gemm(g, s));
  }
  return trsm_tree(Ai + n1, lda, Lo + n1, ldi, D + (size_t)n1 * ldi + n1, rows, n2, depth + 1, s);
}

// One node of the tree (depth: its own; its children's in the side stream's events is one more).
static int binv_rec(double* A, int N, int lda, double* Li, int ldi, int* flag, double* tmp,
                    hipStream_t s, const SideStream* side, int depth) {
  if (binv_leaf(N, depth))
    return potrf_inv_rec(A, N, lda, Li, ldi, flag, tmp, false, s, side, depth);
  const int N1 = split64(N), N2 = N - N1;
  double* A21 = A + (size_t)N1 * lda;
  double* A22 = A21 + N1;
  double* L21 = Li + (size_t)N1 * ldi;  // the (2, 1) block of Li keeps L21 itself
  double* Li22 = L21 + N1;
  // each child joins its own side-stream product before it returns, so tmp is free again
  LRSDP_TRY(binv_rec(A, N1, lda, Li, ldi, flag, tmp, s, side, depth + 1));
  // L21 = A21 L11^{-T}
  LRSDP_TRY(trsm_tree(A21, lda, L21, ldi, Li, N2, N1, depth + 1, s));
  {  // A22 -= L21 L21^T (lower)
    GemmArgs g;
    g.M = N2; g.N = N2; g.K = N1;
    g.A = L21; g.lda = ldi;
    g.B = L21; g.ldb = ldi; g.transB = true;
    g.C = A22; g.ldc = lda;
    g.alpha = -1.0; g.beta = 1.0; g.flags = kLowerOut;
    LRSDP_TRY(gemm(g, s));
  }
  return binv_rec(A22, N2, lda, Li22, ldi, flag, tmp, s, side, depth + 1);
}

int potrf_binv(double* A, int N, int lda, double* Li, int ldi, int* flag, double* tmp,
               hipStream_t s, const SideStream* side, int* split) {
  *split = 0;
  LRSDP_TRY(binv_rec(A, N, lda, Li, ldi, flag, tmp, s, side, 0));
  if (!binv_leaf(N, 0)) *split = split64(N);
  return LRSDP_OK;
}

int binv_apply(const double* M, int N, int split, int ld, const double* x, const double* xsub,
               double* tmp, double* y, bool accumulate, hipStream_t s) {
  if (split <= 0) return trmv_pair_ex(M, N, ld, x, xsub, tmp, y, accumulate, s);
  int offs[kBinvMaxBlocks + 1];
  const int nb = binv_blocks(N, offs);
  if (nb < 2 || split != split64(N)) return LRSDP_ERR_INVALID_ARG;
  ProfMark pm = prof_begin(LRSDP_K_GEMV, s);
  double* F = tmp;          // f = L^{-1} (x - xsub)
  double* R = tmp + N;      // a block's right-hand side after the other blocks' terms
  double* Yr = tmp + 2 * N; // L^{-T} f, block by block (y may be accumulating)
  const int acc = accumulate ? 1 : 0;
  // forward, left-looking: block b (rows [a, e)): r = (x - xsub)_b - L_{b, <a} f_{<a};
  // f_b = L_bb^{-1} r
  for (int b = 0; b < nb; ++b) {
    const int a = offs[b], e = offs[b + 1], h = e - a, g = (h + 3) / 4;
    const double* Mb = M + (size_t)a * ld;
    if (b == 0) {
      const double* xb = x;
      if (xsub) {  // x - xsub into R's first block (not used otherwise)
        k_sub_vec<<<(h + 255) / 256, 256, 0, s>>>(h, x, xsub, R);
        xb = R;
      }
      k_gemv_tri<false><<<g, 256, 0, s>>>(M, h, h, ld, xb, F, 0, nullptr, 0);
      continue;
    }
    if (xsub)
      k_gemv_rect<true><<<g, 256, 0, s>>>(Mb, h, a, ld, F, x + a, xsub + a, R + a);
    else
      k_gemv_rect<false><<<g, 256, 0, s>>>(Mb, h, a, ld, F, x + a, nullptr, R + a);
    k_gemv_tri<false><<<g, 256, 0, s>>>(Mb + a, h, h, ld, R + a, F + a, 0, nullptr, 0);
  }
  // backward, left-looking over the mirrored upper part (which holds L_bb^{-T} and the
  // L21^T of every node): r = f_b - L_{>e, b}^T y_{>e}; y_b = L_bb^{-T} r
  for (int b = nb - 1; b >= 0; --b) {
    const int a = offs[b], e = offs[b + 1], h = e - a, g = (h + 3) / 4;
    const double* Mb = M + (size_t)a * ld;
    const double* rhs = F + a;
    if (e < N) {
      k_gemv_rect<false><<<g, 256, 0, s>>>(Mb + e, h, N - e, ld, Yr + e, F + a, nullptr, R + a);
      rhs = R + a;
    }
    k_gemv_tri<false><<<g, 256, 0, s>>>(Mb + a, h, h, ld, rhs, Yr + a, 1, y + a, acc);
  }
  LRSDP_HIP(hipGetLastError());
  prof_end(pm, s, 8.0 * (double)N * (N + 1) + 32.0 * nb * N, 2.0 * (double)N * (N + 1));
  return LRSDP_OK;
}

// (L^{-1})_21 = -L22^{-1} L21 L11^{-1} for the node of order N at Li (both blocks already hold
// explicit inverses); tmp: (N - N1) N1 doubles
static int binv_node_inverse(double* Li, int N, int ld, double* tmp, int depth, hipStream_t s) {
  if (binv_leaf(N, depth)) return LRSDP_OK;
  const int N1 = split64(N), N2 = N - N1;
  double* L21 = Li + (size_t)N1 * ld;
  LRSDP_TRY(binv_node_inverse(Li, N1, ld, tmp, depth + 1, s));
  LRSDP_TRY(binv_node_inverse(L21 + N1, N2, ld, tmp, depth + 1, s));
  {  // tmp = L21 L11^{-1}
    GemmArgs g;
    g.M = N2; g.N = N1; g.K = N1;
    g.A = L21; g.lda = ld;
    g.B = Li; g.ldb = ld;  // L11^{-1}[k][j], zero for k < j
    g.C = tmp; g.ldc = N1;
    g.flags = kKFromCol | kInverseOnly;
    LRSDP_TRY(gemm(g, s));
  }
  {  // (L^{-1})_21 = -L22^{-1} tmp
    GemmArgs g;
    g.M = N2; g.N = N1; g.K = N2;
    g.A = L21 + N1; g.lda = ld;  // L22^{-1}, zero for k > i
    g.B = tmp; g.ldb = N1;
    g.C = L21; g.ldc = ld;
    g.alpha = -1.0; g.flags = kKToRow | kInverseOnly;
    LRSDP_TRY(gemm(g, s));
  }
  return LRSDP_OK;
}

int binv_full_inverse(double* Li, int N, int split, int ld, double* tmp, hipStream_t s) {
  if (split <= 0) return LRSDP_OK;
  if (split != split64(N)) return LRSDP_ERR_INVALID_ARG;
  return binv_node_inverse(Li, N, ld, tmp, 0, s);
}

int trmv_pair_ex(const double* M, int N, int ld, const double* x, const double* xsub,
                 double* tmp, double* y, bool accumulate, hipStream_t s) {
  ProfMark pm = prof_begin(LRSDP_K_GEMV, s);
  const int grid = (N + 3) / 4;
  const double* xv = x;
  if (xsub) {  // x - xsub into tmp's second half
    k_sub_vec<<<(N + 255) / 256, 256, 0, s>>>(N, x, xsub, tmp + N);
    xv = tmp + N;
  }
  k_gemv_tri<false><<<grid, 256, 0, s>>>(M, N, N, ld, xv, tmp, 0, nullptr, 0);
  if (accumulate)
    k_gemv_tri<true><<<grid, 256, 0, s>>>(M, N, N, ld, tmp, y, 1, nullptr, 0);
  else
    k_gemv_tri<false><<<grid, 256, 0, s>>>(M, N, N, ld, tmp, y, 1, nullptr, 0);
  LRSDP_HIP(hipGetLastError());
  prof_end(pm, s, 8.0 * (double)N * (N + 1) + 32.0 * N, 2.0 * (double)N * (N + 1));
  return LRSDP_OK;
}

int bl_gemv_pair(const BLaunch& L, int xrole, int xsub_role, int tmp_role, int yrole,
                 bool accumulate, hipStream_t s) {
  if (L.b.count <= 0 || L.tot[kKgemv] <= 0) return LRSDP_OK;
  const int grid = L.tot[kKgemv];
  int xr = xrole;
  if (xsub_role >= 0) {  // x - xsub into the h2 work vector first, as trmv_pair_ex does
    k_sub_vec_b<<<L.tot[kKnk256], 256, 0, s>>>(L.b, xrole, xsub_role, kVwh2);
    xr = kVwh2;
  }
  k_gemv_tri_b<false><<<grid, 256, 0, s>>>(L.b, xr, tmp_role, 0);
  if (accumulate)
    k_gemv_tri_b<true><<<grid, 256, 0, s>>>(L.b, tmp_role, yrole, 1);
  else
    k_gemv_tri_b<false><<<grid, 256, 0, s>>>(L.b, tmp_role, yrole, 1);
  LRSDP_HIP(hipGetLastError());
  return LRSDP_OK;
}

int trmv_pair(const double* M, int N, int ld, const double* x, double* tmp, double* y,
              hipStream_t s) {
  return trmv_pair_ex(M, N, ld, x, nullptr, tmp, y, false, s);
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
