// Dense FP64 kernels on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64), used by the
// setup steps: Cholesky of 2 W0 + U U^T (size n) and of bold S (size nk) with their inverse
// factors, the explicit bold S^{-1} = L^{-T} L^{-1}, and the GEMMs that form bold S.
#pragma once

#include "internal.h"

namespace lrsdp {

// Triangular-structure hints: K-range trimming per output tile, so a product with a
// triangular operand skips its zero tiles; inside the tiles it does compute, the entries a
// flag declares zero are never read (they are staged as zeros), so the other triangle of a
// triangular operand may hold anything.
enum GemmFlags : unsigned {
  kKFromRow = 1u,   // op(A)[i][k] == 0 for k < i   -> k starts at the tile's first row
  kKToRow = 2u,     // op(A)[i][k] == 0 for k > i   -> k ends after the tile's last row
  kKFromCol = 4u,   // op(B)[k][j] == 0 for k < j
  kKToCol = 8u,     // op(B)[k][j] == 0 for k > j
  kLowerOut = 16u,  // compute / write only C[i][j] with j <= i
  kInverseOnly = 32u,  // accounting only: a product of the explicit inverse factor L^{-1},
                       // not of the factorization itself (timed as its own kernel class)
};

struct GemmArgs {
  int M = 0, N = 0, K = 0;
  const double* A = nullptr;
  int lda = 0;
  bool transA = false;  // false: A is M x K row-major; true: A is K x M
  const double* B = nullptr;
  int ldb = 0;
  bool transB = false;  // false: B is K x N; true: B is N x K
  double* C = nullptr;
  int ldc = 0;
  double alpha = 1.0, beta = 0.0;
  const double* alpha_dev = nullptr;  // device scalar that replaces alpha when given
  unsigned flags = 0;
  int batch = 1;                  // with offs: number of products (grid.y)
  const int64_t* offs = nullptr;  // device, 3 x batch element offsets of A, B, C
};

// C = alpha op(A) op(B) + beta C (row-major), FP64 MFMA.
int gemm(const GemmArgs& g, hipStream_t s);

// Cholesky A = L L^T and L^{-1} in one pass.  Li (N x N, distinct from A) receives L^{-1}
// in its lower triangle with zeros above the diagonal inside each 64-aligned diagonal block
// (the rest of the upper triangle is left as is).  With want_L, A's lower triangle receives
// L under the same zero convention; without it, A is used as scratch and left undefined.
// tmp: potrf_inv_tmp_doubles(N) doubles.  On a non-positive pivot *flag (device int) gets 1
// and the result is garbage.
// A second stream on which the factorization runs the one product per recursion node that
// the rest of the node does not wait for (P = L21 L11^{-1}, needed only at the node's end),
// with events to join it back; ev holds two events per recursion depth.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t* ev = nullptr;
  int depths = 0;
};
// The context's side stream and events (created on first use).
int ctx_side(lrsdp_ctx* ctx, SideStream* out);
size_t potrf_inv_tmp_doubles(int N);
int potrf_inv(double* A, int N, int lda, double* Li, int ldi, int* flag, double* tmp,
              bool want_L, hipStream_t s, const SideStream* side = nullptr);
// Cholesky A = L L^T with a block-explicit inverse.  Below a size (4096) the result is that of
// potrf_inv (Li holds L^{-1}, *split = 0).  From it on a node keeps L21 itself in Li's (2, 1)
// block, and each of its diagonal blocks is again such a node while it is that large, else its
// explicit inverse (*split = N1 of the top node).  The diagonal is then the leaves of a binary
// tree (binv_blocks), each holding its explicit inverse, and every entry below the leaves' blocks
// is L's: the products that would turn the L21 into (L^{-1})_21 are the largest of the
// factorization, and the block form applies L^{-1} with the same bytes.  A is used as scratch.
int potrf_binv(double* A, int N, int lda, double* Li, int ldi, int* flag, double* tmp,
               hipStream_t s, const SideStream* side, int* split);
// The diagonal blocks (the tree's leaves) of a block-explicit factor of order N: offs[0] = 0 <
// offs[1] < ... < offs[nb] = N (offs: room for kBinvMaxBlocks + 1); returns nb (1: not
// block-explicit).
constexpr int kBinvMaxBlocks = 32;
int binv_blocks(int N, int* offs);
// y (+)= L^{-T} L^{-1} (x - xsub) for a factor of potrf_binv whose lower triangle was mirrored
// into the upper one (so the upper part holds the leaves' L_bb^{-T} and L^T elsewhere); xsub
// may be nullptr.  Row-wise GEMVs over the same bytes as trmv_pair_ex, left-looking block by block.
// tmp: 3 N doubles.
int binv_apply(const double* M, int N, int split, int ld, const double* x, const double* xsub,
               double* tmp, double* y, bool accumulate, hipStream_t s);
// Turns every L21 of a potrf_binv factor into (L^{-1})_21 = -L22^{-1} L21 L11^{-1}, children
// before their node (the lower triangle then holds L^{-1}); tmp: (N - split) split doubles.
int binv_full_inverse(double* Li, int N, int split, int ld, double* tmp, hipStream_t s);
// y = M_up (M_lo x) with M_lo the lower and M_up the upper triangle of M, both including the
// diagonal (two row-wise triangular GEMVs; tmp: N doubles).  With L^{-1} in the lower
// triangle and its transpose mirrored into the upper one this is y = L^{-T} L^{-1} x.
int trmv_pair(const double* M, int N, int ld, const double* x, double* tmp, double* y,
              hipStream_t s);
// y (+)= L^{-T} (L^{-1} (x - xsub)) with the same two passes; xsub may be nullptr, and with
// accumulate the result is added to y.  tmp: N doubles (2 N with xsub).
int trmv_pair_ex(const double* M, int N, int ld, const double* x, const double* xsub,
                 double* tmp, double* y, bool accumulate, hipStream_t s);
// X := M^T M (lower part), M lower triangular N x N; X and M distinct.
int lauum(const double* M, int N, int ldm, double* X, int ldx, hipStream_t s);
// Copy the lower triangle into the upper one.
int mirror_lower(double* A, int N, int lda, hipStream_t s);
// Zero the strict upper triangle.
int zero_upper(double* A, int N, int lda, hipStream_t s);
// Out-of-place transpose (N x N).
int transpose(const double* A, int N, int lda, double* B, int ldb, hipStream_t s);

// y = A x, A N x N row-major (dense GEMV, one wavefront per row).
int gemv(const double* A, int N, int lda, const double* x, double* y, hipStream_t s);

}  // namespace lrsdp
