// Partial symmetric eigensolver for Algorithm 1 step 1a (internal).
#pragma once

#include "internal.h"

namespace lrsdp {

// Bytes of device workspace eig_top_and_min needs for order n and rank k.
size_t eig_workspace_bytes(int n, int k);

// lam_out (device, k + 1): lambda_min(W), then the k largest eigenvalues ascending.
// Vl_out (device, k x n row-major = n x k column-major): their eigenvectors.
int eig_top_and_min(const double* W, int n, int k, void* workspace, double* lam_out,
                    double* Vl_out, hipStream_t s);

// GEMM-based alternative (spectral.hip): the k largest eigenpairs by subspace iteration
// with Rayleigh-Ritz and tau = (tr W - sum of them) / (n - k).  lam_out as above with tau in
// lam_out[0]; tr_out (device, 2, may be null) receives tr W as a double-double pair.
// Returns LRSDP_ERR_EIG when the iteration does not converge within max_sweeps.
size_t spectral_workspace_bytes(int n, int k);
int spectral_top(const double* W, int n, int k, void* ws, double* lam_out, double* Vl_out,
                 double* tr_out, int max_sweeps, double* host_res, int* sweeps_out,
                 hipStream_t s);
// tr W as a double-double pair (device, 2 doubles).
int trace_dd(const double* W, int n, double* out, hipStream_t s);

}  // namespace lrsdp
