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

}  // namespace lrsdp
