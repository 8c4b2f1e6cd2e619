// Small dense FP64 kernels for the host-side factorisation (row-major).
#pragma once
#include <cstdint>

namespace bido {
namespace dense {

// In-place lower Cholesky of the leading n x n block of A (leading dim lda).
// Returns the index of the first non-positive pivot, or -1 on success.
int64_t potrf_lower(int64_t n, double* A, int64_t lda, bool par);

// Linv = L^-1 for a lower-triangular L (n x n, lda); Linv row-major n x n,
// zero above the diagonal.
void trtri_lower(int64_t n, const double* L, int64_t lda, double* Linv, bool par);

// X <- X L^-T for X (m x n, ldx) and lower-triangular L (n x n, ldl).
void trsm_right_lower_t(int64_t m, int64_t n, const double* L, int64_t ldl,
                        double* X, int64_t ldx, bool par);

// C <- C - A B^T with A (m x k), B (n x k), C (m x n); lower_only restricts
// the update to j <= i (C symmetric, m == n).
void gemm_nt_sub(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc,
                 bool lower_only, bool par);

}  // namespace dense
}  // namespace bido
